"""Thin ctypes binding of librpba (include/rpba.h) on torch device tensors.

PyTorch supplies device memory and the stream; every step of the method runs
in the library's HIP kernels.  The functions keep the C names:
``rpba_intersect``, ``rpba_subblock_lm_step``, ``rpba_consensus``,
``rpba_robust_reweight``.  There is no fallback: without the built library or
a GPU, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librpba.so")

RPBA_FP64, RPBA_MIXED = 0, 1
RPBA_SOLVER_CHOL, RPBA_SOLVER_PCG_BJ, RPBA_SOLVER_PCG_LEARNED, RPBA_SOLVER_AUTO, RPBA_SOLVER_AUTO_LEARNED = 0, 1, 2, 3, 4
RPBA_CHOL_DEFAULT, RPBA_CHOL_STEPWISE, RPBA_CHOL_DATAFLOW = 0, 1, 2
(RPBA_VARIANT_EXTENDED, RPBA_VARIANT_ALL_CAMERAS, RPBA_VARIANT_SCALAR, RPBA_VARIANT_PLAIN,
 RPBA_VARIANT_PLAIN_REFINED) = 0, 1, 2, 3, 4
RPBA_OK, RPBA_ERR_NOT_SPD, RPBA_WARN_NONCONVERGED = 0, 4, 100
RPBA_ROBUST_WEIGHT, RPBA_ROBUST_ELIMINATE_POINTS, RPBA_ROBUST_DELETE_OBS = 0, 1, 2
RPBA_DAMPING_FIXED, RPBA_DAMPING_ADAPTIVE = 0, 1
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_HIP", 3: "ERR_WORKSPACE", 4: "ERR_NOT_SPD", 5: "ERR_STATE",
                100: "WARN_NONCONVERGED"}

# every symbol include/rpba.h and include/rpba_testing.h declare
EXPORTS = [
    "rpba_default_options", "rpba_workspace_size", "rpba_create", "rpba_intersect", "rpba_robust_reweight",
    "rpba_subblock_lm_step", "rpba_consensus", "rpba_destroy", "rpba_last_error", "rpba_num_copies",
    "rpba_get_copies", "rpba_get_block_rcs", "rpba_block_cameras", "rpba_selftest_gemm",
    "rpba_set_graph", "rpba_set_timing", "rpba_get_timing", "rpba_get_block_solution", "rpba_block_solver",
    "rpba_precond_num_params", "rpba_set_precond_weights", "rpba_precond_num_samples", "rpba_precond_sample_stride",
    "rpba_precond_harvest", "rpba_precond_train_scratch", "rpba_precond_train_step", "rpba_get_robust",
    "rpba_step_status", "rpba_ratio_update", "rpba_camera_order", "rpba_get_precond_blocks", "rpba_factor_flops",
    "rpba_precond_train_step_noalloc", "rpba_partition_default_options", "rpba_partition", "rpba_covariance",
    "rpba_get_damping",
]
TRAIN_NOALLOC_MAX_SAMPLES = 8192   # RPBA_TRAIN_NOALLOC_MAX_SAMPLES
PHASES = ["intersect", "point_blocks", "schur_rows", "chol_forward", "chol_backward", "update", "consensus",
          "robust", "iterative_solve", "schur_pairs", "intersect_export"]


class RpbaError(RuntimeError):
    pass


class ProblemDesc(ctypes.Structure):
    _fields_ = [
        ("M", ctypes.c_int32), ("N", ctypes.c_int32), ("K", ctypes.c_int32), ("L", ctypes.c_int32),
        ("f", ctypes.c_double), ("cx", ctypes.c_double), ("cy", ctypes.c_double), ("sigma_px", ctypes.c_double),
        ("cam_R", ctypes.c_void_p), ("cam_C", ctypes.c_void_p), ("pts", ctypes.c_void_p),
        ("obs_xy", ctypes.c_void_p), ("obs_info", ctypes.c_void_p),
        ("obs_cam", ctypes.c_void_p), ("obs_pt", ctypes.c_void_p), ("cam_block", ctypes.c_void_p),
        ("cam_intr", ctypes.c_void_p),
    ]


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32), ("solver", ctypes.c_int32), ("lam", ctypes.c_double),
        ("int_tol", ctypes.c_double), ("int_maxit", ctypes.c_int32), ("pcg_maxit", ctypes.c_int32),
        ("pcg_tol", ctypes.c_double), ("ir_tol", ctypes.c_double), ("ir_maxit", ctypes.c_int32),
        ("pcg_min_cams", ctypes.c_int32), ("t_v", ctypes.c_double), ("down_weight", ctypes.c_double),
        ("chol_tile", ctypes.c_int32), ("chol_schedule", ctypes.c_int32),
        ("robust", ctypes.c_int32), ("pair_lanes", ctypes.c_int32), ("variant", ctypes.c_int32),
        ("rho", ctypes.c_double), ("rho_growth", ctypes.c_double), ("filter_px", ctypes.c_double),
        ("covariance", ctypes.c_int32), ("damping", ctypes.c_int32), ("lambda_up", ctypes.c_double),
        ("lambda_down", ctypes.c_double), ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
        ("intrinsics", ctypes.c_int32),
    ]


class PartitionOptions(ctypes.Structure):
    _fields_ = [("parts", ctypes.c_int32), ("imbalance", ctypes.c_double), ("min_cams", ctypes.c_int32),
                ("refine_passes", ctypes.c_int32), ("cost_cams3", ctypes.c_double), ("cost_obs", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load librpba.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RpbaError(f"{path} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
    L.rpba_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        getattr(L, name)  # every declared symbol must resolve
    L.rpba_default_options.argtypes = [ctypes.POINTER(Options)]
    L.rpba_workspace_size.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(Options), ctypes.POINTER(ctypes.c_size_t)]
    L.rpba_create.argtypes = [ctypes.POINTER(ProblemDesc), ctypes.POINTER(Options), vp, ctypes.c_size_t, vp,
                              ctypes.POINTER(vp)]
    L.rpba_intersect.argtypes = [vp, dp, dp, dp]
    L.rpba_robust_reweight.argtypes = [vp, i32, dp]
    L.rpba_get_robust.argtypes = [vp, vp, vp]
    L.rpba_subblock_lm_step.argtypes = [vp, dp, dp]
    L.rpba_consensus.argtypes = [vp, dp]
    L.rpba_destroy.argtypes = [vp]
    L.rpba_num_copies.restype = i64
    L.rpba_num_copies.argtypes = [vp]
    L.rpba_get_copies.argtypes = [vp, vp, vp, vp, vp]
    L.rpba_get_block_rcs.argtypes = [vp, i32, vp, vp]
    L.rpba_block_cameras.restype = i32
    L.rpba_block_cameras.argtypes = [vp, i32]
    L.rpba_selftest_gemm.argtypes = [dp, dp, dp, vp]
    L.rpba_precond_num_params.restype = i32
    L.rpba_precond_num_params.argtypes = []
    L.rpba_set_precond_weights.argtypes = [vp, vp]
    L.rpba_precond_num_samples.restype = i32
    L.rpba_precond_num_samples.argtypes = [vp]
    L.rpba_precond_sample_stride.restype = i32
    L.rpba_precond_sample_stride.argtypes = [i32]
    L.rpba_precond_harvest.argtypes = [vp, vp, i32, vp]
    L.rpba_precond_train_scratch.restype = ctypes.c_size_t
    L.rpba_precond_train_scratch.argtypes = [i32]
    L.rpba_precond_train_step.argtypes = [vp, i32, i32, vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, i32, vp]
    L.rpba_get_block_solution.argtypes = [vp, i32, vp]
    L.rpba_block_solver.restype = i32
    L.rpba_block_solver.argtypes = [vp, i32]
    L.rpba_step_status.argtypes = [vp, vp, vp]
    L.rpba_ratio_update.restype = i32
    L.rpba_ratio_update.argtypes = [i32, vp, ctypes.c_double, vp, vp, vp]
    L.rpba_camera_order.argtypes = [vp, vp]
    L.rpba_get_precond_blocks.argtypes = [vp, i32, vp]
    L.rpba_factor_flops.argtypes = [vp, vp]
    L.rpba_precond_train_step_noalloc.argtypes = [vp, i32, i32, vp, vp, vp, i32, ctypes.c_float, vp, vp, i32, vp]
    L.rpba_partition_default_options.argtypes = [ctypes.POINTER(PartitionOptions)]
    L.rpba_partition.argtypes = [i32, i32, i32, vp, vp, ctypes.POINTER(PartitionOptions), vp, vp, vp]
    L.rpba_covariance.argtypes = [vp, ctypes.c_double, vp, vp]
    L.rpba_get_damping.argtypes = [vp, vp, vp]
    L.rpba_set_graph.argtypes = [vp, i32]
    L.rpba_set_timing.argtypes = [vp, i32]
    L.rpba_get_timing.restype = i32
    L.rpba_get_timing.argtypes = [vp, vp, vp, vp, i32]
    for name in EXPORTS:
        if name not in ("rpba_last_error", "rpba_num_copies", "rpba_block_cameras", "rpba_get_timing",
                        "rpba_block_solver", "rpba_precond_num_params", "rpba_precond_num_samples",
                        "rpba_precond_sample_stride", "rpba_precond_train_scratch", "rpba_ratio_update"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        msg = _lib.rpba_last_error().decode(errors="replace")
        raise RpbaError(f"{what}: {STATUS_NAMES.get(rc, rc)}: {msg}")


def default_options(**kw) -> Options:
    L = load_library()
    o = Options()
    _check(L.rpba_default_options(ctypes.byref(o)), "rpba_default_options")
    names = {f[0] for f in Options._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def precond_num_params():
    return int(load_library().rpba_precond_num_params())


def precond_train_step(samples, nz, W, m, v, t, lr, scratch, grad, loss, apply=True, stream=None):
    """One training step of the preconditioner network on `samples` (FP32
    device tensor [n][stride]); with apply=False only loss and gradient."""
    import torch
    L = load_library()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(L.rpba_precond_train_step(_ptr(samples), int(samples.shape[0]), nz, _ptr(W), _ptr(m), _ptr(v), int(t),
                                     float(lr), _ptr(scratch), _ptr(grad), _ptr(loss), int(apply),
                                     ctypes.c_void_p(st.cuda_stream)), "rpba_precond_train_step")


def precond_train_step_noalloc(samples, nz, W, m, v, t, lr, grad, loss, apply=True, stream=None):
    """The training step through rpba_precond_train_step_noalloc (the
    library's own device scratch, at most TRAIN_NOALLOC_MAX_SAMPLES samples)."""
    import torch
    L = load_library()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(L.rpba_precond_train_step_noalloc(_ptr(samples), int(samples.shape[0]), nz, _ptr(W), _ptr(m), _ptr(v),
                                             int(t), float(lr), _ptr(grad), _ptr(loss), int(apply),
                                             ctypes.c_void_p(st.cuda_stream)), "rpba_precond_train_step_noalloc")


def precond_train_scratch_bytes(nsamp):
    return int(load_library().rpba_precond_train_scratch(int(nsamp)))


def ratio_update(cost, best, grace, active, ratio=1.01):
    """Improvement test of Sec. 5.4 for len(cost) loops at once, in the
    library (rpba_ratio_update): updates best (float64), grace and active
    (uint8) in place and returns the number of loops still active."""
    L = load_library()
    cost = np.ascontiguousarray(cost, dtype=np.float64)
    for a, t in ((best, np.float64), (grace, np.uint8), (active, np.uint8)):
        assert a.dtype == t and a.flags.c_contiguous and a.shape == cost.shape
    n = L.rpba_ratio_update(int(cost.size), cost.ctypes.data, float(ratio), best.ctypes.data, grace.ctypes.data,
                            active.ctypes.data)
    if n < 0:
        raise RpbaError("rpba_ratio_update: bad arguments")
    return int(n)


def selftest_gemm(A, B):
    """C = A B^T through the library's FP64 matrix-core tile product (64x64)."""
    import torch
    L = load_library()
    C = torch.empty_like(A)
    _check(L.rpba_selftest_gemm(_ptr(A), _ptr(B), _ptr(C), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
           "rpba_selftest_gemm")
    return C


def partition(scene, parts, **opts):
    """Sub-blocks from the visibility graph (rpba_partition, Sec. 5.2), on
    the host.  Returns (cam_block [M] int32, node_weight [M], stats dict)."""
    L = load_library()
    o = PartitionOptions()
    _check(L.rpba_partition_default_options(ctypes.byref(o)), "rpba_partition_default_options")
    o.parts = int(parts)
    for k, v in opts.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown partition option {k}")
        setattr(o, k, v)
    cam = np.ascontiguousarray(scene.obs_cam, dtype=np.int32)
    pt = np.ascontiguousarray(scene.obs_pt, dtype=np.int32)
    blk = np.zeros(scene.M, dtype=np.int32)
    nw = np.zeros(scene.M)
    st = np.zeros(8)
    _check(L.rpba_partition(scene.M, scene.N, scene.K, cam.ctypes.data, pt.ctypes.data, ctypes.byref(o),
                            blk.ctypes.data, nw.ctypes.data, st.ctypes.data), "rpba_partition")
    names = ["parts", "edge_cut", "tie_points", "point_copies", "weight_max_over_mean", "cost_max_over_mean",
             "min_cams", "max_cams"]
    return blk, nw, {k: (int(v) if k not in ("weight_max_over_mean", "cost_max_over_mean") else float(v))
                     for k, v in zip(names, st)}


class Problem:
    """One problem on the GPU: device state tensors, workspace, handle."""

    def __init__(self, scene, device="cuda", obs_info=None, **opts):
        """A scene with cam_f / cam_k1 (scenes.with_intrinsics) is adjusted
        with its intrinsics (options intrinsics=1, solver Cholesky) unless
        intrinsics=0 is given."""
        import torch
        self.torch = torch
        L = load_library()
        self.L_ = L
        dev = torch.device(device)
        self.dev = dev
        f64 = torch.float64
        self.M, self.N, self.K, self.L = scene.M, scene.N, scene.K, scene.L
        self.cam_R = torch.as_tensor(np.ascontiguousarray(scene.cam_R), dtype=f64).to(dev)
        self.cam_C = torch.as_tensor(np.ascontiguousarray(scene.cam_C), dtype=f64).to(dev)
        self.pts = torch.as_tensor(np.ascontiguousarray(scene.pts), dtype=f64).to(dev)
        self.obs_xy = torch.as_tensor(np.ascontiguousarray(scene.obs_xy), dtype=f64).to(dev)
        self.obs_info = None if obs_info is None else torch.as_tensor(np.ascontiguousarray(obs_info), dtype=f64).to(dev)
        self._obs_cam = np.ascontiguousarray(scene.obs_cam, dtype=np.int32)
        self._obs_pt = np.ascontiguousarray(scene.obs_pt, dtype=np.int32)
        self._cam_block = np.ascontiguousarray(scene.cam_block, dtype=np.int32)
        if getattr(scene, "cam_f", None) is not None and "intrinsics" not in opts:
            opts["intrinsics"] = 1
        self.np = 8 if opts.get("intrinsics", 0) else 6
        self.cam_intr = None
        if self.np == 8:
            self.cam_intr = torch.as_tensor(np.ascontiguousarray(np.stack([scene.cam_f, scene.cam_k1])),
                                            dtype=f64).to(dev)
        d = ProblemDesc()
        d.M, d.N, d.K, d.L = self.M, self.N, self.K, self.L
        d.f, d.cx, d.cy, d.sigma_px = scene.f, scene.cx, scene.cy, scene.sigma_px
        d.cam_R, d.cam_C, d.pts = self.cam_R.data_ptr(), self.cam_C.data_ptr(), self.pts.data_ptr()
        d.obs_xy = self.obs_xy.data_ptr()
        d.obs_info = None if self.obs_info is None else self.obs_info.data_ptr()
        d.obs_cam = self._obs_cam.ctypes.data
        d.obs_pt = self._obs_pt.ctypes.data
        d.cam_block = self._cam_block.ctypes.data
        d.cam_intr = None if self.cam_intr is None else self.cam_intr.data_ptr()
        self.desc = d
        self.opt = default_options(**opts)
        nbytes = ctypes.c_size_t(0)
        _check(L.rpba_workspace_size(ctypes.byref(d), ctypes.byref(self.opt), ctypes.byref(nbytes)), "rpba_workspace_size")
        self.ws_bytes = nbytes.value
        self.workspace = torch.empty(max(self.ws_bytes, 256), dtype=torch.uint8, device=dev)
        # a dedicated stream: graph capture is not possible on the NULL stream
        self.stream = torch.cuda.Stream(dev)
        h = ctypes.c_void_p(0)
        _check(L.rpba_create(ctypes.byref(d), ctypes.byref(self.opt), ctypes.c_void_p(self.workspace.data_ptr()),
                             self.ws_bytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "rpba_create")
        self.h = h
        self.cov = torch.zeros((6, self.N), dtype=f64, device=dev)
        self.status = torch.zeros(self.N, dtype=torch.int32, device=dev)
        self.int_stats = torch.zeros(4, dtype=f64, device=dev)
        self.block_stats = torch.zeros((self.L, 4), dtype=f64, device=dev)
        self.cons_stats = torch.zeros(2, dtype=f64, device=dev)
        self.rob_stats = torch.zeros(2, dtype=f64, device=dev)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.L_.rpba_destroy(self.h)
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self):
        self.stream.synchronize()

    def set_graph(self, on=True):
        _check(self.L_.rpba_set_graph(self.h, int(on)), "rpba_set_graph")

    def set_timing(self, on=True):
        _check(self.L_.rpba_set_timing(self.h, int(on)), "rpba_set_timing")

    def timing(self):
        n = len(PHASES)
        ms = np.zeros(n)
        la = np.zeros(n, dtype=np.int64)
        ca = np.zeros(n, dtype=np.int64)
        self.L_.rpba_get_timing(self.h, ms.ctypes.data, la.ctypes.data, ca.ctypes.data, n)
        return {PHASES[q]: dict(ms=float(ms[q]), launches=int(la[q]), calls=int(ca[q])) for q in range(n)}

    # --- the method's calls (asynchronous on self.stream; stats stay on the device) ---
    def _order(self):
        # work queued by torch on the caller's stream (e.g. an `active` mask
        # copy) must land before the library's kernels read it
        self.stream.wait_stream(self.torch.cuda.current_stream(self.dev))

    def _hold(self, t):
        # a caller tensor read by work queued on the handle's stream: its
        # memory must not be handed out again (by torch's caching allocator,
        # on the caller's stream) before that work has run
        if t is not None:
            t.record_stream(self.stream)

    def rpba_intersect(self, cov=True, status=True):
        self._order()
        _check(self.L_.rpba_intersect(self.h, _ptr(self.cov) if cov else None, _ptr(self.status) if status else None,
                                      _ptr(self.int_stats)), "rpba_intersect")
        return self.int_stats

    def rpba_robust_reweight(self, mode=0):
        """mode: RPBA_ROBUST_WEIGHT (0 / False), RPBA_ROBUST_ELIMINATE_POINTS
        (1 / True) or RPBA_ROBUST_DELETE_OBS (2).  Device stats [2]: flagged
        observations, eliminated points."""
        self._order()
        _check(self.L_.rpba_robust_reweight(self.h, int(mode), _ptr(self.rob_stats)), "rpba_robust_reweight")
        return self.rob_stats

    def covariance(self, lam=1e-6):
        """(camera covariances [M][np][np] caller order (np = 6, or 8 with
        intrinsics), copy covariances [n_copies][6] in copies() order) of the
        sub-block systems damped by lam (rpba_covariance; the handle needs
        covariance=1)."""
        torch = self.torch
        cc = torch.zeros((self.M, self.np, self.np), dtype=torch.float64, device=self.dev)
        n = int(self.L_.rpba_num_copies(self.h))
        xc = torch.zeros((n, 6), dtype=torch.float64, device=self.dev)
        self._order()
        _check(self.L_.rpba_covariance(self.h, float(lam), _ptr(cc), _ptr(xc)), "rpba_covariance")
        self.sync()
        return cc.cpu().numpy(), xc.cpu().numpy()

    def damping(self):
        """(lambda [L], last step taken back [L]) of the sub-blocks."""
        lam = np.zeros(self.L)
        rej = np.zeros(self.L, dtype=np.int32)
        _check(self.L_.rpba_get_damping(self.h, lam.ctypes.data, rej.ctypes.data), "rpba_get_damping")
        return lam, rej

    def robust_result(self):
        """(sigma_cam [M], obs_weight [K]) of the last robust re-weighting,
        caller order, on the host."""
        sc = np.zeros(self.M)
        w = np.zeros(self.K)
        _check(self.L_.rpba_get_robust(self.h, sc.ctypes.data, w.ctypes.data), "rpba_get_robust")
        return sc, w

    def rpba_subblock_lm_step(self, active=None):
        self._order()
        _check(self.L_.rpba_subblock_lm_step(self.h, _ptr(active), _ptr(self.block_stats)), "rpba_subblock_lm_step")
        self._hold(active)
        return self.block_stats

    def rpba_consensus(self):
        self._order()
        _check(self.L_.rpba_consensus(self.h, _ptr(self.cons_stats)), "rpba_consensus")
        return self.cons_stats

    # --- inspection (synchronous) ---
    def num_copies(self):
        return int(self.L_.rpba_num_copies(self.h))

    def copies(self):
        n = self.num_copies()
        blk = np.zeros(n, dtype=np.int32)
        pt = np.zeros(n, dtype=np.int32)
        X = np.zeros((n, 3))
        om = np.zeros((n, 6))
        _check(self.L_.rpba_get_copies(self.h, blk.ctypes.data, pt.ctypes.data, X.ctypes.data, om.ctypes.data),
               "rpba_get_copies")
        return blk, pt, X, om

    def block_rcs(self, l):
        n6 = self.np * int(self.L_.rpba_block_cameras(self.h, l))
        S = np.zeros((n6, n6))
        e = np.zeros(n6)
        _check(self.L_.rpba_get_block_rcs(self.h, l, S.ctypes.data, e.ctypes.data), "rpba_get_block_rcs")
        return S, e

    def block_solution(self, l):
        n6 = self.np * int(self.L_.rpba_block_cameras(self.h, l))
        x = np.zeros(n6)
        _check(self.L_.rpba_get_block_solution(self.h, l, x.ctypes.data), "rpba_get_block_solution")
        return x

    def set_precond_weights(self, W):
        """W: FP32 device tensor of rpba_precond_num_params() parameters."""
        self._order()
        _check(self.L_.rpba_set_precond_weights(self.h, _ptr(W)), "rpba_set_precond_weights")
        self._hold(W)

    def precond_harvest(self, z):
        """Training samples of the systems at the current state; z: FP32 device
        tensor (nz, M, 6) of probe vectors."""
        nz = int(z.shape[0])
        ns = int(self.L_.rpba_precond_num_samples(self.h))
        stride = int(self.L_.rpba_precond_sample_stride(nz))
        out = self.torch.empty((ns, stride), dtype=self.torch.float32, device=self.dev)
        self._order()
        _check(self.L_.rpba_precond_harvest(self.h, _ptr(z), nz, _ptr(out)), "rpba_precond_harvest")
        self._hold(z)
        # the samples are read on the caller's stream: order it after the harvest
        self.torch.cuda.current_stream(self.dev).wait_stream(self.stream)
        return out

    def block_solver(self, l):
        return int(self.L_.rpba_block_solver(self.h, l))

    def step_status(self):
        """(status code, sub-blocks not positive definite, iterative sub-blocks
        above the refinement tolerance) of the last LM step."""
        a = ctypes.c_int32(0)
        b = ctypes.c_int32(0)
        rc = int(self.L_.rpba_step_status(self.h, ctypes.byref(a), ctypes.byref(b)))
        if rc not in (RPBA_OK, RPBA_ERR_NOT_SPD, RPBA_WARN_NONCONVERGED):
            _check(rc, "rpba_step_status")
        return rc, a.value, b.value

    def factor_flops(self):
        """(method's FP64 operations on the factor's nonzero tiles, dense
        count, matrix-core operations issued) of one factorisation."""
        out = np.zeros(3)
        _check(self.L_.rpba_factor_flops(self.h, out.ctypes.data), "rpba_factor_flops")
        return dict(executed=float(out[0]), dense=float(out[1]), mfma_issued=float(out[2]))

    def camera_order(self):
        """Caller index of every camera in the library's order."""
        o = np.zeros(self.M, dtype=np.int32)
        _check(self.L_.rpba_camera_order(self.h, o.ctypes.data), "rpba_camera_order")
        return o

    def precond_blocks(self, l):
        """CG preconditioner blocks (ncam, 6, 6) of iterative sub-block l from
        the last LM step, cameras in ascending caller index."""
        n = int(self.L_.rpba_block_cameras(self.h, l))
        P = np.zeros((n, 6, 6))
        _check(self.L_.rpba_get_precond_blocks(self.h, l, P.ctypes.data), "rpba_get_precond_blocks")
        return P

    def cameras(self):
        self.stream.synchronize()
        return self.cam_R.cpu().numpy(), self.cam_C.cpu().numpy()

    def intrinsics(self):
        """(f [M], k1 [M]) as the last rpba_consensus wrote them (with
        intrinsics), else the shared f and zeros."""
        self.stream.synchronize()
        if self.cam_intr is None:
            return np.full(self.M, self.desc.f), np.zeros(self.M)
        a = self.cam_intr.cpu().numpy()
        return a[0].copy(), a[1].copy()

    def points(self):
        self.stream.synchronize()
        return self.pts.cpu().numpy()

    def intersection(self):
        self.stream.synchronize()
        return self.pts.cpu().numpy(), self.cov.cpu().numpy(), self.status.cpu().numpy()


def _host(p, t):
    p.sync()
    return t.cpu().numpy().copy()


def _robust_setup(robust, opts):
    """Final mode of the robust cycle (Sec. 5.3): the parallel variant (robust
    True or "parallel", t_v = 4) eliminates whole points, the serial one
    ("serial", t_v = 3) deletes observations."""
    if not robust:
        return None
    if robust not in (True, "parallel", "serial"):
        raise ValueError("robust must be False, True, 'parallel' or 'serial'")
    opts.setdefault("robust", 1)
    if robust == "serial":
        opts.setdefault("t_v", 3.0)
        return RPBA_ROBUST_DELETE_OBS
    return RPBA_ROBUST_ELIMINATE_POINTS


def run_schedule(scene, T=6, I=4, robust=False, t_r=2, callback=None, graph=False, **opts):
    """Fixed schedule on the GPU: T outer iterations of (intersect [, robust
    re-weighting, re-intersect], I LM steps, consensus), then a final
    intersection [, the final robust step of the variant, intersection].
    robust: False, True / "parallel" or "serial"; re-weighting from outer
    iteration t_r on."""
    final_mode = _robust_setup(robust, opts)
    p = Problem(scene, **opts)
    if graph:
        p.set_graph(True)
    hist = []
    for t in range(T):
        st = _host(p, p.rpba_intersect())
        if robust and t >= t_r:
            p.rpba_robust_reweight(RPBA_ROBUST_WEIGHT)
            st = _host(p, p.rpba_intersect())
        rec = dict(t=t, int_stats=st, steps=[])
        for s in range(I):
            bs = _host(p, p.rpba_subblock_lm_step())
            rec["steps"].append(bs)
        rec["consensus"] = _host(p, p.rpba_consensus())
        hist.append(rec)
        if callback:
            callback(p, rec)
    if robust:
        p.rpba_intersect()
        p.rpba_robust_reweight(final_mode)
    final = _host(p, p.rpba_intersect())
    hist.append(dict(t=T, int_stats=final))
    return p, hist


def run_ratio_rule(scene, T_max=10, I_max=10, ratio=1.01, graph=False, robust=False, **opts):
    """Schedule driven by the improvement test of the method (Sec. 5.4,
    rpba_ratio_update): inner loop per sub-block on its cost, a stopped
    sub-block being masked out of the later steps of the outer iteration (the
    `active` mask of rpba_subblock_lm_step); outer loop on the reprojection
    RMS of the intersections.  Returns the problem and per outer iteration
    the number of LM steps each sub-block took.

    With `robust` (True / "parallel" or "serial") the full robust cycle of
    Sec. 5.3: after this basic convergence a second outer loop re-weights
    after every intersection and re-intersects, its improvement test on the
    weighted cost sum v^T W v (what the re-weighted adjustment minimises);
    then the final robust step of the variant and a last intersection.  The
    records of the second loop carry robust=True."""
    import torch
    final_mode = _robust_setup(robust, opts)
    p = Problem(scene, **opts)
    if graph:
        p.set_graph(True)
    L = scene.L
    hist = []
    act_dev = torch.ones(L, dtype=torch.uint8, device=p.dev)

    def outer_loop(weighted):
        o_best, o_grace, o_act = np.zeros(1), np.zeros(1, np.uint8), np.ones(1, np.uint8)
        for t in range(T_max):
            st = _host(p, p.rpba_intersect())
            if weighted:
                p.rpba_robust_reweight(RPBA_ROBUST_WEIGHT)
                st = _host(p, p.rpba_intersect())
            crit = st[0:1] if weighted else st[2:3]
            if t == 0:
                o_best[0] = crit[0]
            elif ratio_update(crit, o_best, o_grace, o_act, ratio) == 0:
                break
            active = np.ones(L, dtype=np.uint8)
            steps = np.zeros(L, dtype=np.int64)
            best = grace = None
            for s in range(I_max):
                act_dev.copy_(torch.as_tensor(active))
                bs = _host(p, p.rpba_subblock_lm_step(act_dev))
                steps[active.astype(bool)] += 1
                if best is None:
                    best, grace = bs[:, 0].copy(), np.zeros(L, np.uint8)
                if ratio_update(bs[:, 1], best, grace, active, ratio) == 0:
                    break
            p.rpba_consensus()
            hist.append(dict(t=len(hist), int_stats=st, steps=steps, robust=weighted))

    outer_loop(False)
    if robust:
        outer_loop(True)
        p.rpba_intersect()
        p.rpba_robust_reweight(final_mode)
    final = _host(p, p.rpba_intersect())
    hist.append(dict(t=len(hist), int_stats=final))
    return p, hist
