"""ctypes wrapper of the FP64 CPU oracle (``rpba_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg; the product path never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["rpba_oracle.cpp", "rpba_oracle_solvers.cpp"]
LIB = os.path.join(HERE, "liboracle.so")

ST_OK, ST_NOT_CONVERGED, ST_BEHIND, ST_ILL, ST_ELIMINATED, ST_FILTERED = 0, 1, 2, 3, 4, 5
V_EXTENDED, V_ALL_CAMERAS, V_SCALAR, V_PLAIN, V_PLAIN_REFINED = 0, 1, 2, 3, 4
ROBUST_WEIGHT, ROBUST_ELIMINATE_POINTS, ROBUST_DELETE_OBS = 0, 1, 2


def build(force: bool = True, native: bool = False, path: str | None = None) -> str:
    """Compile the oracle with g++ (-O3, OpenMP).  native=True adds
    -march=native (for timing it on the host that runs it; the default build
    stays portable because it travels with the tree)."""
    srcs = [os.path.join(HERE, s) for s in SOURCES if os.path.exists(os.path.join(HERE, s))]
    out = path or LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        cmd = ["g++", "-std=c++17", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp] + srcs
        if native:
            cmd.insert(2, "-march=native")
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)
    return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=True)
        load(LIB)
    return _lib


def load(path):
    """Use the oracle library at `path` (e.g. a native build) from now on."""
    global _lib
    _lib = ctypes.CDLL(path)
    _declare(_lib)
    return _lib


def set_num_threads(n):
    lib().orc_set_num_threads(int(n))


def num_threads():
    return int(lib().orc_num_threads())


_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)
_up = ctypes.POINTER(ctypes.c_uint8)


def _declare(L):
    L.orc_create.restype = ctypes.c_void_p
    L.orc_create.argtypes = [ctypes.c_int] * 4 + [ctypes.c_double] * 4 + [_dp] * 4 + [_ip, _ip, _dp, _ip,
                                                                                     ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                                                                     ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                                                                     ctypes.c_double]
    L.orc_destroy.argtypes = [ctypes.c_void_p]
    L.orc_intersect.argtypes = [ctypes.c_void_p, _dp]
    L.orc_set_damping.restype = None
    L.orc_set_damping.argtypes = [ctypes.c_void_p, ctypes.c_int] + [ctypes.c_double] * 4
    L.orc_get_damping.restype = None
    L.orc_get_damping.argtypes = [ctypes.c_void_p, _dp, _ip]
    L.orc_covariance.restype = ctypes.c_int
    L.orc_covariance.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp]
    L.orc_robust_reweight.restype = ctypes.c_int
    L.orc_robust_reweight.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
    L.orc_lm_step.restype = ctypes.c_int
    L.orc_lm_step.argtypes = [ctypes.c_void_p, _up, _dp]
    L.orc_consensus.argtypes = [ctypes.c_void_p, _dp]
    L.orc_get_cameras.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.orc_set_cameras.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.orc_get_points.argtypes = [ctypes.c_void_p, _dp]
    L.orc_get_intersection.argtypes = [ctypes.c_void_p, _dp, _dp, _ip]
    L.orc_num_copies.restype = ctypes.c_int
    L.orc_num_copies.argtypes = [ctypes.c_void_p]
    L.orc_get_copies.argtypes = [ctypes.c_void_p, _ip, _ip, _dp, _dp]
    L.orc_get_weights.argtypes = [ctypes.c_void_p, _dp]
    L.orc_set_copies.argtypes = [ctypes.c_void_p, _dp]
    L.orc_get_duals.argtypes = [ctypes.c_void_p, _dp]
    L.orc_set_residuals.argtypes = [ctypes.c_void_p, _dp]
    L.orc_get_residuals.argtypes = [ctypes.c_void_p, _dp]
    L.orc_block_rcs.restype = ctypes.c_int
    L.orc_block_rcs.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    L.orc_block_step.restype = ctypes.c_int
    L.orc_block_step.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp]
    L.orc_linearise.argtypes = [_dp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp, _dp, _dp]
    L.orc_linearise_cal.argtypes = [_dp, _dp, _dp] + [ctypes.c_double] * 4 + [_dp, _dp, _dp]
    L.orc_set_intrinsics.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.orc_get_intrinsics.argtypes = [ctypes.c_void_p, _dp, _dp]
    L.orc_rodrigues.argtypes = [_dp, _dp]
    L.orc_cholesky.restype = ctypes.c_int
    L.orc_cholesky.argtypes = [ctypes.c_int, _dp]
    L.orc_num_threads.restype = ctypes.c_int
    L.orc_set_num_threads.argtypes = [ctypes.c_int]
    _declare_solvers(L)


def _declare_solvers(L):
    if not hasattr(L, "orc_pcg"):
        return
    L.orc_pcg.restype = ctypes.c_int
    L.orc_pcg.argtypes = [ctypes.c_int, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int, _dp, _dp]
    L.orc_mlp_features.argtypes = [ctypes.c_int, _dp, _dp, ctypes.c_double, _dp]
    L.orc_mlp_blocks.argtypes = [ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    L.orc_mlp_loss_grad.restype = ctypes.c_double
    L.orc_mlp_loss_grad.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _dp, _dp, _dp, _dp]
    L.orc_mlp_num_params.restype = ctypes.c_int
    L.orc_mlp_num_params.argtypes = []


def _p(a, t=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleProblem:
    """Stateful oracle run on one scene (same call sequence as the library)."""

    def __init__(self, scene, lam=1e-4, int_tol=1e-12, int_maxit=20, obs_info=None, variant=V_EXTENDED, rho=1000.0,
                 rho_growth=1.01, filter_px=1000.0):
        L = lib()
        self._keep = dict(R=f64(scene.cam_R), C=f64(scene.cam_C), X=f64(scene.pts), xy=f64(scene.obs_xy),
                          cam=i32(scene.obs_cam), pt=i32(scene.obs_pt), blk=i32(scene.cam_block),
                          info=None if obs_info is None else f64(obs_info))
        k = self._keep
        self.M, self.N, self.K, self.L = scene.M, scene.N, scene.K, scene.L
        self.h = L.orc_create(self.M, self.N, self.K, self.L, scene.f, scene.cx, scene.cy, scene.sigma_px,
                              _p(k["R"]), _p(k["C"]), _p(k["X"]), _p(k["xy"]), _p(k["cam"], _ip), _p(k["pt"], _ip),
                              _p(k["info"]), _p(k["blk"], _ip), lam, int_tol, int_maxit, int(variant), float(rho),
                              float(rho_growth), float(filter_px))
        self._lib = L
        # intrinsics (f and k1 per camera, estimated with the poses) when the
        # scene carries them
        self.np = 6
        if getattr(scene, "cam_f", None) is not None:
            f, k1 = f64(scene.cam_f), f64(scene.cam_k1)
            L.orc_set_intrinsics(self.h, _p(f), _p(k1))
            self.np = 8

    def __del__(self):
        if getattr(self, "h", None):
            self._lib.orc_destroy(self.h)
            self.h = None

    def intersect(self):
        s = np.zeros(4)
        self._lib.orc_intersect(self.h, _p(s))
        return s

    def robust_reweight(self, t_v=4.0, down_weight=1e-4, mode=ROBUST_WEIGHT):
        """Per-camera MAD scales and flags (Sec. 5.3); mode ROBUST_WEIGHT,
        ROBUST_ELIMINATE_POINTS (parallel variant) or ROBUST_DELETE_OBS
        (serial variant).  Returns (flagged observations, scales [M])."""
        sc = np.zeros(self.M)
        n = self._lib.orc_robust_reweight(self.h, t_v, down_weight, int(mode), _p(sc))
        return n, sc

    def lm_step(self, active=None):
        bs = np.zeros((self.L, 4))
        act = None if active is None else np.ascontiguousarray(active, dtype=np.uint8)
        fails = self._lib.orc_lm_step(self.h, _p(act, _up), _p(bs))
        return bs, fails

    def consensus(self):
        s = np.zeros(2)
        self._lib.orc_consensus(self.h, _p(s))
        return s

    def cameras(self):
        R = np.zeros((self.M, 9))
        C = np.zeros((3, self.M))
        self._lib.orc_get_cameras(self.h, _p(R), _p(C))
        return R, C

    def intrinsics(self):
        """(f [M], k1 [M]): the cameras' own focal lengths and distortions
        with intrinsics, else the shared f and zeros."""
        f = np.zeros(self.M)
        k1 = np.zeros(self.M)
        self._lib.orc_get_intrinsics(self.h, _p(f), _p(k1))
        return f, k1

    def set_cameras(self, R, C):
        R, C = f64(R), f64(C)
        self._lib.orc_set_cameras(self.h, _p(R), _p(C))

    def points(self):
        X = np.zeros((3, self.N))
        self._lib.orc_get_points(self.h, _p(X))
        return X

    def intersection(self):
        X = np.zeros((3, self.N))
        cov = np.zeros((6, self.N))
        st = np.zeros(self.N, dtype=np.int32)
        self._lib.orc_get_intersection(self.h, _p(X), _p(cov), _p(st, _ip))
        return X, cov, st

    def copies(self):
        n = self._lib.orc_num_copies(self.h)
        blk = np.zeros(n, dtype=np.int32)
        pt = np.zeros(n, dtype=np.int32)
        X = np.zeros((n, 3))
        om = np.zeros((n, 6))
        self._lib.orc_get_copies(self.h, _p(blk, _ip), _p(pt, _ip), _p(X), _p(om))
        return blk, pt, X, om

    def set_copies(self, X):
        """Test hook: X [n_copies][3] in the order of copies()."""
        X = f64(X)
        assert X.shape == (self._lib.orc_num_copies(self.h), 3)
        self._lib.orc_set_copies(self.h, _p(X))

    def duals(self):
        """Dual offsets Xtilde [n_copies][3] of the plain variants."""
        Xt = np.zeros((self._lib.orc_num_copies(self.h), 3))
        self._lib.orc_get_duals(self.h, _p(Xt))
        return Xt

    def set_residuals(self, res):
        """Test hook: residuals [2][K] of the last intersection (pixels)."""
        res = f64(res)
        assert res.shape == (2, self.K)
        self._lib.orc_set_residuals(self.h, _p(res))

    def weights(self):
        w = np.zeros(self.K)
        self._lib.orc_get_weights(self.h, _p(w))
        return w

    def residuals(self):
        r = np.zeros((2, self.K))
        self._lib.orc_get_residuals(self.h, _p(r))
        return r

    def set_damping(self, mode=1, up=10.0, down=10.0, lam_min=1e-12, lam_max=1e8):
        """Adaptive damping per sub-block (mode 1) or the fixed lambda (0)."""
        self._lib.orc_set_damping(self.h, int(mode), float(up), float(down), float(lam_min), float(lam_max))

    def damping(self):
        """(lambda [L], last step rejected [L])."""
        lam = np.zeros(self.L)
        rej = np.zeros(self.L, dtype=np.int32)
        self._lib.orc_get_damping(self.h, _p(lam), _p(rej, _ip))
        return lam, rej

    def covariance(self, lam=1e-6):
        """(camera covariances [M][np][np], copy covariances [n_copies][6])
        of the sub-block normal equations damped by lam (Sec. 2); np = 6, or 8
        with intrinsics."""
        cc = np.zeros((self.M, self.np, self.np))
        xc = np.zeros((self._lib.orc_num_copies(self.h), 6))
        rc = self._lib.orc_covariance(self.h, float(lam), _p(cc), _p(xc))
        if rc < 0:
            raise np.linalg.LinAlgError(f"sub-block {-rc - 1} not positive definite")
        return cc, xc

    def block_rcs(self, l, n6):
        S = np.zeros((n6, n6))
        e = np.zeros(n6)
        n = self._lib.orc_block_rcs(self.h, l, _p(S), _p(e))
        if n < 0:
            raise RuntimeError("singular point block")
        return S, e

    def block_step(self, l, n6, n_copies):
        dC = np.zeros(n6)
        dX = np.zeros(3 * n_copies)
        nc = self._lib.orc_block_step(self.h, l, _p(dC), _p(dX))
        if nc < 0:
            raise RuntimeError(f"block step failed {nc}")
        return dC, dX[: 3 * nc].reshape(-1, 3)


def linearise(R9, C3, X3, f=1000.0, cx=500.0, cy=500.0):
    R9, C3, X3 = f64(R9), f64(C3), f64(X3)
    g = np.zeros(2)
    A = np.zeros((2, 6))
    B = np.zeros((2, 3))
    lib().orc_linearise(_p(R9), _p(C3), _p(X3), f, cx, cy, _p(g), _p(A), _p(B))
    return g, A, B


def linearise_cal(R9, C3, X3, f=1000.0, k1=0.0, cx=500.0, cy=500.0):
    """Projection with the camera's own f and k1: (g [2], A [2][8] =
    dg/d(w, C, f, k1), B [2][3])."""
    R9, C3, X3 = f64(R9), f64(C3), f64(X3)
    g = np.zeros(2)
    A = np.zeros((2, 8))
    B = np.zeros((2, 3))
    lib().orc_linearise_cal(_p(R9), _p(C3), _p(X3), f, k1, cx, cy, _p(g), _p(A), _p(B))
    return g, A, B


def rodrigues(w):
    w = f64(w)
    R = np.zeros(9)
    lib().orc_rodrigues(_p(w), _p(R))
    return R.reshape(3, 3)


def cholesky(A):
    A = f64(A).copy()
    n = A.shape[0]
    rc = lib().orc_cholesky(n, _p(A))
    if rc:
        raise np.linalg.LinAlgError("not SPD")
    return np.tril(A)


def pcg(S, e, P=None, tol=1e-8, maxit=1000):
    """Block-preconditioned CG (x0 = 0) on a dense symmetric system; P: (n/6, 6, 6)
    blocks or None for block-Jacobi.  Returns (x, iterations, relative residuals)."""
    S, e = f64(S), f64(e)
    n = S.shape[0]
    x = np.zeros(n)
    hist = np.zeros(maxit)
    Pp = None if P is None else f64(P)
    it = lib().orc_pcg(n, _p(S), _p(e), _p(Pp), tol, maxit, _p(x), _p(hist))
    if it < 0:
        raise np.linalg.LinAlgError("diagonal block not positive definite")
    return x, it, hist[:it]


MLP_NF, MLP_NH, MLP_NO = 26, 64, 21


def mlp_num_params():
    return int(lib().orc_mlp_num_params())


def mlp_features(S, obs_tp, lam=1e-4):
    S = f64(S)
    n = S.shape[0]
    obs_tp = f64(obs_tp)
    feat = np.zeros((n // 6, MLP_NF))
    lib().orc_mlp_features(n, _p(S), _p(obs_tp), lam, _p(feat))
    return feat


def mlp_blocks(S, feat, params=None):
    """(P blocks (nb, 6, 6), G^-1 blocks (nb, 6, 6))"""
    S = f64(S)
    n = S.shape[0]
    feat = f64(feat)
    P = np.zeros((n // 6, 6, 6))
    Gi = np.zeros((n // 6, 6, 6))
    pp = None if params is None else f64(params)
    lib().orc_mlp_blocks(n, _p(S), _p(feat), _p(pp), _p(P), _p(Gi))
    return P, Gi


def mlp_loss_grad(Ginv, feat, params, zw):
    """Hutchinson SPAI loss and gradient; zw: (nz, 2, n) probe pairs (z, S z)."""
    Ginv, feat, params, zw = f64(Ginv), f64(feat), f64(params), f64(zw)
    nb = Ginv.shape[0]
    grad = np.zeros(mlp_num_params())
    loss = lib().orc_mlp_loss_grad(nb, zw.shape[0], _p(Ginv), _p(feat), _p(params), _p(zw), _p(grad))
    return loss, grad


def _robust_mode(robust, t_v):
    """(final mode, t_v) of the robust cycle (Sec. 5.3): parallel variant
    (True or "parallel"): points eliminated, t_v = 4; serial ("serial"):
    observations deleted, t_v = 3."""
    if not robust:
        return None, t_v
    if robust not in (True, "parallel", "serial"):
        raise ValueError("robust must be False, True, 'parallel' or 'serial'")
    if robust == "serial":
        return ROBUST_DELETE_OBS, 3.0 if t_v is None else t_v
    return ROBUST_ELIMINATE_POINTS, 4.0 if t_v is None else t_v


def run_schedule(scene, T=6, I=4, robust=False, t_r=2, t_v=None, down_weight=1e-4, callback=None, **kw):
    """Fixed schedule: T outer iterations of (intersect [, robust re-weighting,
    re-intersect], I LM steps, consensus), then a final intersection [, the
    final robust step of the variant, intersection].  Returns the oracle
    problem and a list of per-iteration records."""
    final_mode, t_v = _robust_mode(robust, t_v)
    op = OracleProblem(scene, **kw)
    hist = []
    for t in range(T):
        st = op.intersect()
        if robust and t >= t_r:
            op.robust_reweight(t_v, down_weight, ROBUST_WEIGHT)
            st = op.intersect()
        rec = dict(t=t, int_stats=st, steps=[])
        for s in range(I):
            bs, fails = op.lm_step()
            rec["steps"].append((bs, fails))
        rec["consensus"] = op.consensus()
        hist.append(rec)
        if callback:
            callback(op, rec)
    if robust:
        op.intersect()
        op.robust_reweight(t_v, down_weight, final_mode)
    final = op.intersect()
    hist.append(dict(t=T, int_stats=final))
    return op, hist


class RatioRule:
    """Improvement test that ends a loop (Sec. 5.4): the best cost reached
    so far is compared with the current one; a ratio below `ratio` (1.01)
    is tolerated once, the second such step ends the loop.  `first` is the
    cost before the first step.  step(cost) returns False when the loop
    ends with this step."""

    def __init__(self, first, ratio=1.01):
        self.best = float(first)
        self.ratio = float(ratio)
        self.grace = False

    def step(self, cost):
        slow = self.best / cost < self.ratio
        self.best = min(self.best, cost)
        if slow:
            if self.grace:
                return False
            self.grace = True
        return True


def run_ratio_rule(scene, T_max=10, I_max=10, ratio=1.01, robust=False, t_v=None, down_weight=1e-4, **kw):
    """Schedule driven by the improvement test (RatioRule): inner loop per
    sub-block on its cost (a sub-block that stops is left out of the later
    steps of this outer iteration), outer loop on the reprojection RMS of the
    intersections.  Returns the problem and per outer iteration the number of
    steps each sub-block took.

    With `robust` (True / "parallel" or "serial"), the robust cycle of Sec.
    5.3: after this basic convergence, a second outer loop that re-weights
    after each intersection and intersects again, stopped by the same test on
    the weighted cost sum v^T W v; then the final robust step of the variant
    and a last intersection."""
    final_mode, t_v = _robust_mode(robust, t_v)
    op = OracleProblem(scene, **kw)
    L = scene.L
    hist = []

    def outer_loop(weighted):
        outer = None
        for t in range(T_max):
            st = op.intersect()
            if weighted:
                op.robust_reweight(t_v, down_weight, ROBUST_WEIGHT)
                st = op.intersect()
            crit = st[0] if weighted else st[2]
            if outer is None:
                outer = RatioRule(crit, ratio)
            elif not outer.step(crit):
                break
            active = np.ones(L, dtype=np.uint8)
            steps = np.zeros(L, dtype=np.int64)
            rules = None
            for s in range(I_max):
                bs, fails = op.lm_step(active)
                if rules is None:
                    rules = [RatioRule(bs[l, 0], ratio) for l in range(L)]
                for l in range(L):
                    if active[l]:
                        steps[l] += 1
                        if not rules[l].step(bs[l, 1]):
                            active[l] = 0
                if not active.any():
                    break
            op.consensus()
            hist.append(dict(t=len(hist), int_stats=st, steps=steps, robust=weighted))

    outer_loop(False)
    if robust:
        outer_loop(True)
        op.intersect()
        op.robust_reweight(t_v, down_weight, final_mode)
    final = op.intersect()
    hist.append(dict(t=len(hist), int_stats=final))
    return op, hist
