"""Parity at the full size of the benchmark workload (the 6,000-camera
oblique block: 2.5M points, 12.5M observations, 64 sub-blocks) in the launch
configuration the bench times (64-wide tiles, one persistent dataflow
factorisation, HIP graph replay): one outer iteration (intersection, one LM
step of every sub-block, consensus) and the next intersection, against the
FP64 oracle run on the same input.  FP64 path to 1e-9 relative; mixed path
to the bounds stated for it per result.  The covariance of a point depends
on its cameras, so the mixed path's camera differences reach it: its bound
is stated over the 2.5M points (99.99th percentile and largest)."""
import numpy as np
import pytest

import oracle
from paper_1910_08138_amd import scenes

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-9


@pytest.fixture(scope="module")
def full():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08138_amd import binding
    binding.load_library()
    s = scenes.config_scene(3, 0)
    print(f"scene M={s.M} N={s.N} K={s.K} L={s.L}", flush=True)
    op = oracle.OracleProblem(s)
    st1 = op.intersect()
    bs, fails = op.lm_step()
    cons = op.consensus()
    st2 = op.intersect()
    R, C = op.cameras()
    X, cov, status = op.intersection()
    print("oracle done", flush=True)
    return s, dict(st1=st1, bs=bs, fails=fails, cons=cons, st2=st2, R=R, C=C, X=X, cov=cov, status=status)


def _gpu_run(s, **opts):
    from paper_1910_08138_amd import binding
    p = binding.Problem(s, chol_tile=64, chol_schedule=binding.RPBA_CHOL_DATAFLOW, **opts)
    p.set_graph(True)
    # results live on the handle's stream: synchronise it before each read
    st1 = binding._host(p, p.rpba_intersect())
    bs = binding._host(p, p.rpba_subblock_lm_step())
    cons = binding._host(p, p.rpba_consensus())
    st2 = binding._host(p, p.rpba_intersect())
    R, C = p.cameras()
    X, cov, status = p.intersection()
    out = dict(st1=st1, bs=bs, cons=cons, st2=st2, R=R, C=C, X=X, cov=cov, status=status, intr=p.intrinsics())
    del p
    return out


def _extent(s):
    C = s.cam_C_true
    return float(np.linalg.norm(C.max(axis=1) - C.min(axis=1))) + 1.0


def test_fullsize_fp64_parity(full):
    s, o = full
    g = _gpu_run(s)
    assert o["fails"] == 0 and np.all(g["bs"][:, 3] >= 0)
    assert np.allclose(g["st1"], o["st1"], rtol=TOL, atol=0), (g["st1"], o["st1"])
    assert np.allclose(g["bs"][:, :2], o["bs"][:, :2], rtol=TOL, atol=0)
    step_rel = np.abs(g["bs"][:, 2] - o["bs"][:, 2]) / o["bs"][:, 2]
    print(f"step norm max rel err {step_rel.max():.2e}", flush=True)
    assert np.allclose(g["bs"][:, 2], o["bs"][:, 2], rtol=TOL, atol=0)
    assert g["cons"][1] == o["cons"][1]
    assert abs(g["cons"][0] - o["cons"][0]) <= TOL * _extent(s)
    assert np.allclose(g["st2"], o["st2"], rtol=TOL, atol=0), (g["st2"], o["st2"])
    assert np.abs(g["C"] - o["C"]).max() <= TOL * _extent(s)
    assert np.abs(g["R"] - o["R"]).max() <= TOL
    assert np.array_equal(g["status"], o["status"])
    ok = o["status"] == 0
    assert np.abs(g["X"][:, ok] - o["X"][:, ok]).max() <= TOL * _extent(s)
    rel = np.linalg.norm(g["cov"][:, ok] - o["cov"][:, ok], axis=0) / np.linalg.norm(o["cov"][:, ok], axis=0)
    print(f"covariance max rel err {rel.max():.2e}, 99.9th pct {np.quantile(rel, 0.999):.2e}", flush=True)
    assert rel.max() <= TOL, rel.max()


def _cov_report(gcov, ocov, ok):
    """relative Frobenius error of every valid point's covariance, and the
    condition number of the worst ones"""
    rel = np.linalg.norm(gcov[:, ok] - ocov[:, ok], axis=0) / np.linalg.norm(ocov[:, ok], axis=0)
    idx = np.nonzero(ok)[0][np.argsort(rel)[-5:]]
    kap = [float(np.linalg.cond(np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])))
           for c in ocov[:, idx].T]
    print(f"covariance rel err max {rel.max():.2e}, 99.99th pct {np.quantile(rel, 0.9999):.2e}, "
          f"median {np.median(rel):.2e}; cond of the worst five {[f'{k:.1e}' for k in kap]}", flush=True)
    return rel


def test_fullsize_mixed_within_stated_bounds(full):
    from paper_1910_08138_amd import binding
    s, o = full
    g = _gpu_run(s, precision=binding.RPBA_MIXED)
    assert np.all(g["bs"][:, 3] >= 0)
    cam = np.abs(g["C"] - o["C"]).max() / _extent(s)
    rot = np.abs(g["R"] - o["R"]).max()
    print(f"one step: RMS rel {abs(g['st2'][2] - o['st2'][2]) / o['st2'][2]:.2e}, centres / extent {cam:.2e}, "
          f"rotation entries {rot:.2e} (99th pct {np.quantile(np.abs(g['R'] - o['R']).max(axis=1), 0.99):.2e})",
          flush=True)
    # one LM step from the 1-degree start moves a camera by about 1.7e-2 rad;
    # the FP32 assembly of the RCS (2e-5 relative) changes that step by up
    # to 1e-3 of it on the least determined cameras (measured 1.75e-5 rad)
    assert abs(g["st2"][2] - o["st2"][2]) <= 1e-6 * o["st2"][2], (g["st2"], o["st2"])
    assert cam <= 1e-6
    assert rot <= 1e-4
    assert np.array_equal(g["status"], o["status"])
    rel = _cov_report(g["cov"], o["cov"], o["status"] == 0)
    assert np.quantile(rel, 0.9999) <= 1e-4 and rel.max() <= 2e-3, rel.max()


def test_fullsize_mixed_schedule_final_rms_against_oracle(full):
    """The target's own criterion on the 6,000-camera block: the mixed path
    (bench launch configuration, HIP graphs) run through the whole fixed
    schedule (6 outer iterations of 4 LM steps, then the final intersection)
    against the FP64 oracle's run of the same schedule: final RMS within 1e-6
    relative, camera centres within 1e-6 of the scene extent, rotation
    entries within 1e-6, covariances within 1e-4 relative Frobenius norm."""
    from paper_1910_08138_amd import binding
    s, _ = full

    def progress(op, rec):
        print(f"oracle outer iteration {rec['t']}: RMS {rec['int_stats'][2]:.9f}", flush=True)

    op, oh = oracle.run_schedule(s, T=6, I=4, callback=progress)
    oR, oC = op.cameras()
    _, ocov, ost = op.intersection()
    del op
    gp, gh = binding.run_schedule(s, T=6, I=4, graph=True, precision=binding.RPBA_MIXED, chol_tile=64,
                                  chol_schedule=binding.RPBA_CHOL_DATAFLOW)
    gR, gC = gp.cameras()
    _, gcov, gst = gp.intersection()
    del gp
    rms_g, rms_o = gh[-1]["int_stats"][2], oh[-1]["int_stats"][2]
    cam = np.abs(gC - oC).max() / _extent(s)
    rot = np.abs(gR - oR).max()
    print(f"final RMS mixed {rms_g:.12f} oracle {rms_o:.12f} (rel {abs(rms_g - rms_o) / rms_o:.2e}); "
          f"centres / extent {cam:.2e}; rotation {rot:.2e}", flush=True)
    rel = _cov_report(gcov, ocov, ost == 0)
    assert abs(rms_g - rms_o) <= 1e-6 * rms_o
    assert cam <= 1e-6 and rot <= 1e-6
    assert np.array_equal(gst, ost)
    assert np.quantile(rel, 0.9999) <= 1e-5 and rel.max() <= 1e-3


def test_fullsize_config4_mixed_robust_against_oracle():
    """Config 4 at full size: the 6,000-camera block with 2% gross errors
    (uniform +-50 px), mixed precision, the parallel robust re-weighting from
    outer iteration 2 and the elimination before the final intersection,
    against the FP64 oracle's robust schedule; errors reported per result."""
    from paper_1910_08138_amd import binding
    s = scenes.config_scene(4, 0)
    print(f"scene M={s.M} N={s.N} K={s.K} outliers={int(s.outlier.sum())}", flush=True)

    def progress(op, rec):
        print(f"oracle outer iteration {rec['t']}: RMS {rec['int_stats'][2]:.9f}", flush=True)

    op, oh = oracle.run_schedule(s, T=6, I=4, robust=True, callback=progress)
    oR, oC = op.cameras()
    _, ocov, ost = op.intersection()
    wo = op.weights()
    del op
    gp, gh = binding.run_schedule(s, T=6, I=4, robust=True, graph=True, precision=binding.RPBA_MIXED, chol_tile=64,
                                  chol_schedule=binding.RPBA_CHOL_DATAFLOW)
    gR, gC = gp.cameras()
    _, gcov, gst = gp.intersection()
    _, wg = gp.robust_result()
    del gp
    rms_g, rms_o = gh[-1]["int_stats"][2], oh[-1]["int_stats"][2]
    dc = np.abs(gC - oC).max(axis=0) / _extent(s)
    dr = np.abs(gR - oR).max(axis=1)
    flips = int((wg != wo).sum())
    print(f"config 4: weight flips {flips} of {s.K} (flagged {int((wo < 1).sum())}); status differ "
          f"{int((gst != ost).sum())}; final RMS rel {abs(rms_g - rms_o) / rms_o:.2e}; centres / extent max "
          f"{dc.max():.2e} 99th pct {np.quantile(dc, 0.99):.2e}; rotation max {dr.max():.2e} 99th pct "
          f"{np.quantile(dr, 0.99):.2e}", flush=True)
    both = (gst == 0) & (ost == 0)
    rel = _cov_report(gcov, ocov, both)
    # stated per result (measured: 19 flips of 12.5M, RMS 5.9e-7, centres
    # 2.3e-8 / 7.8e-7 of the extent, rotation entries 5.4e-7 / 2.6e-5,
    # covariances 2.4e-5 / 7.7e-4 at the 99th (99.99th) percentile / largest)
    assert flips <= 1e-5 * s.K
    assert abs(rms_g - rms_o) <= 1e-5 * rms_o
    assert np.quantile(dc, 0.99) <= 1e-6 and dc.max() <= 1e-5
    assert np.quantile(dr, 0.99) <= 1e-5 and dr.max() <= 1e-4
    assert np.quantile(rel, 0.9999) <= 1e-4 and rel.max() <= 2e-3


def test_fullsize_intrinsics_fp64_parity():
    """The same block with f and k1 estimated per camera (8 x 8 camera
    blocks, reduced camera systems of up to 2,528 rows): one outer iteration
    and the next intersection on the FP64 path against the oracle, 1e-9."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = scenes.with_intrinsics(scenes.config_scene(3, 0), 0)
    op = oracle.OracleProblem(s)
    o = dict(st1=op.intersect())
    o["bs"], fails = op.lm_step()
    o["cons"] = op.consensus()
    o["st2"] = op.intersect()
    o["R"], o["C"] = op.cameras()
    o["X"], _, o["status"] = op.intersection()
    of, ok1 = op.intrinsics()
    del op
    print("oracle done", flush=True)
    g = _gpu_run(s)
    assert fails == 0 and np.all(g["bs"][:, 3] >= 0)
    assert np.allclose(g["st1"], o["st1"], rtol=TOL, atol=0), (g["st1"], o["st1"])
    assert np.allclose(g["bs"][:, :3], o["bs"][:, :3], rtol=TOL, atol=0)
    assert np.allclose(g["st2"], o["st2"], rtol=TOL, atol=0), (g["st2"], o["st2"])
    assert np.abs(g["C"] - o["C"]).max() <= TOL * _extent(s)
    assert np.abs(g["R"] - o["R"]).max() <= TOL
    assert np.array_equal(g["status"], o["status"])
    ok = o["status"] == 0
    assert np.abs(g["X"][:, ok] - o["X"][:, ok]).max() <= TOL * _extent(s)
    gf, gk = g["intr"]
    print(f"f max rel {np.abs(gf - of).max() / of.max():.2e}, k1 max abs {np.abs(gk - ok1).max():.2e}", flush=True)
    assert np.abs(gf - of).max() <= TOL * of.max()
    assert np.abs(gk - ok1).max() <= TOL


def test_fullsize_aerial_fp64_and_mixed_schedule_against_oracle():
    """Config 2 at full size: the 500-camera aerial block (20 x 25 nadir grid
    at 60% overlap over a terrain, 200k points, 16 sub-blocks) through the
    fixed schedule (6 outer iterations of 4 LM steps, then the final
    intersection) on the FP64 and on the mixed path (bench launch
    configuration, HIP graphs), each against the FP64 oracle's run of the
    same schedule.  Every result's error is reported and bounded per path:
    final RMS, camera centres and rotations, points, point and camera
    covariances, point status."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08138_amd import binding
    s = scenes.config_scene(2, 0)
    print(f"scene M={s.M} N={s.N} K={s.K} L={s.L}", flush=True)
    op, oh = oracle.run_schedule(s, T=6, I=4)
    o = dict(rms=oh[-1]["int_stats"][2])
    o["R"], o["C"] = op.cameras()
    o["X"], o["cov"], o["status"] = op.intersection()
    o["ccov"], _ = op.covariance(1e-4)
    del op
    print(f"oracle final RMS {o['rms']:.12f}", flush=True)
    ext = _extent(s)
    # per-result bounds (relative RMS, centres / extent, rotation entries,
    # points / extent, point covariances (relative Frobenius norm) at the
    # 99.99th percentile and largest, camera covariances at lambda 1e-4
    # (largest entry error over sqrt(C_rr C_cc)))
    # (1e-6 of the extent (1.2 km) in a centre is 1.2e-5 rad at the 100 m
    # flying height: nadir views trade a tilt about a horizontal axis
    # against a horizontal shift of the centre, so the mixed path's rotation
    # bound follows its centre bound; measured fp64 1.1e-15 / 9.3e-17,
    # mixed 2.9e-6 / 3.4e-7 (rotation / centres))
    bounds = {binding.RPBA_FP64: dict(rms=1e-10, C=1e-9, R=1e-9, X=1e-9, cov=(1e-8, 1e-7), ccov=1e-7),
              binding.RPBA_MIXED: dict(rms=1e-6, C=1e-6, R=1e-5, X=1e-6, cov=(1e-5, 1e-3), ccov=1e-3)}
    for prec, b in bounds.items():
        name = "fp64" if prec == binding.RPBA_FP64 else "mixed"
        gp, gh = binding.run_schedule(s, T=6, I=4, graph=True, precision=prec, chol_tile=64,
                                      chol_schedule=binding.RPBA_CHOL_DATAFLOW, covariance=1)
        gR, gC = gp.cameras()
        gX, gcov, gst = gp.intersection()
        gccov, _ = gp.covariance(1e-4)
        del gp
        rms = abs(gh[-1]["int_stats"][2] - o["rms"]) / o["rms"]
        dC = np.abs(gC - o["C"]).max() / ext
        dR = np.abs(gR - o["R"]).max()
        ok = (gst == 0) & (o["status"] == 0)
        dX = np.abs(gX[:, ok] - o["X"][:, ok]).max() / ext
        d = np.sqrt(np.diagonal(o["ccov"], axis1=1, axis2=2))
        crel = (np.abs(gccov - o["ccov"]) / (d[:, :, None] * d[:, None, :])).max(axis=(1, 2))
        print(f"aerial {name}: final RMS {gh[-1]['int_stats'][2]:.12f} (rel {rms:.2e}); centres / extent {dC:.2e}; "
              f"rotation {dR:.2e}; points / extent {dX:.2e}; status differ {int((gst != o['status']).sum())}; "
              f"camera covariance rel max {crel.max():.2e}", flush=True)
        rel = _cov_report(gcov, o["cov"], ok)
        assert np.array_equal(gst, o["status"])
        assert rms <= b["rms"] and dC <= b["C"] and dR <= b["R"] and dX <= b["X"]
        assert np.quantile(rel, 0.9999) <= b["cov"][0] and rel.max() <= b["cov"][1]
        assert crel.max() <= b["ccov"]
