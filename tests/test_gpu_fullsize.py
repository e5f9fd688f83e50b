"""Parity at the full size of the benchmark workload (the 6,000-camera
oblique block: 2.5M points, 12.5M observations, 64 sub-blocks) in the launch
configuration the bench times (64-wide tiles, one persistent dataflow
factorisation, HIP graph replay): one outer iteration (intersection, one LM
step of every sub-block, consensus) and the next intersection, against the
FP64 oracle run on the same input.  FP64 path to 1e-9 relative; mixed path
to the bounds stated for it (RMS 1e-6 relative, camera centres 1e-6 of the
scene extent)."""
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
    out = dict(st1=st1, bs=bs, cons=cons, st2=st2, R=R, C=C, X=X, cov=cov, status=status)
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
    assert np.allclose(g["bs"][:, 2], o["bs"][:, 2], rtol=1e-7, atol=0)
    assert g["cons"][1] == o["cons"][1]
    assert abs(g["cons"][0] - o["cons"][0]) <= TOL * _extent(s)
    assert np.allclose(g["st2"], o["st2"], rtol=TOL, atol=0), (g["st2"], o["st2"])
    assert np.abs(g["C"] - o["C"]).max() <= TOL * _extent(s)
    assert np.abs(g["R"] - o["R"]).max() <= TOL
    assert np.array_equal(g["status"], o["status"])
    ok = o["status"] == 0
    assert np.abs(g["X"][:, ok] - o["X"][:, ok]).max() <= TOL * _extent(s)
    rel = np.linalg.norm(g["cov"][:, ok] - o["cov"][:, ok], axis=0) / np.linalg.norm(o["cov"][:, ok], axis=0)
    assert rel.max() <= 1e-8, rel.max()


def test_fullsize_mixed_within_stated_bounds(full):
    from paper_1910_08138_amd import binding
    s, o = full
    g = _gpu_run(s, precision=binding.RPBA_MIXED)
    assert np.all(g["bs"][:, 3] >= 0)
    assert abs(g["st2"][2] - o["st2"][2]) <= 1e-6 * o["st2"][2], (g["st2"], o["st2"])
    assert np.abs(g["C"] - o["C"]).max() <= 1e-6 * _extent(s)
    assert np.array_equal(g["status"], o["status"])
