"""The variants of the method on the GPU against the oracle (FP64, 1e-9
relative per result): tie-point weights from all cameras or a scalar
(Sec. 6.4), the plain ADMM consensus (Sec. 4, eq:admm7-eq:admm9) with its
growing scalar weight and filters (Sec. 6.3), and the plain consensus with
the weights of Sec. 5.1.  Whole fixed schedules: intersection (or, for the
plain variants, evaluation at the consensus point), LM steps, consensus."""
import numpy as np
import pytest

import oracle
from paper_1910_08138_amd import scenes

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def rp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08138_amd import binding
    binding.load_library()
    return binding


def _extent(scene):
    C = scene.cam_C_true
    return float(np.linalg.norm(C.max(axis=1) - C.min(axis=1))) + 1.0


VARIANTS = [("all-cameras", 1, 1000.0), ("scalar", 2, 2000.0), ("plain", 3, 2000.0), ("plain-refined", 4, 1000.0)]


@pytest.mark.parametrize("name,variant,rho", VARIANTS)
@pytest.mark.parametrize("scene", ["ring", "aerial-small"])
def test_variant_fixed_schedule_parity(rp, name, variant, rho, scene):
    s = scenes.config_scene(1, 41) if scene == "ring" else scenes.config_scene(2, 41, small=True)
    T, I = 4, 3
    gp, gh = rp.run_schedule(s, T=T, I=I, graph=True, variant=variant, rho=rho)
    op, oh = oracle.run_schedule(s, T=T, I=I, variant=variant, rho=rho)
    for g, o in zip(gh, oh):
        assert np.allclose(g["int_stats"], o["int_stats"], rtol=TOL, atol=0), (g["t"], g["int_stats"], o["int_stats"])
        for bg, (bo, fails) in zip(g.get("steps", []), o.get("steps", [])):
            assert fails == 0
            assert np.allclose(bg[:, :3], bo[:, :3], rtol=TOL, atol=1e-300)
        if "consensus" in g:
            assert g["consensus"][1] == o["consensus"][1]
            assert abs(g["consensus"][0] - o["consensus"][0]) <= TOL * _extent(s)
    gR, gC = gp.cameras()
    oR, oC = op.cameras()
    assert np.abs(gC - oC).max() <= TOL * _extent(s)
    assert np.abs(gR - oR).max() <= TOL
    gX, _, gst = gp.intersection()
    oX, _, ost = op.intersection()
    assert np.array_equal(gst, ost)
    ok = ost == 0
    assert np.abs(gX[:, ok] - oX[:, ok]).max() <= TOL * _extent(s)
    gb, gpt, gXc, gom = gp.copies()
    ob, opt_, oXc, oom = op.copies()
    o1, o2 = np.lexsort((gpt, gb)), np.lexsort((opt_, ob))
    assert np.abs(gom[o1] - oom[o2]).max() <= TOL * np.abs(oom).max()
    if variant >= 3:
        # the plain copies are never reset: compare them directly
        assert np.abs(gXc[o1] - oXc[o2]).max() <= TOL * _extent(s)


def test_plain_filter_on_gpu(rp):
    """Sec. 6.3 filter: a point with a reprojection error above filter_px
    (one observation moved by 1,500 px) is dropped by the plain evaluation,
    with the same status as in the oracle."""
    s = scenes.ring_scene(33, n_pts=300)
    k = int(np.nonzero(s.obs_pt == 7)[0][0])
    s.obs_xy = s.obs_xy.copy()
    s.obs_xy[0, k] += 1500.0
    gp = rp.Problem(s, variant=rp.RPBA_VARIANT_PLAIN)
    op = oracle.OracleProblem(s, variant=oracle.V_PLAIN)
    gst = gp.rpba_intersect()
    gp.sync()
    ost = op.intersect()
    assert np.allclose(gst.cpu().numpy(), ost, rtol=TOL, atol=0)
    X, _, st = gp.intersection()
    _, _, sto = op.intersection()
    assert np.array_equal(st, sto) and st[7] == oracle.ST_FILTERED
    assert np.array_equal(X[:, st == 0], s.pts[:, st == 0])
