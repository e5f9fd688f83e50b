"""Robust re-weighting (paper Sec. 5.3, parallel variant) on the GPU vs the
FP64 oracle: per-camera MAD scales, the observation weight multipliers, the
flag and elimination counts, and whole robust schedules.

The scales are exact order statistics on both sides (a sort in the oracle, a
radix select on the GPU) of whitened residuals that agree to rounding, so
they agree to 1e-9 relative; the weights are compared exactly (a flip would
need a residual within rounding of the t_v threshold)."""
import numpy as np
import pytest

import oracle
from paper_1910_08138_amd import scenes

pytestmark = pytest.mark.gpu

TOL = 1e-9
LDS_COMPONENTS = 8192   # whitened components a camera may stage in LDS


@pytest.fixture(scope="module")
def rp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08138_amd import binding
    binding.load_library()
    return binding


def _one_reweight(rp, s, eliminate):
    gp = rp.Problem(s, robust=1)
    op = oracle.OracleProblem(s)
    gp.rpba_intersect()
    op.intersect()
    gst = gp.rpba_robust_reweight(eliminate)
    gp.sync()
    gst = gst.cpu().numpy()
    n_o, sc_o = op.robust_reweight(4.0, 1e-4, eliminate=eliminate)
    sc_g, w_g = gp.robust_result()
    return gp, op, gst, n_o, sc_o, sc_g, w_g


@pytest.mark.parametrize("eliminate", [False, True])
def test_scales_weights_and_flags(rp, eliminate):
    s = scenes.config_scene(4, 2, small=True)
    assert s.outlier is not None and s.outlier.sum() > 0
    gp, op, gst, n_o, sc_o, sc_g, w_g = _one_reweight(rp, s, eliminate)
    assert np.all(sc_o > 0)
    assert np.abs(sc_g - sc_o).max() <= TOL * sc_o.max()
    assert np.array_equal(w_g, op.weights())
    assert int(gst[0]) == n_o and n_o > 0
    # gross errors are flagged far more often than clean observations
    assert (w_g[s.outlier] < 1).mean() > 20 * (w_g[~s.outlier] < 1).mean()
    gp.rpba_intersect()
    op.intersect()
    _, _, gstat = gp.intersection()
    _, _, ostat = op.intersection()
    assert np.array_equal(gstat, ostat)
    if eliminate:
        assert int(gst[1]) == int((ostat == 4).sum()) > 0
    else:
        assert int(gst[1]) == 0 and not np.any(ostat == 4)


def test_cameras_beyond_lds_use_global_staging(rp):
    """Cameras with more residual components than the LDS holds select their
    medians from a global slice of the workspace."""
    s = scenes.ring_scene(4, n_cams=10, n_pts=9000, views=(2, 10))
    per_cam = np.bincount(s.obs_cam, minlength=s.M)
    assert 2 * per_cam.max() > LDS_COMPONENTS
    gp, op, gst, n_o, sc_o, sc_g, w_g = _one_reweight(rp, s, False)
    assert np.abs(sc_g - sc_o).max() <= TOL * sc_o.max()
    assert np.array_equal(w_g, op.weights())
    assert int(gst[0]) == n_o


def test_camera_without_valid_points_has_zero_scale(rp):
    """A camera whose every point is invalid gets scale 0 and flags nothing:
    turned half a revolution about its y axis, it sees all its points behind
    it, so the intersection rejects them."""
    s = scenes.ring_scene(5, n_cams=12, n_pts=600)
    i0 = 3
    R = s.cam_R[i0].reshape(3, 3)
    s.cam_R[i0] = (np.diag([-1.0, 1.0, -1.0]) @ R).ravel()
    gp, op, gst, n_o, sc_o, sc_g, w_g = _one_reweight(rp, s, False)
    assert sc_o[i0] == 0.0 and sc_g[i0] == 0.0
    assert np.abs(sc_g - sc_o).max() <= TOL * sc_o.max()
    assert np.array_equal(w_g, op.weights())
    assert np.all(w_g[s.obs_cam == i0] == 1.0)


@pytest.mark.parametrize("graph", [False, True])
def test_robust_schedule_parity(rp, graph):
    """Fixed robust schedule (re-weighting from the second outer iteration on,
    final elimination) vs the oracle."""
    from paper_1910_08138_amd import binding
    s = scenes.config_scene(4, 6, small=True)
    T, I = 4, 2
    gp, gh = binding.run_schedule(s, T=T, I=I, robust=True, t_r=1, graph=graph)
    op, oh = oracle.run_schedule(s, T=T, I=I, robust=True, t_r=1)
    for g, o in zip(gh, oh):
        assert np.allclose(g["int_stats"], o["int_stats"], rtol=TOL, atol=0), (g["t"], g["int_stats"], o["int_stats"])
    gR, gC = gp.cameras()
    oR, oC = op.cameras()
    ext = float(np.linalg.norm(s.cam_C_true.max(axis=1) - s.cam_C_true.min(axis=1))) + 1.0
    assert np.abs(gC - oC).max() <= TOL * ext
    _, _, gst = gp.intersection()
    _, _, ost = op.intersection()
    assert np.array_equal(gst, ost)
    assert (ost == 4).sum() > 0
