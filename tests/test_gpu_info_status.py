"""GPU vs the FP64 oracle with a 2x2 information matrix per observation
(W_k = C_xk^-1, paper Sec. 2), and the failure statuses of the boundary:
point statuses forced from the inputs, the step status of the LM step, and
the input checks of rpba_create.

FP64 bar: 1e-9 relative per result, as on the isotropic path."""
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


def _info(K, seed):
    """Seeded SPD information matrices: W = R diag(1/s1^2, 1/s2^2) R^T with
    s1, s2 ~ U[0.3, 0.8] px and R a rotation by an angle ~ U[0, pi)."""
    rng = np.random.default_rng(seed)
    s1 = rng.uniform(0.3, 0.8, K)
    s2 = rng.uniform(0.3, 0.8, K)
    th = rng.uniform(0.0, np.pi, K)
    c, sn = np.cos(th), np.sin(th)
    a = c * c / s1 ** 2 + sn * sn / s2 ** 2
    b = c * sn * (1.0 / s1 ** 2 - 1.0 / s2 ** 2)
    d = sn * sn / s1 ** 2 + c * c / s2 ** 2
    return np.stack([a, b, d])


def _sym(c):
    return np.array([[c[0], c[1], c[2]], [c[1], c[3], c[4]], [c[2], c[4], c[5]]])


def _extent(scene):
    C = scene.cam_C_true
    return float(np.linalg.norm(C.max(axis=1) - C.min(axis=1))) + 1.0


def _scene(name, seed):
    if name == "ring":
        return scenes.config_scene(1, seed)
    if name == "aerial-small":
        return scenes.config_scene(2, seed, small=True)
    return scenes.config_scene(4, seed, small=True)


@pytest.mark.parametrize("name", ["ring", "aerial-small"])
def test_info_intersection_and_rcs_parity(rp, name):
    """eq:bars and the RCS with per-observation weights: points, covariances,
    refined weights Omega of every copy, S and e of every sub-block."""
    s = _scene(name, 21)
    W = _info(s.K, 21)
    gp = rp.Problem(s, obs_info=W)
    op = oracle.OracleProblem(s, obs_info=W)
    gst = gp.rpba_intersect()
    gp.sync()
    gst = gst.cpu().numpy()
    ost = op.intersect()
    assert np.allclose(gst, ost, rtol=TOL, atol=0), (gst, ost)
    gX, gcov, gstat = gp.intersection()
    oX, ocov, ostat = op.intersection()
    assert np.array_equal(gstat, ostat)
    ok = ostat == 0
    assert np.abs(gX[:, ok] - oX[:, ok]).max() <= TOL * _extent(s)
    rel = np.linalg.norm(gcov[:, ok] - ocov[:, ok], axis=0) / np.linalg.norm(ocov[:, ok], axis=0)
    print(f"{name}: covariance max rel err {rel.max():.2e}")
    assert rel.max() <= TOL
    gb, gpt, gXc, gom = gp.copies()
    ob, opt_, oXc, oom = op.copies()
    o1, o2 = np.lexsort((gpt, gb)), np.lexsort((opt_, ob))
    assert np.array_equal(gb[o1], ob[o2]) and np.array_equal(gpt[o1], opt_[o2])
    assert np.abs(gom[o1] - oom[o2]).max() <= TOL * np.abs(oom).max()
    gp.rpba_subblock_lm_step()
    op.lm_step()
    for l in range(s.L):
        Sg, eg = gp.block_rcs(l)
        So, eo = op.block_rcs(l, Sg.shape[0])
        assert np.abs(np.tril(Sg) - np.tril(So)).max() <= TOL * np.abs(So).max(), l
        assert np.abs(eg - eo).max() <= TOL * np.abs(eo).max(), l


@pytest.mark.parametrize("name,robust", [("ring", False), ("oblique-robust-small", True)])
def test_info_fixed_schedule_parity(rp, name, robust):
    """Whole fixed schedule with per-observation weights (and the robust
    re-weighting, which whitens with the Cholesky factor of W), FP64."""
    s = _scene(name, 22)
    W = _info(s.K, 22)
    T, I = (4, 3) if not robust else (4, 2)
    gp, gh = rp.run_schedule(s, T=T, I=I, robust=robust, t_r=1, obs_info=W, graph=True)
    op, oh = oracle.run_schedule(s, T=T, I=I, robust=robust, t_r=1, obs_info=W)
    for g, o in zip(gh, oh):
        assert np.allclose(g["int_stats"], o["int_stats"], rtol=TOL, atol=0), (g["t"], g["int_stats"], o["int_stats"])
        for bg, (bo, fails) in zip(g.get("steps", []), o.get("steps", [])):
            assert fails == 0
            assert np.allclose(bg[:, :2], bo[:, :2], rtol=TOL, atol=0)
    if robust:
        _, wg = gp.robust_result()
        assert np.array_equal(wg, op.weights())
        assert (wg < 1).sum() > 0
    _, gC = gp.cameras()
    _, oC = op.cameras()
    assert np.abs(gC - oC).max() <= TOL * _extent(s)
    _, _, gst = gp.intersection()
    _, _, ost = op.intersection()
    assert np.array_equal(gst, ost)


def _two_view_scene(baseline, start_z, n_pts=3):
    """Two parallel cameras (one per sub-block), points midway at depth 5."""
    R = np.stack([np.eye(3), np.eye(3)])
    C = np.array([[0.0, 0.0, 0.0], [baseline, 0.0, 0.0]])
    X = np.stack([np.array([baseline / 2 + 0.1 * j, 0.05 * j, 5.0]) for j in range(n_pts)])
    obs_pt = np.repeat(np.arange(n_pts), 2)
    obs_cam = np.tile(np.array([0, 1]), n_pts)
    u, v, _ = scenes.render(R[obs_cam], C[obs_cam], X[obs_pt])
    X0 = X.copy()
    X0[:, 2] = start_z
    X0[:, 0] += 0.3
    return scenes.Scene(name="two-view", seed=0, f=1000.0, cx=500.0, cy=500.0, sigma_px=0.5,
                        cam_R=R.reshape(2, 9).copy(), cam_C=C.T.copy(), pts=X0.T.copy(), obs_xy=np.stack([u, v]),
                        obs_cam=obs_cam.astype(np.int32), obs_pt=obs_pt.astype(np.int32),
                        cam_block=np.array([0, 1], dtype=np.int32), cam_R_true=R.reshape(2, 9).copy(),
                        cam_C_true=C.T.copy(), pts_true=X.T.copy())


@pytest.mark.parametrize("case,kw,status", [
    ("ill", dict(baseline=1e-9, start_z=5.0), oracle.ST_ILL),            # depth unobservable
    ("behind", dict(baseline=1.0, start_z=-5.0), oracle.ST_BEHIND),      # start behind both cameras
    ("not-converged", dict(baseline=1.0, start_z=7.0), oracle.ST_NOT_CONVERGED),
])
def test_point_statuses_forced_from_inputs(rp, case, kw, status):
    """Sec. 5.4: points whose intersection fails get a status and weight zero.
    NOT_CONVERGED is forced with one Gauss-Newton iteration from a start 2 m
    off; the statuses must agree exactly with the oracle's."""
    s = _two_view_scene(**kw)
    maxit = 1 if case == "not-converged" else 20
    gp = rp.Problem(s, int_maxit=maxit)
    op = oracle.OracleProblem(s, int_maxit=maxit)
    gst = gp.rpba_intersect()
    gp.sync()
    gst = gst.cpu().numpy()
    ost = op.intersect()
    _, _, gstat = gp.intersection()
    _, _, ostat = op.intersection()
    assert np.array_equal(gstat, ostat)
    assert (ostat == status).all(), ostat
    assert gst[3] == ost[3] == 0.0        # no valid point


def test_step_status_ok_and_nonconverged_forced(rp):
    """rpba_step_status: OK after a normal step; WARN_NONCONVERGED when the
    iterative solve is cut to one CG iteration and one refinement sweep
    (forced from the host options), with the step still applied."""
    s = scenes.config_scene(2, 5, small=True)
    gp = rp.Problem(s)
    gp.rpba_intersect()
    gp.rpba_subblock_lm_step()
    rc, nspd, nnc = gp.step_status()
    assert (rc, nspd, nnc) == (rp.RPBA_OK, 0, 0)
    gq = rp.Problem(s, precision=rp.RPBA_MIXED, solver=rp.RPBA_SOLVER_PCG_BJ, pcg_maxit=1, ir_maxit=1)
    gq.rpba_intersect()
    bs = gq.rpba_subblock_lm_step()
    rc, nspd, nnc = gq.step_status()
    bs = bs.cpu().numpy()
    assert rc == rp.RPBA_WARN_NONCONVERGED and nspd == 0 and nnc == s.L
    assert np.all(bs[:, 3] == 1) and np.all(bs[:, 2] > 0)     # one iteration each, step applied


def test_create_rejects_non_finite_and_indefinite_inputs(rp):
    """rpba_create: non-finite state / observations and information matrices
    that are not positive definite are reported as RPBA_ERR_ARG."""
    s = scenes.config_scene(1, 0)
    bad = scenes.Scene(**{k: getattr(s, k) for k in s.__dataclass_fields__})
    bad.pts = s.pts.copy()
    bad.pts[1, 17] = np.nan
    with pytest.raises(rp.RpbaError, match="1 non-finite"):
        rp.Problem(bad)
    bad.pts = s.pts.copy()
    bad.obs_xy = s.obs_xy.copy()
    bad.obs_xy[0, 3] = np.inf
    with pytest.raises(rp.RpbaError, match="1 non-finite"):
        rp.Problem(bad)
    W = _info(s.K, 1)
    W[1, 5] = 10.0 * np.sqrt(W[0, 5] * W[2, 5])     # |w12| > sqrt(w11 w22): indefinite
    with pytest.raises(rp.RpbaError, match="1 obs_info matrices not positive definite"):
        rp.Problem(s, obs_info=W)
    rp.Problem(s, obs_info=_info(s.K, 1)).close()   # a valid problem still builds
