"""Pins of the oracle's variants of the method (Sec. 4: plain ADMM consensus,
eq:admm7 to eq:admm9; Sec. 6.3: the growing scalar weight and the filters;
Sec. 6.4: tie-point weights from all cameras or a scalar) against facts that
do not come from the oracle: the point information of the covariance, dual
offsets worked out from hand-placed copies, a dense normal-equation solve
with the plain prior, scipy's least-squares optimum, and hand-placed
observations for the filter."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
from paper_1910_08138_amd import scenes


def _full(o):
    return np.array([[o[0], o[1], o[2]], [o[1], o[3], o[4]], [o[2], o[4], o[5]]])


def _four_blocks(seed):
    s = scenes.ring_scene(seed)
    s.cam_block = (np.arange(20) // 5).astype(np.int32)
    return s


@pytest.mark.parametrize("variant,factor", [(oracle.V_EXTENDED, -1), (oracle.V_ALL_CAMERAS, 0)])
def test_tie_point_weights_sum_to_the_point_information(variant, factor):
    """Sec. 5.1 / Sec. 6.4: summed over the c copies of a tie point, the
    weights are (c - 1) H for the outside cameras and c H for all cameras,
    with H the inverse of the intersection covariance; zero for a point in
    one sub-block."""
    s = _four_blocks(31)
    op = oracle.OracleProblem(s, variant=variant)
    op.intersect()
    X, cov, st = op.intersection()
    blk, pt, _, om = op.copies()
    ncopy = np.bincount(pt, minlength=s.N)
    acc = np.zeros((s.N, 3, 3))
    for q in range(len(pt)):
        acc[pt[q]] += _full(om[q])
    checked = 0
    for j in range(0, s.N, 5):
        if ncopy[j] == 1:
            assert np.abs(acc[j]).max() == 0.0
            continue
        H = np.linalg.inv(_full(cov[:, j]))
        assert np.abs(acc[j] - (ncopy[j] + factor) * H).max() <= 1e-9 * np.abs(H).max()
        checked += 1
    assert checked > 100


def test_scalar_weight_grows_per_outer_iteration():
    """Sec. 6.3-6.4: scalar tie-point weight rho_t I with rho_t = rho 1.01^t
    after t consensus exchanges (rho = 200: 200, 202, 204.02)."""
    s = _four_blocks(32)
    op = oracle.OracleProblem(s, variant=oracle.V_SCALAR, rho=200.0)
    for t, rho_t in enumerate([200.0, 202.0, 204.02]):
        op.intersect()
        blk, pt, _, om = op.copies()
        ncopy = np.bincount(pt, minlength=s.N)
        tp = ncopy[pt] > 1
        assert np.allclose(om[tp], np.array([rho_t, 0, 0, rho_t, 0, rho_t]), rtol=1e-14, atol=0)
        assert np.all(om[~tp] == 0.0)
        op.lm_step()
        op.consensus()


def _tiny(cam_block, obs):
    M = len(cam_block)
    obs_cam = np.array([c for c, _ in obs], dtype=np.int32)
    obs_pt = np.array([p for _, p in obs], dtype=np.int32)
    N = int(obs_pt.max()) + 1
    R = np.tile(np.eye(3), (M, 1, 1))
    C = np.stack([np.array([0.5 * i, 0.0, 0.0]) for i in range(M)])
    X = np.stack([np.array([0.3 * j, 0.1, 5.0]) for j in range(N)])
    u, v, _ = scenes.render(R[obs_cam], C[obs_cam], X[obs_pt])
    return scenes.Scene(name="tiny", seed=0, f=1000.0, cx=500.0, cy=500.0, sigma_px=0.5,
                        cam_R=R.reshape(M, 9).copy(), cam_C=C.T.copy(), pts=X.T.copy(),
                        obs_xy=np.stack([u, v]), obs_cam=obs_cam, obs_pt=obs_pt,
                        cam_block=np.asarray(cam_block, dtype=np.int32), cam_R_true=R.reshape(M, 9).copy(),
                        cam_C_true=C.T.copy(), pts_true=X.T.copy())


def test_plain_dual_update_by_hand():
    """eq:admm8-eq:admm9 on hand-placed copies: X_j is the mean of the copies
    and Xtilde_j^l accumulates X_j^l - X_j over the exchanges."""
    s = _tiny([0, 1, 2], [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1)])
    op = oracle.OracleProblem(s, variant=oracle.V_PLAIN)
    blk, pt, _, _ = op.copies()
    assert list(zip(blk, pt)) == [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)]
    X1 = np.array([[3.0, 0, 0], [1.0, 1, 1], [0, 3.0, 0], [1.0, 1, 3], [0, 0, 3.0]])
    op.set_copies(X1)
    op.consensus()
    # means: point 0 (1, 1, 1), point 1 (1, 1, 2)
    assert np.array_equal(op.points()[:, 0], [1.0, 1.0, 1.0])
    assert np.array_equal(op.points()[:, 1], [1.0, 1.0, 2.0])
    Xt1 = np.array([[2.0, -1, -1], [0, 0, -1.0], [-1.0, 2, -1], [0, 0, 1.0], [-1.0, -1, 2]])
    assert np.array_equal(op.duals(), Xt1)
    X2 = np.array([[2.0, 2, 2], [0, 0, 0], [2.0, 2, 2], [2.0, 2, 2], [2.0, 2, 5]])
    op.set_copies(X2)
    op.consensus()
    # means: point 0 (2, 2, 3), point 1 (1, 1, 1); the duals add X2 - mean
    Xt2 = Xt1 + np.array([[0.0, 0, -1], [-1.0, -1, -1], [0, 0, -1.0], [1.0, 1, 1], [0, 0, 2.0]])
    assert np.array_equal(op.duals(), Xt2)


def test_plain_evaluation_keeps_points_and_filters():
    """The plain variants do not intersect: rpba_intersect's counterpart only
    evaluates at the consensus point.  Filter of Sec. 6.3: a point with a
    reprojection error above filter_px is dropped (here one observation moved
    by 1,500 px); the extended method has no such filter (it tries to
    intersect the point, which then fails to converge)."""
    s = scenes.ring_scene(33, n_pts=300)
    k = int(np.nonzero(s.obs_pt == 7)[0][0])
    s.obs_xy = s.obs_xy.copy()
    s.obs_xy[0, k] += 1500.0
    op = oracle.OracleProblem(s, variant=oracle.V_PLAIN)
    op.intersect()
    X, cov, st = op.intersection()
    ok = st == 0
    assert np.array_equal(X[:, ok], s.pts[:, ok])          # evaluated where they start
    assert st[7] == oracle.ST_FILTERED and ok.sum() == s.N - 1
    oe = oracle.OracleProblem(s)
    oe.intersect()
    _, _, ste = oe.intersection()
    assert ste[7] in (oracle.ST_OK, oracle.ST_NOT_CONVERGED)


def test_plain_step_equals_dense_solve_with_the_admm_prior():
    """eq:admm7: the plain LM step of a sub-block (Schur complement, Cholesky,
    back-substitution) equals numpy's dense solve of the damped normal
    equations whose tie-point prior is rho_t |X^l - (X_j - Xtilde_j^l)|^2."""
    s = scenes.ring_scene(34, n_pts=150)
    s.cam_block = (np.arange(20) // 5).astype(np.int32)
    s.pts = s.pts_true + np.random.default_rng(0).normal(size=s.pts.shape) * 0.01
    op = oracle.OracleProblem(s, variant=oracle.V_PLAIN, rho=500.0)
    op.intersect()
    op.lm_step()
    op.consensus()                 # non-zero duals, rho_t = 505
    op.intersect()
    R = s.cam_R.reshape(-1, 3, 3)
    Rc, Cc = op.cameras()
    R = Rc.reshape(-1, 3, 3)
    C = Cc.T
    blk, pt, Xc, om = op.copies()
    Xm = op.points()
    Xt = op.duals()
    ncopy = np.bincount(pt, minlength=s.N)
    w = 1.0 / s.sigma_px ** 2
    lam = 1e-4
    for l in range(4):
        cams = np.nonzero(s.cam_block == l)[0]
        loc = {int(i): a for a, i in enumerate(cams)}
        qs = np.nonzero(blk == l)[0]
        n6, n3 = 6 * len(cams), 3 * len(qs)
        Nm = np.zeros((n6 + n3, n6 + n3))
        g = np.zeros(n6 + n3)
        for r, q in enumerate(qs):
            j = pt[q]
            for k in np.nonzero((s.obs_pt == j) & (s.cam_block[s.obs_cam] == l))[0]:
                i = s.obs_cam[k]
                gk, A, B = oracle.linearise(R[i].ravel(), C[i], Xc[q])
                idx = np.r_[6 * loc[i]:6 * loc[i] + 6, n6 + 3 * r:n6 + 3 * r + 3]   # the row's nonzero columns
                J = np.concatenate([A, B], axis=1)
                v = gk - s.obs_xy[:, k]
                Nm[np.ix_(idx, idx)] += w * J.T @ J
                g[idx] += w * J.T @ v
            if ncopy[j] > 1:
                rho_t = 505.0
                assert np.allclose(_full(om[q]), rho_t * np.eye(3), rtol=1e-14, atol=0)
                Nm[n6 + 3 * r:n6 + 3 * r + 3, n6 + 3 * r:n6 + 3 * r + 3] += rho_t * np.eye(3)
                g[n6 + 3 * r:n6 + 3 * r + 3] += rho_t * (Xc[q] - (Xm[:, j] - Xt[q]))
        Nm[np.diag_indices_from(Nm)] *= 1 + lam
        d = np.linalg.solve(Nm, -g)
        dC, dX = op.block_step(l, n6, len(qs))
        assert np.abs(dC - d[:n6]).max() <= 1e-9 * np.abs(d[:n6]).max()
        assert np.abs(dX.ravel() - d[n6:]).max() <= 1e-9 * np.abs(d[n6:]).max()


def test_plain_single_subblock_reaches_least_squares_optimum():
    """With one sub-block there is no tie point: the plain variant is LM
    bundle adjustment on cameras and points together (no re-intersection);
    its RMS reaches the optimum of scipy.optimize.least_squares."""
    from scipy.optimize import least_squares
    from scipy.sparse import lil_matrix

    s = scenes.ring_scene(35, n_pts=300, n_blocks=1)
    op, hist = oracle.run_schedule(s, T=12, I=4, variant=oracle.V_PLAIN)
    rms_plain = hist[-1]["int_stats"][2]
    M, N, K = s.M, s.N, s.K
    R0 = s.cam_R.reshape(M, 3, 3)

    def resid(x):
        Rm = Rotation.from_rotvec(x[:3 * M].reshape(M, 3)).as_matrix() @ R0
        Cc = x[3 * M:6 * M].reshape(M, 3)
        Xp = x[6 * M:].reshape(N, 3)
        u, v, _ = scenes.render(Rm[s.obs_cam], Cc[s.obs_cam], Xp[s.obs_pt])
        return np.concatenate([u - s.obs_xy[0], v - s.obs_xy[1]])

    sp = lil_matrix((2 * K, 6 * M + 3 * N), dtype=int)
    for k in range(K):
        i, j = s.obs_cam[k], s.obs_pt[k]
        for row in (k, K + k):
            sp[row, 3 * i:3 * i + 3] = 1
            sp[row, 3 * M + 3 * i:3 * M + 3 * i + 3] = 1
            sp[row, 6 * M + 3 * j:6 * M + 3 * j + 3] = 1
    x0 = np.concatenate([np.zeros(3 * M), s.cam_C.T.ravel(), s.pts_true.T.ravel()])
    res = least_squares(resid, x0, jac_sparsity=sp, method="trf", x_scale="jac", xtol=1e-15,
                        ftol=1e-15, gtol=1e-15, max_nfev=200)
    rms_ls = math.sqrt(np.mean(res.fun ** 2))
    assert abs(rms_plain - rms_ls) <= 1e-8 * rms_ls, (rms_plain, rms_ls)


def test_plain_refined_weights_at_the_mean_point():
    """Plain consensus with the weights of Sec. 5.1: Omega^l is evaluated at
    the consensus point (not moved), so summed over the copies of a tie point
    it is (c - 1) times the information there."""
    s = _four_blocks(36)
    op = oracle.OracleProblem(s, variant=oracle.V_PLAIN_REFINED)
    op.intersect()
    X, cov, st = op.intersection()
    assert np.array_equal(X[:, st == 0], s.pts[:, st == 0])
    blk, pt, _, om = op.copies()
    ncopy = np.bincount(pt, minlength=s.N)
    acc = np.zeros((s.N, 3, 3))
    for q in range(len(pt)):
        acc[pt[q]] += _full(om[q])
    for j in range(0, s.N, 11):
        if ncopy[j] > 1 and st[j] == 0:
            H = np.linalg.inv(_full(cov[:, j]))
            assert np.abs(acc[j] - (ncopy[j] - 1) * H).max() <= 1e-9 * np.abs(H).max()
