"""Pin of the oracle's covariances (Sec. 2: camera covariance M_CC = S^-1,
point covariance M_XX = N_XX^-1 + N_XX^-1 N_XC M_CC N_XC^T N_XX^-1, both
from the Schur complement) against the plain definition: the inverse of the
full normal matrix of the sub-block, assembled here with numpy from an
independent linearisation of the pinhole projection.

The test parametrises the rotation increment on the right, R exp([d]x),
where the oracle multiplies it on the left; the two are related by a fixed
invertible map per camera, which leaves the marginal covariances of the
camera centres and of the points unchanged (without damping).  Those are the
blocks compared."""
import numpy as np

import oracle
from paper_1910_08138_amd import scenes


def _skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def _full_normal(s, op, l):
    R9, C = op.cameras()
    blk, pt, Xc, om = op.copies()
    _, _, st = op.intersection()
    cams = np.flatnonzero(s.cam_block == l)
    cam_at = {c: a for a, c in enumerate(cams)}
    cps = [q for q in range(blk.size) if blk[q] == l and st[pt[q]] == 0]
    cp_at = {q: b for b, q in enumerate(cps)}
    nC, n = 6 * cams.size, 6 * cams.size + 3 * len(cps)
    N = np.zeros((n, n))
    w0 = 1.0 / s.sigma_px ** 2
    for k in range(s.K):
        i, j = int(s.obs_cam[k]), int(s.obs_pt[k])
        if s.cam_block[i] != l or st[j] != 0:
            continue
        q = next(q for q in cps if pt[q] == j)
        R = R9[i].reshape(3, 3)
        d = Xc[q] - C[:, i]
        p = R @ d
        Jp = s.f / p[2] * np.array([[1.0, 0.0, -p[0] / p[2]], [0.0, 1.0, -p[1] / p[2]]])
        J = np.zeros((2, n))
        a, b = cam_at[i], cp_at[q]
        J[:, 6 * a:6 * a + 3] = Jp @ (-R @ _skew(d))      # right-multiplied rotation increment
        J[:, 6 * a + 3:6 * a + 6] = Jp @ (-R)              # centre
        J[:, nC + 3 * b:nC + 3 * b + 3] = Jp @ R           # point copy
        N += w0 * J.T @ J
    for q in cps:
        o = om[q]
        b = cp_at[q]
        N[nC + 3 * b:nC + 3 * b + 3, nC + 3 * b:nC + 3 * b + 3] += np.array(
            [[o[0], o[1], o[2]], [o[1], o[3], o[4]], [o[2], o[4], o[5]]])
    return N, cams, cps, nC


def test_covariances_equal_the_inverse_of_the_full_normal_matrix():
    s = scenes.ring_scene(2, n_pts=300)
    op, _ = oracle.run_schedule(s, T=2, I=2)
    cc, xc = op.covariance(lam=0.0)
    for l in range(s.L):
        N, cams, cps, nC = _full_normal(s, op, l)
        M = np.linalg.inv(N)
        for a, i in enumerate(cams):
            ref = M[6 * a + 3:6 * a + 6, 6 * a + 3:6 * a + 6]
            assert np.allclose(cc[i][3:, 3:], ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max())
        for b, q in enumerate(cps):
            B = M[nC + 3 * b:nC + 3 * b + 3, nC + 3 * b:nC + 3 * b + 3]
            ref = B[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
            assert np.allclose(xc[q], ref, rtol=1e-7, atol=1e-9 * np.abs(ref).max())
    # the camera blocks are symmetric positive definite
    for i in range(s.M):
        assert np.allclose(cc[i], cc[i].T, rtol=0, atol=1e-12 * np.abs(cc[i]).max())
        assert np.all(np.linalg.eigvalsh(cc[i]) > 0)


def test_small_damping_barely_changes_the_covariances():
    """lambda = 1e-6 (the paper's setting for covariances) against no
    damping: the change is first order in lambda (lambda = 1e-4 moves the
    covariances about a hundred times more) and small, a few 1e-3 of the
    largest entry on this block."""
    s = scenes.ring_scene(2, n_pts=300)
    op, _ = oracle.run_schedule(s, T=2, I=2)
    c0, x0 = op.covariance(lam=0.0)
    c6, x6 = op.covariance(lam=1e-6)
    c4, x4 = op.covariance(lam=1e-4)
    d6 = np.abs(c6 - c0).max() / np.abs(c0).max()
    d4 = np.abs(c4 - c0).max() / np.abs(c0).max()
    assert d6 < 3e-3 and 50 * d6 < d4 < 200 * d6, (d6, d4)
    assert np.abs(x6 - x0).max() / np.abs(x0).max() < 3e-3
