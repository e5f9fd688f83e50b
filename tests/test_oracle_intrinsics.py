"""Pins of the oracle's intrinsics: every camera with its own focal length f
and first radial distortion parameter k1, estimated with its pose (Sec. 6,
the Final data sets: n (6 + 2) camera parameters).  The model (a reading:
the paper names the parameters, not the formula) distorts the normalised
image coordinates q = (p1/p3, p2/p3): pixel f (1 + k1 |q|^2) q + c.

  * the Jacobian of the projection against central differences of the
    simulator's own forward model (scenes.render_distorted), all eight camera
    columns and the point block;
  * with k1 = 0 the model is the shared pinhole, column for column;
  * noise-free aerial block: the schedule drives the residuals to zero and
    every camera's f and k1 to the values the scene was rendered with;
  * covariances with intrinsics equal the inverse of the full normal matrix
    of a sub-block, assembled with numpy from numerical derivatives.
"""
import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from paper_1910_08138_amd import scenes


def _camera(rng):
    R = Rotation.from_rotvec(rng.normal(scale=0.3, size=3)).as_matrix()
    C = rng.normal(size=3)
    # a point in front of the camera, off its axis
    p = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5), rng.uniform(3.0, 6.0)])
    X = C + R.T @ p
    return R, C, X


def _proj(R, C, X, f, k1):
    u, v = scenes.render_distorted(R[None], C[None], X[None], np.array([f]), np.array([k1]))
    return np.array([u[0], v[0]])


def test_jacobian_matches_central_differences():
    rng = np.random.default_rng(0)
    for trial in range(20):
        R, C, X = _camera(rng)
        f, k1 = rng.uniform(800, 1200), rng.uniform(-0.15, 0.15)
        g, A, B = oracle.linearise_cal(R.ravel(), C, X, f, k1, scenes.CX, scenes.CY)
        assert np.allclose(g, _proj(R, C, X, f, k1), rtol=1e-14, atol=1e-9)
        num = np.zeros((2, 8))
        for t in range(8):
            h = 1e-6 if t < 6 else (1e-4 if t == 6 else 1e-7)
            e = np.zeros(8)
            e[t] = h

            def at(dp):
                Rp = Rotation.from_rotvec(dp[:3]).as_matrix() @ R  # rotation increment on the left
                return _proj(Rp, C + dp[3:6], X, f + dp[6], k1 + dp[7])
            num[:, t] = (at(e) - at(-e)) / (2 * h)
        assert np.allclose(A, num, rtol=1e-6, atol=1e-6 * np.abs(num).max()), (trial, A, num)
        numB = np.zeros((2, 3))
        for t in range(3):
            e = np.zeros(3)
            e[t] = 1e-6
            numB[:, t] = (_proj(R, C, X + e, f, k1) - _proj(R, C, X - e, f, k1)) / 2e-6
        assert np.allclose(B, numB, rtol=1e-6, atol=1e-6 * np.abs(numB).max())


def test_zero_distortion_is_the_pinhole():
    rng = np.random.default_rng(1)
    for trial in range(10):
        R, C, X = _camera(rng)
        f = rng.uniform(800, 1200)
        g1, A1, B1 = oracle.linearise_cal(R.ravel(), C, X, f, 0.0, scenes.CX, scenes.CY)
        g0, A0, B0 = oracle.linearise(R.ravel(), C, X, f, scenes.CX, scenes.CY)
        assert np.allclose(g1, g0, rtol=1e-15, atol=0)
        assert np.allclose(A1[:, :6], A0, rtol=1e-13, atol=1e-13 * np.abs(A0).max())
        assert np.allclose(B1, B0, rtol=1e-13, atol=1e-13 * np.abs(B0).max())
        # dg/df = q = (g - c) / f
        assert np.allclose(A1[:, 6], (g0 - [scenes.CX, scenes.CY]) / f, rtol=1e-13)


def _noise_free_oblique(n_blocks):
    base = scenes.oblique_scene(3, n_strips=2, n_stations=6, n_pts=3000, n_blocks=n_blocks, size_range=(10, 60),
                                noise=0.0)
    return scenes.with_intrinsics(base, 3)


def test_noise_free_block_recovers_focal_lengths_and_distortions():
    """One sub-block of 60 oblique cameras, noise-free: Gauss-Newton (a tiny
    damping; f and the distance along the optical axis are nearly
    interchangeable, which a damping of 1e-4 would slow to a crawl) reaches
    zero residuals and the rendered f and k1 of every camera."""
    s = _noise_free_oblique(1)
    # the start is off: f by about 0.5%, k1 by up to 0.1
    assert np.abs(s.cam_f - s.cam_f_true).max() > 1.0 and np.abs(s.cam_k1_true).max() > 0.05
    op, hist = oracle.run_schedule(s, T=3, I=6, lam=1e-10)
    assert op.np == 8
    assert hist[-1]["int_stats"][2] < 1e-10, hist[-1]["int_stats"]
    f, k1 = op.intrinsics()
    assert np.abs(f - s.cam_f_true).max() < 1e-8 * scenes.F_PX, np.abs(f - s.cam_f_true).max()
    assert np.abs(k1 - s.cam_k1_true).max() < 1e-10, np.abs(k1 - s.cam_k1_true).max()


def test_two_sub_blocks_approach_the_rendered_intrinsics():
    """The same block in two sub-blocks (12 and 48 cameras): the alternation
    of sub-block steps and intersections moves every f and k1 towards the
    rendered values, linearly (about 0.9 per outer iteration here)."""
    s = _noise_free_oblique(2)
    err = []

    def cb(op, rec):
        f, k1 = op.intrinsics()
        err.append((rec["int_stats"][2], np.abs(f - s.cam_f_true).max(), np.abs(k1 - s.cam_k1_true).max()))
    oracle.run_schedule(s, T=30, I=5, lam=1e-10, callback=cb)
    e = np.array(err)
    assert np.all(np.diff(e[1:, 0]) < 0)                      # RMS falls every outer iteration
    assert e[-1, 0] < 0.01 * e[1, 0] and e[-1, 1] < 0.2 * e[5, 1] and e[-1, 2] < 0.2 * e[5, 2], e[[1, 5, -1]]


def _full_normal_numeric(s, op, l):
    """Normal matrix of sub-block l with the tie-point weights, cameras
    parametrised by (right rotation increment, centre, f, k1), from central
    differences of the simulator's forward model."""
    R9, C = op.cameras()
    f, k1 = op.intrinsics()
    blk, pt, Xc, om = op.copies()
    _, _, st = op.intersection()
    cams = np.flatnonzero(s.cam_block == l)
    cam_at = {c: a for a, c in enumerate(cams)}
    cps = [q for q in range(blk.size) if blk[q] == l and st[pt[q]] == 0]
    cp_of = {int(pt[q]): q for q in cps}
    cp_at = {q: b for b, q in enumerate(cps)}
    nC, n = 8 * cams.size, 8 * cams.size + 3 * len(cps)
    N = np.zeros((n, n))
    w0 = 1.0 / s.sigma_px ** 2
    for k in range(s.K):
        i, j = int(s.obs_cam[k]), int(s.obs_pt[k])
        if s.cam_block[i] != l or st[j] != 0:
            continue
        q = cp_of[j]
        R = R9[i].reshape(3, 3)
        J = np.zeros((2, n))
        a, b = cam_at[i], cp_at[q]

        def pr(dp, dx):
            Rp = R @ Rotation.from_rotvec(dp[:3]).as_matrix()
            return _proj(Rp, C[:, i] + dp[3:6], Xc[q] + dx, f[i] + dp[6], k1[i] + dp[7])
        for t in range(8):
            h = [1e-6] * 6 + [1e-3, 1e-7]
            e = np.zeros(8)
            e[t] = h[t]
            J[:, 8 * a + t] = (pr(e, 0) - pr(-e, 0)) / (2 * h[t])
        for t in range(3):
            e = np.zeros(3)
            e[t] = 1e-5
            J[:, nC + 3 * b + t] = (pr(np.zeros(8), e) - pr(np.zeros(8), -e)) / 2e-5
        N += w0 * J.T @ J
    for q in cps:
        o = om[q]
        b = cp_at[q]
        N[nC + 3 * b:nC + 3 * b + 3, nC + 3 * b:nC + 3 * b + 3] += np.array(
            [[o[0], o[1], o[2]], [o[1], o[3], o[4]], [o[2], o[4], o[5]]])
    return N, cams, cps, nC


def test_covariances_with_intrinsics_equal_the_inverse_of_the_full_normal_matrix():
    """The marginal covariances of the centre, f and k1 of each camera, and
    of every point copy, do not depend on how the rotation increment is
    parametrised (left in the oracle, right here)."""
    s = scenes.with_intrinsics(scenes.aerial_scene(4, nx=5, ny=5, n_pts=600, n_blocks=2), 4)
    op, _ = oracle.run_schedule(s, T=2, I=2)
    cc, xc = op.covariance(lam=0.0)
    assert cc.shape == (s.M, 8, 8)
    for l in range(s.L):
        N, cams, cps, nC = _full_normal_numeric(s, op, l)
        M = np.linalg.inv(N)
        for a, i in enumerate(cams):
            ref = M[8 * a + 3:8 * a + 8, 8 * a + 3:8 * a + 8]
            got = cc[i][3:, 3:]
            assert np.allclose(got, ref, rtol=1e-4, atol=1e-6 * np.abs(np.diag(ref)).max()), (i, got, ref)
        for b, q in enumerate(cps):
            B = M[nC + 3 * b:nC + 3 * b + 3, nC + 3 * b:nC + 3 * b + 3]
            ref = B[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
            assert np.allclose(xc[q], ref, rtol=1e-4, atol=1e-6 * np.abs(ref).max())
