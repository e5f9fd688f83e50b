"""Pins of the serial robust variant in the oracle (Sec. 5.3): flagged
observations deleted, points left in one camera eliminated, and deleted
observations out of every later sum.

None of the expected values comes from the oracle's robust code:
  * deleting an observation must be the same as never having had it: the
    oracle run on the scene with the deleted observations (and the
    eliminated points) physically removed gives the same points,
    covariances, statistics and camera steps;
  * the deleted set is recomputed here with numpy from the definition
    (projection, whitening, per-camera MAD x 1.4826, threshold t_v);
  * the elimination rule is checked point by point from the weights.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_1910_08138_amd import scenes

TOL = 1e-9


def _with_gross_errors(seed=3, frac=0.03, n_pts=1500, views=(2, 8)):
    """Ring scene (20 cameras, 2 sub-blocks) with gross errors of 15-40 px on
    a fraction of the observations."""
    return scenes.add_gross_errors(scenes.ring_scene(seed, n_pts=n_pts, views=views), frac, seed)


def _converged(s):
    """The oracle after basic convergence (fixed schedule, no robust step),
    ending with an intersection."""
    op, _ = oracle.run_schedule(s, T=4, I=3)
    return op


def _removed(s, keep_obs, keep_pts, pts_start):
    """The scene with only the kept observations and points (renumbered)."""
    new_id = -np.ones(s.N, dtype=np.int64)
    new_id[keep_pts] = np.arange(keep_pts.size)
    k = keep_obs & (new_id[s.obs_pt] >= 0)
    return dataclasses.replace(
        s, pts=np.ascontiguousarray(pts_start[:, keep_pts]), pts_true=np.ascontiguousarray(s.pts_true[:, keep_pts]),
        obs_xy=np.ascontiguousarray(s.obs_xy[:, k]), obs_cam=np.ascontiguousarray(s.obs_cam[k]),
        obs_pt=np.ascontiguousarray(new_id[s.obs_pt[k]].astype(np.int32)), outlier=None), k


def _project(R9, C, X, cam, pt, f=1000.0, cx=500.0, cy=500.0):
    R = R9.reshape(-1, 3, 3)[cam]
    d = X[:, pt].T - C[:, cam].T
    p = np.einsum("nij,nj->ni", R, d)
    return np.stack([f * p[:, 0] / p[:, 2] + cx, f * p[:, 1] / p[:, 2] + cy])


def _flags_by_hand(s, op, t_v, live):
    """Normalised residuals and the per-camera MAD scale from the definition
    (unit a-priori weights 1/sigma^2), over the live observations of valid
    points: returns the boolean flag of every observation."""
    R, C = op.cameras()
    X, _, st = op.intersection()
    v = _project(R, C, X, s.obs_cam, s.obs_pt) - s.obs_xy
    z = v / s.sigma_px                       # whitened components
    use = live & (st[s.obs_pt] == 0)
    flag = np.zeros(s.K, dtype=bool)
    for i in range(s.M):
        m = use & (s.obs_cam == i)
        comp = z[:, m].ravel()
        if comp.size == 0:
            continue
        s0 = 1.4826 * np.median(np.abs(comp - np.median(comp)))
        vb = np.sqrt((z[:, m] ** 2).sum(0))
        flag[np.flatnonzero(m)[vb > t_v * s0]] = True
    return flag


def test_deleted_set_matches_the_definition_and_later_calls_keep_it():
    s = _with_gross_errors()
    op = _converged(s)
    expect = _flags_by_hand(s, op, 3.0, np.ones(s.K, dtype=bool))
    n, _ = op.robust_reweight(3.0, 1e-4, mode=oracle.ROBUST_DELETE_OBS)
    w = op.weights()
    assert n == int(expect.sum()) > 0
    assert np.array_equal(w == 0.0, expect)
    assert np.all(w[~expect] == 1.0)
    # a later down-weighting call: deleted observations stay at 0 and take no
    # part in the scales; new flags get 1e-4
    op.intersect()
    _, _, st = op.intersection()
    live = w != 0.0
    expect2 = _flags_by_hand(s, op, 3.0, live) & live
    n2, _ = op.robust_reweight(3.0, 1e-4, mode=oracle.ROBUST_WEIGHT)
    w2 = op.weights()
    assert np.all(w2[~live] == 0.0)
    assert n2 == int(expect2.sum())
    assert np.array_equal(w2 == 1e-4, expect2)
    assert np.all(w2[live & ~expect2] == 1.0)


def test_points_left_in_one_camera_are_eliminated():
    s = _with_gross_errors(seed=5, frac=0.06)
    op = _converged(s)
    _, _, st0 = op.intersection()
    op.robust_reweight(3.0, 1e-4, mode=oracle.ROBUST_DELETE_OBS)
    w = op.weights()
    _, _, st = op.intersection()
    live = np.bincount(s.obs_pt, weights=(w != 0).astype(float), minlength=s.N)
    flagged = np.bincount(s.obs_pt, weights=(w == 0).astype(float), minlength=s.N) > 0
    ok0 = st0 == 0
    expect_elim = ok0 & flagged & (live < 2)
    assert np.array_equal(st == 4, expect_elim)
    assert expect_elim.sum() > 0                       # the rule fired
    assert (ok0 & flagged & (live >= 2)).sum() > 0     # and points with deletions survived
    assert np.all(st[~expect_elim] == st0[~expect_elim])


def test_deleting_equals_removing():
    """After the serial robust step, the problem behaves as if the deleted
    observations and eliminated points had never been there: intersection
    (points, covariances, sigma0, RMS, valid count) and a fixed schedule
    (camera poses) agree with the oracle run on the reduced scene."""
    s = _with_gross_errors(seed=7)
    op = _converged(s)
    op.robust_reweight(3.0, 1e-4, mode=oracle.ROBUST_DELETE_OBS)
    w = op.weights()
    X0, _, st = op.intersection()
    keep_pts = np.flatnonzero(st == 0)
    R0, C0 = op.cameras()
    r, kmask = _removed(s, w != 0.0, keep_pts, X0)
    r = dataclasses.replace(r, cam_R=np.ascontiguousarray(R0), cam_C=np.ascontiguousarray(C0))
    assert r.K < s.K and r.N < s.N
    o2 = oracle.OracleProblem(r)
    sa = op.intersect()
    sb = o2.intersect()
    assert np.allclose(sa, sb, rtol=TOL, atol=0), (sa, sb)
    Xa, Ca, sta = op.intersection()
    Xb, Cb, stb = o2.intersection()
    assert np.array_equal(sta[keep_pts], stb)
    assert np.allclose(Xa[:, keep_pts], Xb, rtol=0, atol=TOL * 10)
    assert np.allclose(Ca[:, keep_pts], Cb, rtol=TOL, atol=TOL * np.abs(Cb).max())
    for t in range(2):
        for _ in range(2):
            ba, fa = op.lm_step()
            bb, fb = o2.lm_step()
            assert fa == fb == 0
            assert np.allclose(ba[:, :3], bb[:, :3], rtol=1e-8, atol=0)
        op.consensus()
        o2.consensus()
        sa, sb = op.intersect(), o2.intersect()
        assert np.allclose(sa, sb, rtol=1e-8, atol=0), (t, sa, sb)
    Ra, Ca_ = op.cameras()
    Rb, Cb_ = o2.cameras()
    assert np.abs(Ca_ - Cb_).max() <= 1e-8 * 5.0
    assert np.abs(Ra - Rb).max() <= 1e-8


def test_serial_cycle_on_one_block_removes_the_gross_errors():
    """The serial variant as the paper runs it (one block, t_v = 3): the full
    robust cycle removes almost every gross error and brings sigma0 back to
    the simulated noise (0.5 px).  On points without a gross error the
    deleted share is the Gaussian tail of the rule: a normalised 2-D residual
    beyond 3 has probability exp(-9/2) = 1.1%.  (Observations sharing a point
    with a gross error are deleted with it more often: with few views the
    error spreads over all of them.)"""
    s = _with_gross_errors(seed=11, frac=0.02)
    s1 = s.repartition(np.zeros(s.M, dtype=np.int32))
    plain, ph = oracle.run_ratio_rule(s1, T_max=8, I_max=6)
    op, hist = oracle.run_ratio_rule(s1, T_max=8, I_max=6, robust="serial")
    assert any(h.get("robust") for h in hist[:-1])
    w = op.weights()
    deleted = w == 0.0
    assert set(np.unique(w)) <= {0.0, 1.0}
    assert deleted[s.outlier].mean() > 0.95
    bad_pt = np.bincount(s.obs_pt, weights=s.outlier.astype(float), minlength=s.N) > 0
    clean = ~bad_pt[s.obs_pt]
    assert 0.005 < deleted[clean].mean() < 0.02
    sig_plain = ph[-1]["int_stats"][1]
    sig_rob = hist[-1]["int_stats"][1]
    assert sig_plain > 2.0 and abs(sig_rob - 0.5) < 0.05, (sig_plain, sig_rob)
