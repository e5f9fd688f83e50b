"""Pins of oracle parts whose output has a plain definition that can be worked
out by hand: the consensus mean (eq:admm8 form), the robust MAD scale with an
even number of residual components (Sec. 5.3), the features of the learned
preconditioner, and the improvement test that ends a loop (Sec. 5.4).

Every expected value below is a literal worked out by hand from the
definition (the derivation is in the comment next to it); none comes from
running the oracle.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1910_08138_amd import scenes


def _tiny_scene(cam_block, obs):
    """Cameras on the x axis looking down +z, points in front of them; obs is
    a list of (camera, point) pairs."""
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


# --------------------------------------------------------------- consensus
def test_consensus_mean_spread_and_tie_point_count_by_hand():
    """Sec. 5 (eq:admm8 form): a point's next start value is the mean of its
    sub-block copies; stats = (largest distance of a copy from its mean,
    number of tie points)."""
    # cameras 0 and 3 in sub-block 0, camera 1 in 1, camera 2 in 2.
    # point 0: seen in sub-blocks 0, 1, 2 (three copies)
    # point 1: seen in sub-blocks 0, 1 (two copies)
    # point 2: seen by cameras 0 and 3 only (one copy, not a tie point)
    s = _tiny_scene([0, 1, 2, 0], [(0, 0), (1, 0), (2, 0), (0, 1), (1, 1), (0, 2), (3, 2)])
    op = oracle.OracleProblem(s)
    blk, pt, _, _ = op.copies()
    # copies are ordered by (sub-block, point)
    assert list(zip(blk, pt)) == [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (2, 0)]
    X = np.array([[1.0, 0.0, 0.0],      # point 0 in sub-block 0
                  [10.0, 10.0, 10.0],   # point 1 in sub-block 0
                  [5.0, 5.0, 5.0],      # point 2 (its only copy)
                  [0.0, 2.0, 0.0],      # point 0 in sub-block 1
                  [10.0, 10.0, 12.0],   # point 1 in sub-block 1
                  [0.0, 0.0, 3.0]])     # point 0 in sub-block 2
    op.set_copies(X)
    st = op.consensus()
    P = op.points()
    # point 0: ((1,0,0) + (0,2,0) + (0,0,3)) / 3 = (1/3, 2/3, 1)
    assert np.array_equal(P[:, 0], np.array([1.0, 2.0, 3.0]) / 3.0)
    # point 1: ((10,10,10) + (10,10,12)) / 2 = (10, 10, 11)
    assert np.array_equal(P[:, 1], np.array([10.0, 10.0, 11.0]))
    assert np.array_equal(P[:, 2], np.array([5.0, 5.0, 5.0]))
    # distances of point 0's copies from its mean: |(-1/3, 4/3, -1)| = sqrt(26)/3,
    # |(2/3, -2/3, -1)| = sqrt(17)/3, |(-1/3, -2/3, 2)| = sqrt(41)/3 (the largest);
    # point 1's copies are 1 away
    assert st[0] == pytest.approx(math.sqrt(41.0) / 3.0, rel=1e-15)
    assert st[1] == 2.0


# ------------------------------------------------------------------- MAD
def test_robust_mad_scale_even_counts_by_hand():
    """Sec. 5.3: sigma0_i = 1.4826 * median |c - median(c)| over the whitened
    residual components c of camera i (x and y separately); for an even count
    the median is the mean of the two middle values.  With W = I / 0.5^2 the
    whitened component is 2 v."""
    # sub-block 0: cameras 0, 1; sub-block 1: camera 2
    obs = [(0, 0), (1, 0), (2, 0), (0, 1), (2, 1), (1, 2), (2, 2)]
    s = _tiny_scene([0, 0, 1], obs)
    op = oracle.OracleProblem(s)
    res = np.zeros((2, s.K))
    v = {(0, 0): (0.1, -0.3), (0, 1): (0.5, 0.2),                      # camera 0
         (1, 0): (0.0, 0.0), (1, 2): (0.25, -0.25),                    # camera 1
         (2, 0): (0.5, 1.0), (2, 1): (1.5, -2.0), (2, 2): (-2.5, 3.0)}  # camera 2
    for k, key in enumerate(obs):
        res[:, k] = v[key]
    op.set_residuals(res)
    nflag, sc = op.robust_reweight(t_v=1.5, down_weight=1e-4)
    # camera 0: components 0.2, -0.6, 1.0, 0.4 -> sorted -0.6 0.2 0.4 1.0,
    #   median (0.2 + 0.4) / 2 = 0.3; |c - 0.3| = 0.9 0.1 0.7 0.1 -> sorted
    #   0.1 0.1 0.7 0.9, median 0.4 (an upper median would give 0.7, a lower 0.1)
    # camera 1: 0, 0, 0.5, -0.5 -> median 0; |c| = 0 0 0.5 0.5 -> median 0.25
    # camera 2: 1 2 3 -4 -5 6 -> sorted -5 -4 1 2 3 6, median 1.5;
    #   |c - 1.5| = 0.5 0.5 1.5 4.5 5.5 6.5 (sorted), median 3.0
    assert sc[0] == pytest.approx(1.4826 * 0.4, rel=1e-15)
    assert sc[1] == pytest.approx(1.4826 * 0.25, rel=1e-15)
    assert sc[2] == pytest.approx(1.4826 * 3.0, rel=1e-15)
    # flags: sqrt(v^T W v) / sigma0_i > 1.5
    #   camera 0: 2|(0.1,-0.3)| = 0.632 / 0.593 = 1.07 no; 2|(0.5,0.2)| = 1.077 / 0.593 = 1.82 yes
    #   camera 1: 0 no; 2|(0.25,-0.25)| = 0.707 / 0.371 = 1.91 yes
    #   camera 2: 2|(0.5,1)| = 2.236 / 4.448 = 0.50 no; 2|(1.5,-2)| = 5 / 4.448 = 1.12 no;
    #             2|(-2.5,3)| = 7.81 / 4.448 = 1.76 yes
    w = op.weights()
    expect = {(0, 1), (1, 2), (2, 2)}
    assert nflag == 3
    for k, key in enumerate(obs):
        assert w[k] == (1e-4 if key in expect else 1.0), key


# ------------------------------------------------------- network features
def test_learned_preconditioner_features_by_hand():
    """Features of camera block i of an RCS: log(S_qq / mean diagonal) (6),
    the 15 correlations S_rc / sqrt(S_rr S_cc) (r > c, row-major), log(1 +
    observations), log(1 + neighbouring blocks), sum_k |S_ik|_F / |S_ii|_F,
    log10(lambda), tie-point fraction."""
    S = np.zeros((18, 18))
    S[0:6, 0:6] = 4.0 * np.eye(6)
    S[0, 1] = S[1, 0] = 2.0            # correlation 2 / sqrt(4 * 4) = 0.5
    S[2, 5] = S[5, 2] = -1.0           # correlation -1 / 4 = -0.25
    S[6:12, 6:12] = np.eye(6)
    S[12:18, 12:18] = 2.0 * np.eye(6)  # camera 2 shares no point with 0 or 1
    S[0, 6] = S[6, 0] = 3.0            # block (0, 1): |.|_F = sqrt(9 + 16) = 5
    S[1, 7] = S[7, 1] = 4.0
    obs_tp = np.array([[10, 0.3], [7, 0.0], [4, 1.0]])
    f = oracle.mlp_features(S, obs_tp, lam=1e-4)
    assert f.shape == (3, 26)
    # mean diagonal (6*4 + 6*1 + 6*2) / 18 = 7/3
    assert np.allclose(f[0, :6], math.log(12.0 / 7.0), rtol=0, atol=1e-15)
    assert np.allclose(f[1, :6], math.log(3.0 / 7.0), rtol=0, atol=1e-15)
    assert np.allclose(f[2, :6], math.log(6.0 / 7.0), rtol=0, atol=1e-15)
    corr0 = np.zeros(15)
    corr0[0] = 0.5      # (1, 0) is the first strict-lower entry
    corr0[12] = -0.25   # (5, 2): rows 1..4 hold 1+2+3+4 = 10 entries, then (5,0) (5,1) (5,2)
    assert np.array_equal(f[0, 6:21], corr0)
    assert np.array_equal(f[1, 6:21], np.zeros(15))
    assert np.array_equal(f[2, 6:21], np.zeros(15))
    assert f[0, 21] == pytest.approx(math.log(11.0), rel=1e-15)
    assert f[1, 21] == pytest.approx(math.log(8.0), rel=1e-15)
    assert f[2, 21] == pytest.approx(math.log(5.0), rel=1e-15)
    assert f[0, 22] == pytest.approx(math.log(2.0), rel=1e-15)   # one neighbour
    assert f[1, 22] == pytest.approx(math.log(2.0), rel=1e-15)
    assert f[2, 22] == 0.0                                        # none
    # |S_00|_F = sqrt(6*16 + 2*4 + 2*1) = sqrt(106); |S_11|_F = sqrt(6)
    assert f[0, 23] == pytest.approx(5.0 / math.sqrt(106.0), rel=1e-15)
    assert f[1, 23] == pytest.approx(5.0 / math.sqrt(6.0), rel=1e-15)
    assert f[2, 23] == 0.0
    assert np.allclose(f[:, 24], -4.0, rtol=0, atol=1e-15)
    assert np.array_equal(f[:, 25], np.array([0.3, 0.0, 1.0]))


# ------------------------------------------------------- improvement test
@pytest.mark.parametrize("first,costs,steps", [
    # 100 -> 50 (ratio 2), 49.8 (50/49.8 = 1.004: first short step, tolerated),
    # 30 (49.8/30 = 1.66), 29.9 (30/29.9 = 1.003: second short step, stop)
    (100.0, [50.0, 49.8, 30.0, 29.9, 10.0], 4),
    # two short steps in a row: stop at the second
    (100.0, [99.5, 99.2, 50.0], 2),
    # a cost that rises counts as short (best 10 / 11 < 1.01) and best stays 10
    (10.0, [11.0, 9.0, 8.99, 1.0], 3),
    # always improving by more than 1 %: never stops within the list
    (100.0, [90.0, 80.0, 70.0], 3),
    # exactly 1.01 is not short (101 / 100 = 1.01)
    (101.0, [100.0, 99.0], 2),
])
def test_ratio_rule_hand_sequences(first, costs, steps):
    """Sec. 5.4: best-so-far / current below 1.01 is tolerated once, the
    second time the loop ends (with that step)."""
    r = oracle.RatioRule(first)
    taken = 0
    for c in costs:
        taken += 1
        if not r.step(c):
            break
    assert taken == steps
