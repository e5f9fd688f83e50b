"""Adaptive damping in the oracle (the alternative to a fixed lambda that
Sec. 5.4 and 7 name): one lambda per sub-block, a step that raises the
sub-block's cost is taken back and lambda multiplied by 10, an accepted step
divides it by 10.

Checked from the definition: a taken-back step leaves the cameras and copies
exactly as they were; lambda follows the rule given the sequence of
decisions; the kept costs never rise; with the fixed mode nothing changes."""
import numpy as np

import oracle
from damping_scene import far_start_ring


def _state(op):
    R, C = op.cameras()
    _, _, X, _ = op.copies()
    return R.copy(), C.copy(), X.copy()


def test_rule_and_exact_take_back():
    s = far_start_ring()
    op = oracle.OracleProblem(s, lam=1e-6)
    op.set_damping(1)
    lam = np.full(s.L, 1e-6)
    blk, _, _, _ = op.copies()
    n_rej = n_acc = 0
    for t in range(2):
        op.intersect()
        for i in range(4):
            R0, C0, X0 = _state(op)
            bs, fails = op.lm_step()
            assert fails == 0
            got_lam, rej = op.damping()
            R1, C1, X1 = _state(op)
            for l in range(s.L):
                cams = s.cam_block == l
                if rej[l]:
                    n_rej += 1
                    assert bs[l, 1] == bs[l, 0] and bs[l, 2] == 0.0
                    assert np.array_equal(R1[cams], R0[cams]) and np.array_equal(C1[:, cams], C0[:, cams])
                    assert np.array_equal(X1[blk == l], X0[blk == l])
                    lam[l] = min(lam[l] * 10.0, 1e8)
                else:
                    n_acc += 1
                    assert bs[l, 1] <= bs[l, 0]
                    lam[l] = max(lam[l] / 10.0, 1e-12)
            assert np.array_equal(got_lam, lam)
        op.consensus()
    assert n_rej > 0 and n_acc > 0


def test_fixed_mode_is_unchanged():
    s = far_start_ring()
    a = oracle.OracleProblem(s, lam=1e-4)
    b = oracle.OracleProblem(s, lam=1e-4)
    b.set_damping(0)
    for op in (a, b):
        op.intersect()
    for i in range(3):
        ba, _ = a.lm_step()
        bb, _ = b.lm_step()
        assert np.array_equal(ba, bb)
    lam, rej = b.damping()
    assert np.all(lam == 1e-4) and not rej.any()


def test_adaptive_damping_reaches_a_lower_cost_than_a_tiny_fixed_lambda():
    """From the far start, plain steps with lambda = 1e-10 overshoot; the
    adaptive schedule keeps only steps that lower each sub-block's cost."""
    s = far_start_ring()
    fixed = oracle.OracleProblem(s, lam=1e-10)
    adapt = oracle.OracleProblem(s, lam=1e-10)
    adapt.set_damping(1)
    for op in (fixed, adapt):
        for t in range(3):
            op.intersect()
            for i in range(4):
                op.lm_step()
            op.consensus()
    sf = fixed.intersect()
    sa = adapt.intersect()
    assert sa[0] < sf[0]
