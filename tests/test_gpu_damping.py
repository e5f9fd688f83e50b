"""Adaptive damping on the GPU (per sub-block lambda, steps that raise the
cost taken back) against the oracle: the decisions and lambdas exactly, the
block statistics at 1e-9 and the poses at 1e-9 of the block's extent, on a
far start where both accepted and taken-back steps occur (their cost changes
are far from rounding: the decisions cannot flip)."""
import numpy as np
import pytest

import oracle
from damping_scene import far_start_ring

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


@pytest.mark.parametrize("graph", [False, True])
def test_adaptive_damping_parity(rp, graph):
    s = far_start_ring()
    gp = rp.Problem(s, lam=1e-6, damping=rp.RPBA_DAMPING_ADAPTIVE)
    gp.set_graph(graph)
    op = oracle.OracleProblem(s, lam=1e-6)
    op.set_damping(1)
    n_rej = 0
    for t in range(2):
        g = gp.rpba_intersect()
        o = op.intersect()
        gp.sync()
        assert np.allclose(g.cpu().numpy(), o, rtol=TOL, atol=0)
        for i in range(4):
            gb = gp.rpba_subblock_lm_step()
            gp.sync()
            ob, _ = op.lm_step()
            gl, gr = gp.damping()
            ol, orj = op.damping()
            assert np.array_equal(gr, orj) and np.array_equal(gl, ol), (t, i, gl, ol, gr, orj)
            assert np.allclose(gb.cpu().numpy()[:, :3], ob[:, :3], rtol=TOL, atol=0), (t, i)
            n_rej += int(gr.sum())
        gp.rpba_consensus()
        op.consensus()
    assert n_rej > 0
    _, gC = gp.cameras()
    _, oC = op.cameras()
    assert np.abs(gC - oC).max() <= TOL * 10.0


def test_fixed_damping_reports_lambda(rp):
    s = far_start_ring()
    gp = rp.Problem(s, lam=1e-4)
    gp.rpba_intersect()
    gp.rpba_subblock_lm_step()
    lam, rej = gp.damping()
    assert np.all(lam == 1e-4) and not rej.any()


def test_adaptive_options_are_checked(rp):
    s = far_start_ring()
    with pytest.raises(rp.RpbaError, match="adaptive damping"):
        rp.Problem(s, damping=rp.RPBA_DAMPING_ADAPTIVE, lambda_up=1.0)
    with pytest.raises(rp.RpbaError, match="damping must be"):
        rp.Problem(s, damping=2)
