"""Pins of the oracle's iterative solver and learned block preconditioner."""
import numpy as np
import pytest

import oracle
from paper_1910_08138_amd import scenes


def _rand_spd_blocks(rng, nb, coupled=True, cond=1e4):
    n = 6 * nb
    A = rng.normal(size=(n, n)) / np.sqrt(n)
    S = A @ A.T + np.diag(np.exp(rng.uniform(0, np.log(cond), n)))
    if not coupled:
        mask = np.kron(np.eye(nb), np.ones((6, 6)))
        S = S * mask
    return S


def test_pcg_block_diagonal_system_converges_in_one_iteration():
    """Block-Jacobi preconditioning is exact for a block-diagonal RCS (cameras
    sharing no points): one CG iteration."""
    rng = np.random.default_rng(0)
    S = _rand_spd_blocks(rng, 7, coupled=False)
    e = rng.normal(size=S.shape[0])
    x, it, h = oracle.pcg(S, e, tol=1e-12)
    assert it == 1
    assert np.allclose(x, np.linalg.solve(S, e), rtol=1e-12, atol=1e-14)


def test_pcg_matches_direct_solve_on_a_reduced_camera_system():
    """On a real RCS (two-sub-block aerial scene) PCG to 1e-10 agrees with
    numpy's direct solve; residual history is what the stop rule saw."""
    s = scenes.config_scene(5, 1, small=True)
    op = oracle.OracleProblem(s)
    op.intersect()
    op.lm_step()
    n6 = 6 * int((s.cam_block == 0).sum())
    S, e = op.block_rcs(0, n6)
    x_ref = np.linalg.solve(S, e)
    x, it, h = oracle.pcg(S, e, tol=1e-10, maxit=2000)
    assert h[-1] <= 1e-10 and it < 2000
    assert np.linalg.norm(S @ x - e) <= 1.0000001e-10 * np.linalg.norm(e)
    assert np.abs(x - x_ref).max() <= 1e-5 * np.abs(x_ref).max()


def test_zero_network_output_is_block_jacobi_and_blocks_are_spd():
    """P_i = G^-T L L^T G^-1 with L = I (zero output) is S_ii^-1; any output
    gives symmetric positive definite blocks."""
    rng = np.random.default_rng(1)
    S = _rand_spd_blocks(rng, 9)
    feat = oracle.mlp_features(S, np.stack([rng.integers(10, 100, 9), rng.random(9)], 1))
    P0, Gi = oracle.mlp_blocks(S, feat, None)
    for b in range(9):
        Sii = S[6 * b:6 * b + 6, 6 * b:6 * b + 6]
        assert np.allclose(P0[b] @ Sii, np.eye(6), atol=1e-10)
        assert np.allclose(Gi[b] @ np.linalg.cholesky(Sii), np.eye(6), atol=1e-10)
    params = rng.normal(size=oracle.mlp_num_params()) * 0.3
    P, _ = oracle.mlp_blocks(S, feat, params)
    for b in range(9):
        assert np.allclose(P[b], P[b].T, atol=1e-12 * np.abs(P[b]).max())
        assert np.linalg.eigvalsh(P[b]).min() > 0
    # a zero-output network reproduces block-Jacobi PCG iteration for iteration
    e = rng.normal(size=S.shape[0])
    params0 = params.copy()
    nf, nh, no = oracle.MLP_NF, oracle.MLP_NH, oracle.MLP_NO
    off = nf * nh + nh + nh * nh + nh
    params0[off:] = 0.0                      # last layer zero -> output zero
    Pz, _ = oracle.mlp_blocks(S, feat, params0)
    x1, it1, h1 = oracle.pcg(S, e, tol=1e-10)
    x2, it2, h2 = oracle.pcg(S, e, P=Pz, tol=1e-10)
    assert it1 == it2 and np.allclose(h1, h2, rtol=1e-10, atol=0)


def test_network_gradient_matches_central_differences():
    """Backward pass of the SPAI-type loss vs central differences of the loss."""
    rng = np.random.default_rng(2)
    S = _rand_spd_blocks(rng, 5)
    n = S.shape[0]
    feat = oracle.mlp_features(S, np.stack([rng.integers(10, 100, 5), rng.random(5)], 1))
    _, Gi = oracle.mlp_blocks(S, feat, None)
    params = rng.normal(size=oracle.mlp_num_params()) * 0.2
    z = rng.choice([-1.0, 1.0], size=(3, n))
    zw = np.stack([z, z @ S.T], axis=1)
    loss, grad = oracle.mlp_loss_grad(Gi, feat, params, zw)
    assert loss > 0
    idx = rng.choice(params.size, size=40, replace=False)
    idx = np.concatenate([idx, np.arange(params.size - 21, params.size)])  # include the output biases
    for q in idx:
        h = 1e-6
        pp, pm = params.copy(), params.copy()
        pp[q] += h
        pm[q] -= h
        fd = (oracle.mlp_loss_grad(Gi, feat, pp, zw)[0] - oracle.mlp_loss_grad(Gi, feat, pm, zw)[0]) / (2 * h)
        assert abs(fd - grad[q]) <= 1e-6 * max(1.0, abs(fd)) + 1e-7 * np.abs(grad).max(), (q, fd, grad[q])


def test_spai_loss_of_exact_inverse_is_zero_for_block_diagonal_systems():
    """For a block-diagonal S the zero-output (block-Jacobi) blocks are the exact
    inverse: the Hutchinson loss vanishes."""
    rng = np.random.default_rng(3)
    S = _rand_spd_blocks(rng, 4, coupled=False)
    feat = oracle.mlp_features(S, np.ones((4, 2)))
    _, Gi = oracle.mlp_blocks(S, feat, None)
    params = np.zeros(oracle.mlp_num_params())
    z = rng.choice([-1.0, 1.0], size=(2, S.shape[0]))
    loss, _ = oracle.mlp_loss_grad(Gi, feat, params, np.stack([z, z @ S.T], 1))
    assert loss < 1e-20
