"""Why a block-diagonal learned preconditioner cannot beat block-Jacobi on
the reduced camera systems, checked on a sub-block system of the method
(config 5 at small size) with the oracle's FP64 arithmetic:

  * Kaporin's condition number K(A) = (tr(A)/n)^n / det(A) of the
    preconditioned matrix, which bounds the CG iterations, is smallest for
    block-Jacobi among all block-diagonal SPD preconditioners (the trace of
    P S only sees the diagonal blocks; det(P S) = det(P) det(S), and for each
    block tr(P_i S_ii) / det(P_i)^(1/6) is smallest at P_i = S_ii^-1): the
    trained network's blocks and random SPD blocks both come out larger.
  * The trained network (the weights the bench uses) widens the spectrum of
    the preconditioned system and needs more CG iterations than
    block-Jacobi.
"""
import os

import numpy as np

import oracle
from paper_1910_08138_amd import scenes

WEIGHTS = os.path.join(os.path.dirname(__file__), "..", "paper_1910_08138_amd", "weights", "precond_config5.npy")


def _obs_tp(s):
    nblk = np.zeros(s.N, dtype=np.int64)
    key = np.unique(s.obs_pt.astype(np.int64) * s.L + s.cam_block[s.obs_cam])
    np.add.at(nblk, key // s.L, 1)
    nobs = np.bincount(s.obs_cam, minlength=s.M).astype(np.float64)
    ntp = np.bincount(s.obs_cam, weights=(nblk[s.obs_pt] > 1).astype(np.float64), minlength=s.M)
    return np.stack([nobs, ntp / np.maximum(nobs, 1)], axis=1)


def _system():
    s = scenes.config_scene(5, 30, small=True)
    op = oracle.OracleProblem(s)
    op.intersect()
    op.lm_step()
    op.consensus()
    op.intersect()
    cams = np.nonzero(s.cam_block == 0)[0]
    S, e = op.block_rcs(0, 6 * cams.size)
    return s, cams, S, e


def _blockdiag(P):
    n = P.shape[0]
    out = np.zeros((6 * n, 6 * n))
    for i in range(n):
        out[6 * i:6 * i + 6, 6 * i:6 * i + 6] = P[i]
    return out


def log_kaporin(P, S):
    """log K(P S) = n log(tr(P S) / n) - log det(P S)."""
    A = _blockdiag(P) @ S
    n = S.shape[0]
    sign_p, ld_p = np.linalg.slogdet(_blockdiag(P))
    sign_s, ld_s = np.linalg.slogdet(S)
    assert sign_p > 0 and sign_s > 0
    return n * np.log(np.trace(A) / n) - (ld_p + ld_s)


def test_block_jacobi_minimises_kaporins_condition_number():
    s, cams, S, _ = _system()
    nb = cams.size
    Pbj = np.stack([np.linalg.inv(S[6 * i:6 * i + 6, 6 * i:6 * i + 6]) for i in range(nb)])
    k_bj = log_kaporin(Pbj, S)
    W = np.load(WEIGHTS, allow_pickle=False).astype(np.float64)
    feat = oracle.mlp_features(S, _obs_tp(s)[cams], lam=1e-4)
    Pnet, _ = oracle.mlp_blocks(S, feat, W)
    assert log_kaporin(Pnet, S) > k_bj
    # block-Jacobi scaled per block by any positive factor, or perturbed by
    # random SPD factors, only raises it
    rng = np.random.default_rng(0)
    for trial in range(5):
        Q = []
        for i in range(nb):
            B = np.eye(6) + 0.3 * rng.normal(size=(6, 6))
            Q.append(B @ Pbj[i] @ B.T)
        assert log_kaporin(np.stack(Q), S) > k_bj
        scale = np.exp(rng.normal(size=nb))[:, None, None]
        assert log_kaporin(Pbj * scale, S) > k_bj


def test_trained_network_widens_the_spectrum_and_slows_cg():
    s, cams, S, e = _system()
    nb = cams.size
    W = np.load(WEIGHTS, allow_pickle=False).astype(np.float64)
    feat = oracle.mlp_features(S, _obs_tp(s)[cams], lam=1e-4)
    Pnet, _ = oracle.mlp_blocks(S, feat, W)
    Pbj = np.stack([np.linalg.inv(S[6 * i:6 * i + 6, 6 * i:6 * i + 6]) for i in range(nb)])

    def spectrum(P):
        Lp = np.linalg.cholesky(_blockdiag(P))
        ev = np.linalg.eigvalsh(Lp.T @ S @ Lp)
        return ev[-1] / ev[0]

    k_bj, k_net = spectrum(Pbj), spectrum(Pnet)
    _, it_bj, _ = oracle.pcg(S, e, None, tol=1e-10, maxit=5000)
    _, it_net, _ = oracle.pcg(S, e, Pnet, tol=1e-10, maxit=5000)
    print(f"condition: block-Jacobi {k_bj:.3e}, network {k_net:.3e}; CG iterations {it_bj} vs {it_net}")
    assert k_net > k_bj and it_net > it_bj
