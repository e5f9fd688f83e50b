"""Definitions of the visibility-graph partition (paper Sec. 5.2), written
out plainly with numpy: the graph, the node weights, the quality figures of a
partition, and the best balanced bisection of a tiny graph by enumeration.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; the product path never
imports it.  The partitioner itself is a heuristic; these definitions are
what its output is checked against.
"""
from __future__ import annotations

import itertools

import numpy as np


def _incidence(M, obs_cam, obs_pt):
    import scipy.sparse as sp
    obs_cam = np.asarray(obs_cam)
    obs_pt = np.asarray(obs_pt)
    N = int(obs_pt.max()) + 1
    return sp.csr_matrix((np.ones(obs_cam.size), (obs_pt, obs_cam)), shape=(N, M))


def visibility_graph(M, obs_cam, obs_pt):
    """Dense M x M matrix E: E[a, b] = number of points observed by both
    camera a and camera b (a != b), diagonal 0; E = A^T A without its
    diagonal, A the point-by-camera incidence matrix."""
    A = _incidence(M, obs_cam, obs_pt)
    E = np.rint((A.T @ A).toarray()).astype(np.int64)
    np.fill_diagonal(E, 0)
    return E


def node_weights(M, obs_cam, obs_pt):
    """Cube root of the summed observation counts of the points each camera
    sees."""
    obs_cam = np.asarray(obs_cam)
    obs_pt = np.asarray(obs_pt)
    n_obs = np.bincount(obs_pt)
    return np.cbrt(np.bincount(obs_cam, weights=n_obs[obs_pt].astype(float), minlength=M))


def partition_stats(M, obs_cam, obs_pt, cam_block, E=None):
    """Edge cut, tie points (points seen in >= 2 sub-blocks), point copies
    (sum over points of the sub-blocks seeing them), per-part node weights and
    camera counts."""
    obs_cam = np.asarray(obs_cam)
    obs_pt = np.asarray(obs_pt).astype(np.int64)
    cam_block = np.asarray(cam_block)
    if E is None:
        E = visibility_graph(M, obs_cam, obs_pt)
    diff = cam_block[:, None] != cam_block[None, :]
    cut = int(E[diff].sum() // 2)
    L = int(cam_block.max()) + 1
    pairs = np.unique(obs_pt * L + cam_block[obs_cam])     # distinct (point, sub-block) pairs
    per_pt = np.bincount(pairs // L)
    w = node_weights(M, obs_cam, obs_pt)
    pw = np.bincount(cam_block, weights=w, minlength=L)
    pn = np.bincount(cam_block, minlength=L)
    return dict(edge_cut=cut, tie_points=int((per_pt >= 2).sum()), point_copies=int(per_pt.sum()), part_weight=pw,
                part_cams=pn)


def best_bisection(E, w, f, eps):
    """Smallest cut over all bisections whose side 0 holds at most
    (1 + eps) f W and side 1 at most (1 + eps)(1 - f) W of the node weight W,
    by enumeration (tiny graphs only).  Returns (cut, side array)."""
    M = E.shape[0]
    W = float(np.sum(w))
    cap0, cap1 = (1 + eps) * f * W, (1 + eps) * (1 - f) * W
    best = (None, None)
    for bits in itertools.product((0, 1), repeat=M - 1):
        side = np.array((0,) + bits)          # camera 0 on side 0 (the sides are not symmetric, so try both)
        for s in (side, 1 - side):
            if not (s.any() and (1 - s).any()):
                continue
            w0, w1 = float(np.sum(w[s == 0])), float(np.sum(w[s == 1]))
            if w0 > cap0 or w1 > cap1:
                continue
            cut = int(E[s[:, None] != s[None, :]].sum() // 2)
            if best[0] is None or cut < best[0]:
                best = (cut, s.copy())
    return best
