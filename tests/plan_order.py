"""The library's internal camera order and the tiles of its Cholesky factors
that can be nonzero, recomputed in Python from the plan's rules, for tests
that need to know them (the library does not export its plan).

Cameras are grouped by sub-block and, inside a sub-block, put in reverse
Cuthill-McKee order of the co-visibility graph: two cameras are adjacent if
they observe a common point; each connected part starts at an unvisited
camera of least degree, neighbours are visited by ascending degree, then by
caller order, and the visiting order is reversed."""
import numpy as np


def camera_order(s):
    """Internal camera index: cameras grouped by sub-block, inside a sub-block
    in reverse Cuthill-McKee order of the co-visibility graph (start at an
    unvisited camera of least degree, neighbours by degree, then by caller
    order), as the library's plan orders them."""
    M = s.M
    L = int(s.cam_block.max()) + 1
    off = np.zeros(L + 1, np.int64)
    np.add.at(off, s.cam_block + 1, 1)
    off = np.cumsum(off)
    members = [np.flatnonzero(s.cam_block == l) for l in range(L)]
    loc = np.empty(M, np.int64)
    for l in range(L):
        loc[members[l]] = np.arange(len(members[l]))
    adj = [dict() for _ in range(L)]
    o = np.argsort(s.obs_pt, kind="stable")
    pts, cams = s.obs_pt[o], s.obs_cam[o]
    starts = np.flatnonzero(np.r_[True, pts[1:] != pts[:-1]])
    for a, b in zip(starts, np.r_[starts[1:], len(pts)]):
        cs = cams[a:b]
        for ca in cs:
            for cb in cs:
                if ca != cb and s.cam_block[ca] == s.cam_block[cb]:
                    adj[s.cam_block[ca]].setdefault(loc[ca], set()).add(loc[cb])
    cam_new = np.empty(M, np.int64)
    for l in range(L):
        n = len(members[l])
        nbr = [sorted(adj[l].get(u, ())) for u in range(n)]
        deg = [len(x) for x in nbr]
        seen = [False] * n
        order = []
        while len(order) < n:
            s0 = min((u for u in range(n) if not seen[u]), key=lambda u: (deg[u], u))
            seen[s0] = True
            order.append(s0)
            head = len(order) - 1
            while head < len(order):
                u = order[head]
                head += 1
                nxt = sorted((v for v in nbr[u] if not seen[v]), key=lambda v: (deg[v], v))
                for v in nxt:
                    seen[v] = True
                    order.append(v)
        for q in range(n):
            cam_new[members[l][order[n - 1 - q]]] = off[l] + q
    return cam_new


def factor_tiles(s, tile=64):
    """Per sub-block, a boolean (nt, nt) lower-triangular array: True where a
    tile of the Cholesky factor of the reduced camera system can be nonzero
    (tiles of S touched by a pair of co-visible cameras, diagonal tiles, then
    the fill of a tile factorisation)."""
    cam_new = camera_order(s)
    L = int(s.cam_block.max()) + 1
    off = np.zeros(L + 1, np.int64)
    np.add.at(off, s.cam_block + 1, 1)
    off = np.cumsum(off)
    out = []
    o = np.argsort(s.obs_pt, kind="stable")
    pts, cams = s.obs_pt[o], s.obs_cam[o]
    starts = np.flatnonzero(np.r_[True, pts[1:] != pts[:-1]])
    pairs = [set() for _ in range(L)]
    for a, b in zip(starts, np.r_[starts[1:], len(pts)]):
        cs = cams[a:b]
        for ca in cs:
            for cb in cs:
                if s.cam_block[ca] == s.cam_block[cb]:
                    l = s.cam_block[ca]
                    pairs[l].add((cam_new[ca] - off[l], cam_new[cb] - off[l]))
    for l in range(L):
        n = off[l + 1] - off[l]
        nt = -(-6 * n // tile)
        z = np.eye(nt, dtype=bool)
        for a, b in pairs[l]:
            for ra in {6 * a // tile, (6 * a + 5) // tile}:
                for rb in {6 * b // tile, (6 * b + 5) // tile}:
                    z[max(ra, rb), min(ra, rb)] = True
        for k in range(nt):
            rows = np.flatnonzero(z[k + 1:, k]) + k + 1
            for x in rows:
                z[x, rows[rows <= x]] = True
        out.append(z)
    return out
