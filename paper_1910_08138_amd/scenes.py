"""Seeded synthetic bundle-adjustment scenes.

This module is the ONLY code shared by the HIP path and the CPU oracle: it
draws cameras, points, observations and sub-block partitions, and nothing of
the adjustment itself (no linearisation, no normal equations, no solves).  It
does contain a forward camera model, because a simulator has to render image
observations; that model is written here independently of both solvers.

Scene families (shapes and value distributions of the paper's workloads):

* ``ring``     -- calibrated cameras on a ring around a unit cube of points
                  (tiny block; two halves of the ring are the sub-blocks).
* ``aerial``   -- nadir grid over a terrain height field, the "traditional
                  aerial block" of the paper's simulated data set (Sec. 6),
                  here at 500 cameras and 200k points.
* ``oblique``  -- strips of 5-camera rigs (nadir + four 45 degree obliques),
                  6,000 cameras, 2.5M points, ~12M observations, split into
                  64 uneven sub-blocks (20-400 cameras, log-uniform sizes).
* ``harvest``  -- an aerial scene re-partitioned into two large sub-blocks, the
                  source of reduced camera systems for the learned
                  preconditioner.

Conventions (all float64):
  camera i: rotation R_i (world -> camera, row-major 3x3) and projection
  centre C_i; a point X maps to p = R_i (X - C_i), pixel
  (f p1/p3 + cx, f p2/p3 + cy); the camera looks along +p3.

Array layouts returned (the C-ABI layouts):
  cam_R (M, 9) row-major; cam_C (3, M); pts (3, N); obs_xy (2, K);
  obs_cam (K,) int32; obs_pt (K,) int32; cam_block (M,) int32.

Random streams: one ``SeedSequence(seed)`` spawns independent generators for
geometry, observation noise, perturbation and partitioning, so e.g. changing
the partition never changes the noise.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F_PX = 1000.0
CX = 500.0
CY = 500.0
IMG_W = 1000.0
IMG_H = 1000.0


# --------------------------------------------------------------------------
# small geometry helpers (simulator only)
# --------------------------------------------------------------------------
def _look_rotation(z_axis: np.ndarray, up_hint: np.ndarray) -> np.ndarray:
    """Rows (x_c, y_c, z_c): camera z along ``z_axis``, y_c 'down' w.r.t. up_hint."""
    z = z_axis / np.linalg.norm(z_axis)
    x = np.cross(z, up_hint)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z])


def _quat_rotation(axis: np.ndarray, angle: float) -> np.ndarray:
    """Rotation matrix of a unit quaternion (cos a/2, sin a/2 * axis)."""
    a = axis / np.linalg.norm(axis)
    w = math.cos(angle / 2.0)
    x, y, z = a * math.sin(angle / 2.0)
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _unit_vectors(rng: np.random.Generator, n: int) -> np.ndarray:
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def render(R: np.ndarray, C: np.ndarray, X: np.ndarray):
    """Forward camera model for the simulator.

    R (n, 3, 3), C (n, 3), X (n, 3) -> (u (n,), v (n,), depth (n,)).
    """
    d = X - C
    p = np.einsum("nij,nj->ni", R, d)
    depth = p[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = F_PX * p[:, 0] / depth + CX
        v = F_PX * p[:, 1] / depth + CY
    return u, v, depth


def _in_image(u, v, depth):
    return (depth > 1e-6) & (u >= 0.0) & (u < IMG_W) & (v >= 0.0) & (v < IMG_H)


# --------------------------------------------------------------------------
# partitions
# --------------------------------------------------------------------------
def rcb_partition(pos: np.ndarray, sizes, rng: np.random.Generator) -> np.ndarray:
    """Recursive coordinate bisection of camera positions into parts of the given sizes.

    The size list is shuffled, then split in halves recursively; at each level
    the cameras are cut along the axis of largest extent at the cumulative
    count of the first half.  Ties are broken by camera index, so the result is
    deterministic given ``rng``.  A stand-in for a visibility-graph partitioner.
    """
    sizes = [int(s) for s in sizes]
    order = rng.permutation(len(sizes))
    sizes = [sizes[i] for i in order]
    M = pos.shape[0]
    assert sum(sizes) == M, (sum(sizes), M)
    block = np.empty(M, dtype=np.int32)
    next_id = [0]

    def rec(idx: np.ndarray, parts):
        if len(parts) == 1:
            block[idx] = next_id[0]
            next_id[0] += 1
            return
        half = len(parts) // 2
        p1, p2 = parts[:half], parts[half:]
        n1 = sum(p1)
        sub = pos[idx]
        axis = int(np.argmax(sub.max(axis=0) - sub.min(axis=0)))
        o = np.lexsort((idx, sub[:, axis]))
        rec(idx[o[:n1]], p1)
        rec(idx[o[n1:]], p2)

    rec(np.arange(M), sizes)
    return block


def loguniform_block_sizes(rng: np.random.Generator, n_blocks=64, lo=20, hi=400,
                           total=6000, slack=100, max_draws=1_000_000):
    """Integer log-uniform sizes in [lo, hi], conditioned on summing to ``total``.

    Draws n_blocks i.i.d. sizes until the sum is within ``slack`` of total, then
    moves the largest (or smallest) sizes by one, inside [lo, hi], until the sum
    is exact.
    """
    for _ in range(max_draws):
        s = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi + 1), size=n_blocks))).astype(np.int64)
        s = np.clip(s, lo, hi)
        if abs(int(s.sum()) - total) <= slack:
            break
    else:  # pragma: no cover
        raise RuntimeError("block size sampler did not converge")
    while s.sum() != total:
        if s.sum() > total:
            cand = np.where(s > lo)[0]
            i = cand[np.argmax(s[cand])]
            s[i] -= 1
        else:
            cand = np.where(s < hi)[0]
            i = cand[np.argmax(s[cand])]
            s[i] += 1
    return s


# --------------------------------------------------------------------------
# scene container
# --------------------------------------------------------------------------
@dataclass
class Scene:
    name: str
    seed: int
    f: float
    cx: float
    cy: float
    sigma_px: float
    cam_R: np.ndarray          # (M, 9) initial (perturbed)
    cam_C: np.ndarray          # (3, M) initial (perturbed)
    pts: np.ndarray            # (3, N) initial
    obs_xy: np.ndarray         # (2, K)
    obs_cam: np.ndarray        # (K,) int32
    obs_pt: np.ndarray         # (K,) int32
    cam_block: np.ndarray      # (M,) int32
    cam_R_true: np.ndarray
    cam_C_true: np.ndarray
    pts_true: np.ndarray
    outlier: np.ndarray | None = None   # (K,) bool, gross errors injected
    meta: dict = field(default_factory=dict)
    # intrinsics estimated per camera (focal length f and radial distortion
    # k1 of the normalised image coordinates), None for calibrated scenes
    cam_f: np.ndarray | None = None     # (M,) initial
    cam_k1: np.ndarray | None = None    # (M,) initial
    cam_f_true: np.ndarray | None = None
    cam_k1_true: np.ndarray | None = None

    @property
    def M(self):
        return self.cam_R.shape[0]

    @property
    def N(self):
        return self.pts.shape[1]

    @property
    def K(self):
        return self.obs_xy.shape[1]

    @property
    def L(self):
        return int(self.cam_block.max()) + 1

    def arrays(self):
        """Contiguous copies of the mutable state (cameras, points)."""
        return (np.ascontiguousarray(self.cam_R.copy()), np.ascontiguousarray(self.cam_C.copy()),
                np.ascontiguousarray(self.pts.copy()))

    def repartition(self, cam_block: np.ndarray, name: str | None = None) -> "Scene":
        s = Scene(**{k: getattr(self, k) for k in self.__dataclass_fields__})
        s.cam_block = np.ascontiguousarray(cam_block.astype(np.int32))
        if name:
            s.name = name
        return s


def _streams(seed: int):
    ss = np.random.SeedSequence(seed)
    geo, noise, pert, part = (np.random.default_rng(s) for s in ss.spawn(4))
    return geo, noise, pert, part


def _perturb_cameras(rng, R_true, C_true, shift):
    """Rotate each camera by exactly 1 degree about a uniform axis, shift its
    centre by ``shift[i]`` in a uniform direction."""
    M = R_true.shape[0]
    axes = _unit_vectors(rng, M)
    dirs = _unit_vectors(rng, M)
    R = np.empty_like(R_true)
    for i in range(M):
        R[i] = _quat_rotation(axes[i], math.radians(1.0)) @ R_true[i]
    C = C_true + dirs * np.asarray(shift).reshape(-1, 1)
    return R, C


def _finish(name, seed, R_true, C_true, X_true, obs_cam, obs_pt, cam_block, sigma,
            noise_rng, pert_rng, cam_shift, pt_sigma, outlier_frac=0.0, meta=None, noise=None):
    """Render, add noise N(0, noise^2) (noise defaults to sigma, the a-priori
    standard deviation that the solvers weight with), inject outliers, perturb."""
    K = obs_cam.shape[0]
    u, v, depth = render(R_true[obs_cam], C_true[obs_cam], X_true[obs_pt])
    assert np.all(depth > 0)
    ns = sigma if noise is None else noise
    xy = np.stack([u, v]) + noise_rng.normal(scale=1.0, size=(2, K)) * ns
    outlier = None
    if outlier_frac > 0:
        n_out = int(round(outlier_frac * K))
        idx = noise_rng.choice(K, size=n_out, replace=False)
        xy[:, idx] += noise_rng.uniform(-50.0, 50.0, size=(2, n_out))
        outlier = np.zeros(K, dtype=bool)
        outlier[idx] = True
    R0, C0 = _perturb_cameras(pert_rng, R_true, C_true, cam_shift)
    X0 = X_true + pert_rng.normal(scale=pt_sigma, size=X_true.shape)
    return Scene(
        name=name, seed=seed, f=F_PX, cx=CX, cy=CY, sigma_px=sigma,
        cam_R=np.ascontiguousarray(R0.reshape(-1, 9)),
        cam_C=np.ascontiguousarray(C0.T),
        pts=np.ascontiguousarray(X0.T),
        obs_xy=np.ascontiguousarray(xy),
        obs_cam=np.ascontiguousarray(obs_cam.astype(np.int32)),
        obs_pt=np.ascontiguousarray(obs_pt.astype(np.int32)),
        cam_block=np.ascontiguousarray(cam_block.astype(np.int32)),
        cam_R_true=np.ascontiguousarray(R_true.reshape(-1, 9)),
        cam_C_true=np.ascontiguousarray(C_true.T),
        pts_true=np.ascontiguousarray(X_true.T),
        outlier=outlier, meta=dict(meta or {}))


# --------------------------------------------------------------------------
# ring (tiny block)
# --------------------------------------------------------------------------
def ring_scene(seed=0, n_cams=20, n_pts=2000, radius=5.0, views=(3, 8), sigma=0.5,
               n_blocks=2, noise=None) -> Scene:
    geo, nrng, pert, part = _streams(seed)
    R = np.empty((n_cams, 3, 3))
    C = np.empty((n_cams, 3))
    for i in range(n_cams):
        phi = 2 * math.pi * i / n_cams
        C[i] = (radius * math.cos(phi), radius * math.sin(phi), 0.0)
        R[i] = _look_rotation(-C[i], np.array([0.0, 0.0, 1.0]))
    X = geo.uniform(-0.5, 0.5, size=(n_pts, 3))
    nv = geo.integers(views[0], views[1] + 1, size=n_pts)
    cams = [np.sort(geo.choice(n_cams, size=int(m), replace=False)) for m in nv]
    obs_pt = np.repeat(np.arange(n_pts), nv)
    obs_cam = np.concatenate(cams)
    per = n_cams // n_blocks
    cam_block = np.minimum(np.arange(n_cams) // per, n_blocks - 1)
    return _finish("ring", seed, R, C, X, obs_cam, obs_pt, cam_block, sigma, nrng, pert,
                   cam_shift=np.full(n_cams, 0.01 * radius), pt_sigma=0.01 * radius,
                   meta=dict(radius=radius), noise=noise)


# --------------------------------------------------------------------------
# terrain
# --------------------------------------------------------------------------
class Terrain:
    """Sum of Gaussian bumps, amplitude in [-amp, amp], widths in [wmin, wmax]."""

    def __init__(self, rng, x_range, y_range, n_bumps=8, amp=10.0, wmin=50.0, wmax=200.0):
        self.cx = rng.uniform(*x_range, size=n_bumps)
        self.cy = rng.uniform(*y_range, size=n_bumps)
        self.a = rng.uniform(-amp, amp, size=n_bumps)
        self.w = rng.uniform(wmin, wmax, size=n_bumps)

    def __call__(self, x, y):
        h = np.zeros_like(x)
        for cx, cy, a, w in zip(self.cx, self.cy, self.a, self.w):
            h += a * np.exp(-((x - cx) ** 2 + (y - cy) ** 2) / (2 * w * w))
        return h


def _nadir_R():
    return _look_rotation(np.array([0.0, 0.0, -1.0]), np.array([0.0, 1.0, 0.0]))


# --------------------------------------------------------------------------
# aerial nadir grid
# --------------------------------------------------------------------------
def aerial_scene(seed=0, nx=20, ny=25, H=100.0, spacing=40.0, n_pts=200_000,
                 max_views=12, min_views=3, sigma=0.5, n_blocks=16, noise=None) -> Scene:
    geo, nrng, pert, part = _streams(seed)
    gx, gy = np.meshgrid(np.arange(nx) * spacing, np.arange(ny) * spacing, indexing="ij")
    C = np.stack([gx.ravel(), gy.ravel(), np.full(nx * ny, H)], axis=1)
    M = C.shape[0]
    R = np.broadcast_to(_nadir_R(), (M, 3, 3)).copy()
    half = 0.5 * H * IMG_W / F_PX
    x_range = (-half, (nx - 1) * spacing + half)
    y_range = (-half, (ny - 1) * spacing + half)
    terrain = Terrain(geo, x_range, y_range)

    X_list, obs_pt_l, obs_cam_l = [], [], []
    have = 0
    while have < n_pts:
        nb = max(4096, int((n_pts - have) * 1.3))
        x = geo.uniform(*x_range, size=nb)
        y = geo.uniform(*y_range, size=nb)
        Xb = np.stack([x, y, terrain(x, y)], axis=1)
        ix0 = np.floor(x / spacing).astype(np.int64)
        iy0 = np.floor(y / spacing).astype(np.int64)
        cand_pt, cand_cam = [], []
        reach = int(math.ceil((half + 20.0) / spacing)) + 1
        for dx in range(-reach + 1, reach + 1):
            for dy in range(-reach + 1, reach + 1):
                ix, iy = ix0 + dx, iy0 + dy
                ok = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny)
                pi = np.nonzero(ok)[0]
                ci = (ix[pi] * ny + iy[pi])
                u, v, d = render(R[ci], C[ci], Xb[pi])
                vis = _in_image(u, v, d)
                cand_pt.append(pi[vis])
                cand_cam.append(ci[vis])
        cp = np.concatenate(cand_pt)
        cc = np.concatenate(cand_cam)
        # random subset of at most max_views per point: random keys, rank within point
        key = geo.random(cp.shape[0])
        o = np.lexsort((key, cp))
        cp, cc = cp[o], cc[o]
        starts = np.searchsorted(cp, np.arange(nb))
        counts = np.bincount(cp, minlength=nb)
        rank = np.arange(cp.shape[0]) - starts[cp]
        keep = rank < max_views
        cp, cc = cp[keep], cc[keep]
        counts = np.minimum(counts, max_views)
        good = counts >= min_views
        good_idx = np.nonzero(good)[0][: n_pts - have]
        remap = -np.ones(nb, dtype=np.int64)
        remap[good_idx] = np.arange(good_idx.shape[0]) + have
        sel = remap[cp] >= 0
        X_list.append(Xb[good_idx])
        obs_pt_l.append(remap[cp[sel]])
        obs_cam_l.append(cc[sel])
        have += good_idx.shape[0]
    X = np.concatenate(X_list)
    obs_pt = np.concatenate(obs_pt_l)
    obs_cam = np.concatenate(obs_cam_l)
    o = np.lexsort((obs_cam, obs_pt))
    obs_pt, obs_cam = obs_pt[o], obs_cam[o]
    base, extra = divmod(M, n_blocks)
    sizes = [base + 1] * extra + [base] * (n_blocks - extra)
    cam_block = rcb_partition(C[:, :2], sizes, part)
    return _finish("aerial", seed, R, C, X, obs_cam, obs_pt, cam_block, sigma, nrng, pert,
                   cam_shift=np.full(M, 0.01 * H), pt_sigma=0.01 * H,
                   meta=dict(H=H, spacing=spacing, nx=nx, ny=ny), noise=noise)


# --------------------------------------------------------------------------
# oblique strips with 5-camera rigs
# --------------------------------------------------------------------------
def _rig_rotations(tilt_deg=45.0):
    t = math.radians(tilt_deg)
    up = np.array([0.0, 1.0, 0.0])
    dirs = [np.array([0.0, 0.0, -1.0])]
    for hx, hy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        dirs.append(np.array([math.sin(t) * hx, math.sin(t) * hy, -math.cos(t)]))
    return np.stack([_look_rotation(d, up) for d in dirs])


def oblique_scene(seed=0, n_strips=12, n_stations=100, H=100.0, along=40.0, across=60.0,
                  n_pts=2_500_000, views=(3, 7), sigma=0.5, n_blocks=64, size_range=(20, 400),
                  outlier_frac=0.0, draws_per_round=24, max_rounds=16, chunk=250_000,
                  noise=None) -> Scene:
    geo, nrng, pert, part = _streams(seed)
    rig = _rig_rotations()
    n_rig = rig.shape[0]
    sx = np.arange(n_stations) * along
    sy = np.arange(n_strips) * across
    st_x, st_y = np.meshgrid(sx, sy, indexing="xy")          # (strips, stations)
    st = np.stack([st_x.ravel(), st_y.ravel(), np.full(st_x.size, H)], axis=1)
    n_st = st.shape[0]
    M = n_st * n_rig
    C = np.repeat(st, n_rig, axis=0)                          # camera = station * 5 + rig
    R = np.tile(rig, (n_st, 1, 1))
    margin = 50.0
    x_range = (-margin, sx[-1] + margin)
    y_range = (-margin, sy[-1] + margin)
    terrain = Terrain(geo, x_range, y_range)
    # ground footprints of the rig cameras relative to the station, from the
    # depth range over the terrain: nadir |dx|, |dy| <= d/2; a 45 degree oblique
    # with a +-26.57 degree field sees (1/3 .. 3) d along its tilt and
    # +-sqrt(2) d across it.  Candidate stations per camera are the stations
    # whose footprint box can contain the point.
    gx_s = np.linspace(*x_range, 200)
    gy_s = np.linspace(*y_range, 60)
    hz = terrain(*np.meshgrid(gx_s, gy_s))
    dmin = H - hz.max() - 5.0
    dmax = H - hz.min() + 5.0
    boxes = [(-0.5 * dmax - 1, 0.5 * dmax + 1, -0.5 * dmax - 1, 0.5 * dmax + 1)]  # (xlo, xhi, ylo, yhi) of point - station
    near, far, side = dmin / 3.0 - 1, 3.0 * dmax + 1, math.sqrt(2.0) * dmax + 1
    boxes += [(near, far, -side, side), (-far, -near, -side, side), (-side, side, near, far), (-side, side, -far, -near)]

    X_list, obs_pt_l, obs_cam_l = [], [], []
    have = 0
    while have < n_pts:
        nb = min(chunk, int((n_pts - have) * 1.1) + 1024)
        x = geo.uniform(*x_range, size=nb)
        y = geo.uniform(*y_range, size=nb)
        Xb = np.stack([x, y, terrain(x, y)], axis=1)
        want = geo.integers(views[0], views[1] + 1, size=nb)
        # per point and rig: station index windows and candidate counts
        lo_a = np.empty((nb, n_rig), np.int64)
        lo_c = np.empty((nb, n_rig), np.int64)
        na_ = np.empty((nb, n_rig), np.int64)
        nc_ = np.empty((nb, n_rig), np.int64)
        for r, (xl, xh, yl, yh) in enumerate(boxes):
            a0 = np.maximum(np.ceil((x - xh) / along), 0).astype(np.int64)
            a1 = np.minimum(np.floor((x - xl) / along), n_stations - 1).astype(np.int64)
            c0 = np.maximum(np.ceil((y - yh) / across), 0).astype(np.int64)
            c1 = np.minimum(np.floor((y - yl) / across), n_strips - 1).astype(np.int64)
            lo_a[:, r], lo_c[:, r] = a0, c0
            na_[:, r] = np.maximum(a1 - a0 + 1, 0)
            nc_[:, r] = np.maximum(c1 - c0 + 1, 0)
        ncand = na_ * nc_
        cum = np.cumsum(ncand, axis=1)
        tot = cum[:, -1]
        chosen = np.full((nb, views[1]), -1, dtype=np.int64)
        nchosen = np.zeros(nb, dtype=np.int64)
        active = np.nonzero(tot > 0)[0]
        for _ in range(max_rounds):
            if active.size == 0:
                break
            na = active.size
            D = draws_per_round
            u = (geo.random((na, D)) * tot[active, None]).astype(np.int64)
            cact = cum[active]
            rig_id = (u[:, :, None] >= cact[:, None, :]).sum(axis=2)
            prev_cum = np.where(rig_id > 0, np.take_along_axis(cact, np.maximum(rig_id - 1, 0), axis=1), 0)
            w = u - prev_cum
            ncr = np.take_along_axis(nc_[active], rig_id, axis=1)
            ia = np.take_along_axis(lo_a[active], rig_id, axis=1) + w // ncr
            ic = np.take_along_axis(lo_c[active], rig_id, axis=1) + w % ncr
            cam = (ic * n_stations + ia) * n_rig + rig_id
            flat_p = np.repeat(active, D)
            flat_c = cam.ravel()
            vis = np.zeros(flat_c.shape[0], dtype=bool)
            dxyz = Xb[flat_p] - C[flat_c]
            rig_of = rig_id.ravel()
            for r in range(n_rig):
                sel = np.nonzero(rig_of == r)[0]
                pr = dxyz[sel] @ rig[r].T
                with np.errstate(divide="ignore", invalid="ignore"):
                    uu = F_PX * pr[:, 0] / pr[:, 2] + CX
                    vv = F_PX * pr[:, 1] / pr[:, 2] + CY
                vis[sel] = _in_image(uu, vv, pr[:, 2])
            cam = np.where(vis.reshape(na, D), cam, -1)
            # drop draws that repeat an earlier draw or an already chosen camera
            prev = chosen[active]
            allc = np.concatenate([prev, cam], axis=1)
            o = np.argsort(allc, axis=1, kind="stable")
            sc = np.take_along_axis(allc, o, axis=1)
            dup_sorted = np.zeros_like(sc, dtype=bool)
            dup_sorted[:, 1:] = (sc[:, 1:] == sc[:, :-1]) & (sc[:, 1:] >= 0)
            dup = np.zeros_like(dup_sorted)
            np.put_along_axis(dup, o, dup_sorted, axis=1)
            newc = np.where(dup[:, prev.shape[1]:], -1, cam)
            # append the new distinct visible cameras in draw order, up to `want`
            valid = newc >= 0
            pos = nchosen[active][:, None] + np.cumsum(valid, axis=1) - 1
            take = valid & (pos < want[active][:, None])
            rr, cc = np.nonzero(take)
            chosen[active[rr], pos[rr, cc]] = newc[rr, cc]
            nchosen[active] = np.minimum(nchosen[active] + valid.sum(axis=1), want[active])
            active = active[nchosen[active] < want[active]]
        good = nchosen >= 2
        good_idx = np.nonzero(good)[0][: n_pts - have]
        cnt = nchosen[good_idx]
        X_list.append(Xb[good_idx])
        obs_pt_l.append(np.repeat(np.arange(good_idx.shape[0]) + have, cnt))
        rows = chosen[good_idx]
        obs_cam_l.append(rows[np.arange(views[1])[None, :] < cnt[:, None]])
        have += good_idx.shape[0]
    X = np.concatenate(X_list)
    obs_pt = np.concatenate(obs_pt_l)
    obs_cam = np.concatenate(obs_cam_l)
    o = np.lexsort((obs_cam, obs_pt))
    obs_pt, obs_cam = obs_pt[o], obs_cam[o]
    n_cams_total = M
    sizes = loguniform_block_sizes(part, n_blocks, size_range[0], size_range[1], n_cams_total,
                                   slack=max(2, n_cams_total // 60))
    cam_block = rcb_partition(C[:, :2], sizes, part)
    return _finish("oblique", seed, R, C, X, obs_cam, obs_pt, cam_block, sigma, nrng, pert,
                   cam_shift=np.full(M, 0.01 * H), pt_sigma=0.01 * H, outlier_frac=outlier_frac,
                   meta=dict(H=H, n_strips=n_strips, n_stations=n_stations), noise=noise)


def add_gross_errors(scene: Scene, frac: float, seed: int, lo: float = 15.0, hi: float = 40.0) -> Scene:
    """A copy of the scene with gross errors on round(frac K) observations
    drawn without replacement: displacements of uniform length in [lo, hi] px
    in a uniform direction (marked in `outlier`, together with any the scene
    already had)."""
    import dataclasses
    rng = np.random.default_rng(np.random.SeedSequence([seed, 7919]))
    idx = rng.choice(scene.K, size=int(round(frac * scene.K)), replace=False)
    ang = rng.uniform(0.0, 2.0 * math.pi, idx.size)
    mag = rng.uniform(lo, hi, idx.size)
    xy = scene.obs_xy.copy()
    xy[0, idx] += mag * np.cos(ang)
    xy[1, idx] += mag * np.sin(ang)
    out = np.zeros(scene.K, dtype=bool) if scene.outlier is None else scene.outlier.copy()
    out[idx] = True
    return dataclasses.replace(scene, obs_xy=np.ascontiguousarray(xy), outlier=out)


def render_distorted(R: np.ndarray, C: np.ndarray, X: np.ndarray, f: np.ndarray, k1: np.ndarray):
    """Forward model with per-observation focal length f (n,) and radial
    distortion k1 (n,) of the normalised coordinates q = p12 / p3:
    pixel f (1 + k1 |q|^2) q + (CX, CY)."""
    d = X - C
    p = np.einsum("nij,nj->ni", R, d)
    qx, qy = p[:, 0] / p[:, 2], p[:, 1] / p[:, 2]
    s = f * (1.0 + k1 * (qx * qx + qy * qy))
    return s * qx + CX, s * qy + CY


def with_intrinsics(scene: Scene, seed: int, f_rel: float = 0.02, k1_max: float = 0.1,
                    f_start_rel: float = 0.005) -> Scene:
    """A copy of the scene whose cameras have their own focal length and
    radial distortion, as in the paper's Final data sets (f and k1 per camera,
    Sec. 6).  True values: f = F_PX (1 + f_rel N(0, 1)), k1 ~ U(-k1_max,
    k1_max).  The observations are rendered again with them, keeping the
    scene's noise (and gross errors); start values: f off by f_start_rel
    N(0, 1) relative, k1 = 0."""
    import dataclasses
    rng = np.random.default_rng(np.random.SeedSequence([seed, 104729]))
    M = scene.M
    f_true = F_PX * (1.0 + f_rel * rng.normal(size=M))
    k1_true = rng.uniform(-k1_max, k1_max, size=M)
    f0 = f_true * (1.0 + f_start_rel * rng.normal(size=M))
    Rt = scene.cam_R_true.reshape(-1, 3, 3)[scene.obs_cam]
    Ct = scene.cam_C_true.T[scene.obs_cam]
    Xt = scene.pts_true.T[scene.obs_pt]
    u0, v0, _ = render(Rt, Ct, Xt)
    u1, v1 = render_distorted(Rt, Ct, Xt, f_true[scene.obs_cam], k1_true[scene.obs_cam])
    xy = scene.obs_xy + np.stack([u1 - u0, v1 - v0])
    return dataclasses.replace(scene, name=scene.name + "+intrinsics", obs_xy=np.ascontiguousarray(xy),
                               cam_f=np.ascontiguousarray(f0), cam_k1=np.zeros(M),
                               cam_f_true=f_true, cam_k1_true=k1_true)


def harvest_partition(scene: Scene, seed: int) -> Scene:
    """Two compact sub-blocks of s and M-s cameras, s ~ U{200..300} (for M=500)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(5)[4])
    M = scene.M
    lo, hi = int(0.4 * M), int(0.6 * M)
    s = int(rng.integers(lo, hi + 1))
    blk = rcb_partition(scene.cam_C_true.T[:, :2], [s, M - s], rng)
    return scene.repartition(blk, name=scene.name + "-harvest")


# --------------------------------------------------------------------------
# the five workload configurations
# --------------------------------------------------------------------------
def config_scene(config: int, seed: int = 0, small: bool = False) -> Scene:
    """Scenes of the five workloads; ``small`` shrinks 2-5 for CPU-side tests
    (same structure, fewer cameras and points)."""
    if config == 1:
        return ring_scene(seed)
    if config == 2:
        if small:
            return aerial_scene(seed, nx=8, ny=10, n_pts=12_000, n_blocks=4)
        return aerial_scene(seed)
    if config in (3, 4):
        frac = 0.02 if config == 4 else 0.0
        if small:
            return oblique_scene(seed, n_strips=4, n_stations=20, n_pts=40_000, n_blocks=10,
                                 size_range=(15, 80), outlier_frac=frac)
        return oblique_scene(seed, outlier_frac=frac)
    if config == 5:
        base = aerial_scene(seed, nx=8, ny=10, n_pts=12_000, n_blocks=2) if small else aerial_scene(seed)
        return harvest_partition(base, seed)
    raise ValueError(config)
