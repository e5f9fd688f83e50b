"""The plan's camera order and the tiles of the Cholesky factor it declares
nonzero, on the CPU (the plan code compiled with g++, no GPU):

* the camera order inside each sub-block is the reverse Cuthill-McKee order
  that the Python replica in plan_order.py computes;
* every tile that is nonzero in a numerically computed Cholesky factor of an
  SPD matrix with the reduced camera system's 6x6 block pattern is declared
  nonzero (skipping a declared-zero tile would drop real fill);
* the dataflow task list covers every declared tile and passes its own
  dependency-order check."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import plan_order
from paper_1910_08138_amd import scenes

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
T = 64

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("plan") / "plan_probe")
    csrc = os.path.join(ROOT, "paper_1910_08138_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", csrc, "-I", os.path.join(ROOT, "include"),
                    os.path.join(HERE, "plan_probe.cpp"), os.path.join(csrc, "rpba_plan.cpp"), "-o", exe],
                   check=True)
    return exe


def _run(probe, s, tmp_path):
    f = tmp_path / "topo.bin"
    with open(f, "wb") as fh:
        np.array([s.M, s.N, s.K, int(s.cam_block.max()) + 1], np.int32).tofile(fh)
        s.obs_cam.astype(np.int32).tofile(fh)
        s.obs_pt.astype(np.int32).tofile(fh)
        s.cam_block.astype(np.int32).tofile(fh)
    out = subprocess.run([probe, str(f)], capture_output=True, text=True, check=True).stdout.splitlines()
    cam_orig = np.array(out[0].split()[1:], dtype=np.int64)
    tiles = []
    for line in out[1:-1]:
        w = line.split()
        nt = int(w[2])
        z = np.zeros((nt, nt), bool)
        z[np.tril_indices(nt)] = np.array(w[3:], dtype=int) != 0
        tiles.append(z)
    ntask = int(out[-1].split()[1])
    return cam_orig, tiles, ntask


SCENES = {
    "ring": lambda: scenes.ring_scene(3, n_cams=40, n_pts=2000, n_blocks=3),
    "oblique-small": lambda: scenes.config_scene(3, 1, small=True),
    "oblique-banded": lambda: scenes.oblique_scene(2, n_strips=4, n_stations=30, n_pts=30_000, n_blocks=4,
                                                  size_range=(120, 180)),
}


@pytest.mark.parametrize("name", list(SCENES))
def test_camera_order_and_factor_tiles(probe, tmp_path, name):
    s = SCENES[name]()
    cam_orig, tiles, ntask = _run(probe, s, tmp_path)
    cam_new = plan_order.camera_order(s)
    ref = np.empty(s.M, np.int64)
    ref[cam_new] = np.arange(s.M)
    assert np.array_equal(cam_orig, ref)
    assert [z.shape[0] for z in tiles] == [z.shape[0] for z in plan_order.factor_tiles(s, T)]
    # the declared pattern holds the numeric fill of a random SPD matrix with
    # the system's block pattern, in the plan's camera order
    rng = np.random.default_rng(0)
    L = int(s.cam_block.max()) + 1
    off = np.concatenate([[0], np.cumsum(np.bincount(s.cam_block, minlength=L))])
    o = np.argsort(s.obs_pt, kind="stable")
    pts, cams = s.obs_pt[o], s.obs_cam[o]
    starts = np.flatnonzero(np.r_[True, pts[1:] != pts[:-1]])
    for l in range(L):
        n = off[l + 1] - off[l]
        adj = np.eye(n, dtype=bool)
        for a, b in zip(starts, np.r_[starts[1:], len(pts)]):
            cs = [cam_new[c] - off[l] for c in cams[a:b] if s.cam_block[c] == l]
            for x in cs:
                adj[x, cs] = True
        nt = tiles[l].shape[0]
        mask = np.kron(adj, np.ones((6, 6), bool))
        A = np.where(mask, rng.normal(size=mask.shape), 0.0)
        A = A + A.T
        A += np.diag(np.abs(A).sum(axis=1) + 1.0)
        Lf = np.linalg.cholesky(A)
        pad = np.zeros((nt * T, nt * T))
        pad[:6 * n, :6 * n] = Lf
        nz = np.abs(pad.reshape(nt, T, nt, T)).max(axis=(1, 3)) > 0
        assert not np.any(np.tril(nz) & ~tiles[l]), (name, l)
        assert np.array_equal(np.diag(tiles[l]), np.ones(nt, bool))
    # every declared tile plus the right-hand-side row is one task
    assert ntask == sum(int(z.sum()) + z.shape[0] for z in tiles)
    if name == "oblique-banded":
        assert sum(int(z.sum()) for z in tiles) < sum(z.shape[0] * (z.shape[0] + 1) // 2 for z in tiles)
