"""CPU-side checks of the C-ABI library: it loads, exports every symbol that
include/rpba.h declares, and its host-side validation (rpba_workspace_size
plans without touching the GPU) rejects malformed problems."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1910_08138_amd import binding, scenes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = "".join(open(os.path.join(ROOT, "include", h)).read() for h in ("rpba.h", "rpba_testing.h"))
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rpba_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = binding.load_library()
    names = _declared()
    assert "rpba_intersect" in names and "rpba_subblock_lm_step" in names and "rpba_consensus" in names
    for n in names:
        assert hasattr(L, n), n
    assert sorted(binding.EXPORTS) == names


def _desc(s):
    d = binding.ProblemDesc()
    d.M, d.N, d.K, d.L = s.M, s.N, s.K, s.L
    d.f, d.cx, d.cy, d.sigma_px = s.f, s.cx, s.cy, s.sigma_px
    fake = ctypes.c_void_p(256)     # never dereferenced by the planner
    d.cam_R = d.cam_C = d.pts = d.obs_xy = fake.value
    keep = [np.ascontiguousarray(s.obs_cam, np.int32), np.ascontiguousarray(s.obs_pt, np.int32),
            np.ascontiguousarray(s.cam_block, np.int32)]
    d.obs_cam, d.obs_pt, d.cam_block = (a.ctypes.data for a in keep)
    return d, keep


def _size(s, **kw):
    L = binding.load_library()
    d, keep = _desc(s)
    o = binding.default_options(**kw)
    n = ctypes.c_size_t(0)
    rc = L.rpba_workspace_size(ctypes.byref(d), ctypes.byref(o), ctypes.byref(n))
    return rc, n.value, L.rpba_last_error().decode()


def test_workspace_size_for_valid_scene():
    s = scenes.config_scene(1, 0)
    rc, n, msg = _size(s)
    assert rc == 0, msg
    assert n > s.K * 16


@pytest.mark.parametrize("mutate,needle", [
    (lambda s: s.obs_cam.__setitem__(0, s.M), "obs_cam out of range"),
    (lambda s: s.obs_pt.__setitem__(3, -1), "obs_pt out of range"),
    (lambda s: s.cam_block.__setitem__(0, -1), "cam_block out of range"),
])
def test_validation_rejects_bad_indices(mutate, needle):
    s = scenes.config_scene(1, 0)
    s.obs_cam = s.obs_cam.copy()
    s.obs_pt = s.obs_pt.copy()
    s.cam_block = s.cam_block.copy()
    mutate(s)
    rc, _, msg = _size(s)
    assert rc == 1 and needle in msg


def test_validation_rejects_single_view_point_and_repeated_pair():
    s = scenes.config_scene(1, 0)
    keep = s.obs_pt != 5
    first = np.nonzero(s.obs_pt == 5)[0][0]
    keep[first] = True                       # point 5 keeps one observation
    s1 = scenes.Scene(**{k: getattr(s, k) for k in s.__dataclass_fields__})
    s1.obs_xy, s1.obs_cam, s1.obs_pt = s.obs_xy[:, keep], s.obs_cam[keep], s.obs_pt[keep]
    rc, _, msg = _size(s1)
    assert rc == 1 and "fewer than 2" in msg
    s2 = scenes.Scene(**{k: getattr(s, k) for k in s.__dataclass_fields__})
    s2.obs_cam = s.obs_cam.copy()
    j = s.obs_pt[0]
    idx = np.nonzero(s.obs_pt == j)[0]
    s2.obs_cam[idx[1]] = s2.obs_cam[idx[0]]
    rc, _, msg = _size(s2)
    assert rc == 1 and "repeated" in msg


def test_validation_rejects_empty_subblock_and_bad_tile():
    s = scenes.config_scene(1, 0)
    s.cam_block = np.zeros(s.M, dtype=np.int32)
    s.cam_block[10:] = 2                     # sub-block 1 empty (L = 3)
    rc, _, msg = _size(s)
    assert rc == 1 and "no camera" in msg
    s = scenes.config_scene(1, 0)
    rc, _, msg = _size(s, chol_tile=48)
    assert rc == 1 and "chol_tile" in msg
    rc, _, msg = _size(s, chol_schedule=7)
    assert rc == 1 and "chol_schedule" in msg
    rc, _, msg = _size(s, pair_lanes=5)
    assert rc == 1 and "pair_lanes" in msg
    rc, _, msg = _size(s, robust=2)
    assert rc == 1 and "robust" in msg
    rc, _, msg = _size(s, solver=5)
    assert rc == 1 and "solver" in msg
    rc, _, msg = _size(s, covariance=2)
    assert rc == 1 and "covariance" in msg
    rc, _, msg = _size(s, damping=binding.RPBA_DAMPING_ADAPTIVE, lambda_down=0.5)
    assert rc == 1 and "adaptive damping" in msg
    with pytest.raises(TypeError, match="unknown option"):
        binding.default_options(lamda=1e-3)


def test_intrinsics_options_are_validated_and_size_the_camera_system():
    """Intrinsics (f and k1 per camera, Sec. 6) need their start values, the
    direct solver and the extended variant; the reduced camera systems then
    have 8 rows per camera (the dense RCS grows by (8/6)^2)."""
    s = scenes.config_scene(1, 0)
    L = binding.load_library()
    d, keep = _desc(s)
    fake = ctypes.c_void_p(512)
    n = ctypes.c_size_t(0)

    def size(cam_intr, **kw):
        d.cam_intr = cam_intr
        rc = L.rpba_workspace_size(ctypes.byref(d), ctypes.byref(binding.default_options(**kw)), ctypes.byref(n))
        return rc, n.value, L.rpba_last_error().decode()
    rc, _, msg = size(None, intrinsics=1)
    assert rc == 1 and "cam_intr" in msg
    rc, _, msg = size(fake.value, intrinsics=1, solver=binding.RPBA_SOLVER_PCG_BJ)
    assert rc == 1 and "RPBA_SOLVER_CHOL" in msg
    rc, _, msg = size(fake.value, intrinsics=1, variant=binding.RPBA_VARIANT_PLAIN)
    assert rc == 1 and "RPBA_VARIANT_EXTENDED" in msg
    rc, _, msg = size(fake.value, intrinsics=2)
    assert rc == 1 and "intrinsics" in msg
    rc6, n6, _ = size(None)
    rc8, n8, _ = size(fake.value, intrinsics=1)
    assert rc6 == 0 and rc8 == 0 and n8 > n6


def test_optional_arrays_take_workspace_only_when_asked():
    """The covariance array (one more dense RCS) and the adaptive-damping
    copy positions (24 bytes per copy) are laid out only with their options."""
    s = scenes.config_scene(1, 0)
    rc0, n0, _ = _size(s)
    rc1, n1, _ = _size(s, covariance=1)
    rc2, n2, _ = _size(s, damping=binding.RPBA_DAMPING_ADAPTIVE)
    assert rc0 == rc1 == rc2 == 0
    assert n1 > n0 and n2 - n0 >= 24 * s.N   # at least one copy per point


def test_residuals_take_workspace_only_when_kept():
    """A handle without the robust option keeps no residuals (16 bytes per
    observation less)."""
    s = scenes.config_scene(1, 0)
    rc0, n0, _ = _size(s, robust=0)
    rc1, n1, _ = _size(s, robust=1)
    assert rc0 == 0 and rc1 == 0
    assert n1 - n0 >= 16 * s.K


@pytest.mark.parametrize("first,costs,steps", [
    # the hand-worked sequences of the oracle's pin (tests/test_oracle_hand_pins.py)
    (100.0, [50.0, 49.8, 30.0, 29.9, 10.0], 4),
    (100.0, [99.5, 99.2, 50.0], 2),
    (10.0, [11.0, 9.0, 8.99, 1.0], 3),
    (100.0, [90.0, 80.0, 70.0], 3),
    (101.0, [100.0, 99.0], 2),
])
def test_library_ratio_rule_hand_sequences(first, costs, steps):
    """Sec. 5.4 improvement test in the library (host code, no GPU work):
    a step with best-so-far / cost below 1.01 is tolerated once, the second
    ends the loop."""
    best, grace, act = np.array([first]), np.zeros(1, np.uint8), np.ones(1, np.uint8)
    taken = 0
    for c in costs:
        taken += 1
        if binding.ratio_update(np.array([c]), best, grace, act) == 0:
            break
    assert taken == steps


def test_library_ratio_rule_many_loops_at_once():
    """Loops are independent and an inactive loop is left untouched."""
    best = np.array([100.0, 100.0, 5.0])
    grace = np.array([0, 1, 0], np.uint8)
    act = np.array([1, 1, 0], np.uint8)
    n = binding.ratio_update(np.array([99.5, 99.5, 1.0]), best, grace, act)
    # loop 0: short, first time -> grace; loop 1: short with grace -> stops;
    # loop 2: inactive, unchanged
    assert n == 1
    assert act.tolist() == [1, 0, 0] and grace.tolist() == [1, 1, 0]
    assert best.tolist() == [99.5, 99.5, 5.0]


def test_tuner_stages_with_intrinsics():
    """With f and k1 per camera only the factorisation is searched (the pair
    pass takes 8 lanes, every sub-block is solved directly)."""
    from paper_1910_08138_amd import tune
    st = tune.stages(binding.RPBA_MIXED, intrinsics=True)
    assert len(st) == 1 and all(c["pcg_min_cams"] is None and c["pair_lanes"] == 8 for c in st[0])
    assert len(tune.stages(binding.RPBA_MIXED)) == 3 and len(tune.stages(binding.RPBA_FP64)) == 2
    s = scenes.config_scene(1, 0)
    assert tune.signature(s, binding.RPBA_MIXED) != tune.signature(scenes.with_intrinsics(s, 0), binding.RPBA_MIXED)
