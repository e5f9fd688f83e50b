"""Seeded scene for the adaptive-damping tests: the ring block with its
cameras turned by 25 degrees about random axes and shifted by 0.4 units, so
that undamped Gauss-Newton steps overshoot and get taken back."""
import dataclasses

import numpy as np

from paper_1910_08138_amd import scenes


def _rotation(axis, angle):
    a = axis / np.linalg.norm(axis)
    K = np.array([[0.0, -a[2], a[1]], [a[2], 0.0, -a[0]], [-a[1], a[0], 0.0]])
    return np.eye(3) + np.sin(angle) * K + (1.0 - np.cos(angle)) * K @ K


def far_start_ring(seed=2, deg=25.0, shift=0.4, n_pts=400):
    s = scenes.ring_scene(2, n_pts=n_pts)
    rng = np.random.default_rng(seed)
    R = s.cam_R.reshape(-1, 3, 3)
    axes = rng.normal(size=(s.M, 3))
    Rp = np.stack([_rotation(axes[i], np.deg2rad(deg)) @ R[i] for i in range(s.M)])
    Cp = s.cam_C + shift * rng.normal(size=s.cam_C.shape)
    return dataclasses.replace(s, cam_R=np.ascontiguousarray(Rp.reshape(-1, 9)), cam_C=np.ascontiguousarray(Cp))
