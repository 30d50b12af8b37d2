"""The oracle's ray casting (brute-force closest hit) against exact hand cases
and an independent float64 reference (tests/raycast_pins.py)."""
import numpy as np

import oracle
import raycast_pins


def _fn(verts, tris, lo, hi, rays, tmax):
    return oracle.raycast(verts, tris, lo, hi, rays, float(tmax))


def test_hand_cases():
    assert raycast_pins.hand_cases_pass(_fn)


def test_random_rays_against_float64_reference():
    assert raycast_pins.random_cases_pass(_fn, seed=0)
    assert raycast_pins.random_cases_pass(_fn, seed=1)


def test_grid_box_clip_and_tmax():
    # a triangle straddling the box face: its hit inside the box counts, beyond it not
    verts, tris = raycast_pins._soup([[[-0.5, 0.5, -1.0], [1.5, 0.5, -1.0], [0.5, 0.5, 3.0]]])
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    rays = raycast_pins._rays([[0.5, 0.0, 0.5], [0.5, 0.0, 2.0]], [[0, 1, 0], [0, 1, 0]])
    t, i = oracle.raycast(verts, tris, lo, hi, rays)
    assert t[0] == np.float32(0.5) and i[0] == 0
    assert i[1] == 0xFFFFFFFF and np.isinf(t[1])   # the ray at z = 2 never enters the box
