"""Pins of the test helpers that place a row mismatch relative to the voxel
faces (the allowed class: the path passes within 1e-4 mm of a voxel face),
on straight segments whose distances to a unit box are known in closed form."""
import numpy as np

from helpers import FACE_TOL, max_penetration, near_face_length, signed_depth

LO, HI = np.zeros(3), np.ones(3)


def test_signed_depth_closed_forms():
    assert signed_depth([0.5, 0.5, 0.5], LO, HI) == 0.5
    assert signed_depth([0.5, 0.5, 0.9], LO, HI) == 0.09999999999999998
    assert abs(signed_depth([1.3, 0.5, 0.5], LO, HI) + 0.3) < 1e-15
    assert abs(signed_depth([1.3, 1.4, 0.5], LO, HI) + 0.5) < 1e-15


def test_penetration_of_grazing_and_deep_paths():
    # a chord through the middle: half the side
    assert abs(max_penetration(np.array([[-1, 0.5, 0.5], [2, 0.5, 0.5]]), LO, HI) - 0.5) < 1e-12
    # parallel to the face z = 1 inside it by 3e-5: penetration 3e-5
    p = np.array([[-1, 0.5, 1 - 3e-5], [2, 0.5, 1 - 3e-5]])
    assert abs(max_penetration(p, LO, HI) - 3e-5) < 1e-12
    # a V-shaped polyline that dips 7e-5 into the box through the face y = 0
    v = np.array([[0.2, -0.5, 0.5], [0.5, 7e-5, 0.5], [0.8, -0.5, 0.5]])
    assert abs(max_penetration(v, LO, HI) - 7e-5) < 1e-10
    # one that misses the box by 2e-5
    w = np.array([[0.2, -0.5, 0.5], [0.5, -2e-5, 0.5], [0.8, -0.5, 0.5]])
    assert abs(max_penetration(w, LO, HI) + 2e-5) < 1e-10


def test_near_face_length_by_crossing_angle():
    # perpendicular crossing of the face x = 1: about 2 * tol of path near it
    p = np.array([[0.5, 0.5, 0.5], [1.5, 0.5, 0.5]])
    assert abs(near_face_length(p, LO, HI) - 2 * FACE_TOL) < 1e-4
    # crossing z = 1 with a slope of 1e-3 (sine ~1e-3): about 2 tol / 1e-3 = 0.2 mm
    q = np.array([[0.0, 0.5, 1 - 5e-4], [1.0, 0.5, 1 + 5e-4]])
    assert abs(near_face_length(q, LO, HI) - 0.2) < 2e-3
    # running along the face z = 1 at 5e-5 outside: the whole in-face length (1 mm + tol each side)
    r = np.array([[-0.5, 0.5, 1 + 5e-5], [1.5, 0.5, 1 + 5e-5]])
    assert abs(near_face_length(r, LO, HI) - (1.0 + 2 * FACE_TOL)) < 1e-3
