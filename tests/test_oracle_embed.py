"""Pins of the FP64 embedding oracle (oracle/embed.py, Eq. m2y) against what
linear shape functions must do: reproduce the rest points at rest, reproduce
affine motions exactly, give the unit vectors at the tet's corners, and equal
the barycentric coordinates of the textbook 4x4 system."""

import numpy as np

import synth
from oracle.embed import embed, shape_values


def _box():
    p = synth.problem_by_name("box")
    tet, P = synth.yarn_points(p.X, p.tets, per_tet=3, seed=4)
    return p, tet, P


def test_rest_positions_are_reproduced():
    p, tet, P = _box()
    N = shape_values(p.X, p.tets, tet, P)
    assert np.abs(embed(p.X, p.tets, tet, N) - P).max() < 1e-15
    assert np.abs(N.sum(axis=1) - 1).max() < 1e-13
    assert N.min() > -1e-12                        # the points lie inside their tets


def test_affine_motion_is_reproduced():
    p, tet, P = _box()
    N = shape_values(p.X, p.tets, tet, P)
    A = np.array([[1.2, 0.3, -0.1], [0.05, 0.8, 0.2], [-0.3, 0.1, 1.1]])
    b = np.array([0.01, -0.02, 0.5])
    assert np.abs(embed(p.X @ A.T + b, p.tets, tet, N) - (P @ A.T + b)).max() < 1e-14


def test_corners_give_unit_vectors():
    p = synth.problem_by_name("box")
    tet = np.repeat(np.arange(5), 4)
    P = p.X[p.tets[tet, np.tile(np.arange(4), 5)]]
    N = shape_values(p.X, p.tets, tet, P)
    assert np.abs(N - np.tile(np.eye(4), (5, 1))).max() < 1e-12


def test_matches_barycentric_linear_system():
    p, tet, P = _box()
    N = shape_values(p.X, p.tets, tet, P)
    for i in range(0, len(tet), 97):
        Xa = p.X[p.tets[tet[i]]]                                   # [4, 3]
        A = np.vstack([Xa.T, np.ones(4)])                          # [4, 4]
        lam = np.linalg.solve(A, np.append(P[i], 1.0))
        assert np.abs(lam - N[i]).max() < 1e-12
