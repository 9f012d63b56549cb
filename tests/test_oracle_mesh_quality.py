"""Oracle mesh-quality observables (smallest triangle angle, shortest and
longest edge) against closed forms: the regular icosahedron (all angles 60
degrees, edge R / sin 72 degrees), a tetrahedron with right-angled faces
(smallest angle atan(1/4)), invariance under rotation and scaling, and the
law of cosines on a sheared icosphere."""
import math

import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import icosphere


def _outward(V, T):
    c = V.mean(axis=0)
    T = np.array(T, dtype=np.int32)
    for k, (a, b, d) in enumerate(T):
        if np.dot(np.cross(V[b] - V[a], V[d] - V[a]), V[a] - c) < 0:
            T[k] = (a, d, b)
    return T


def test_icosahedron():
    R = 3.0
    V, T = icosphere(0, R)
    q = oracle.shape(V, T, radius=R)
    assert q["min_angle_deg"] == pytest.approx(60.0, abs=1e-12)
    a = R / math.sin(2 * math.pi / 5)
    assert q["edge_min"] == pytest.approx(a, rel=1e-13)
    assert q["edge_max"] == pytest.approx(a, rel=1e-13)


def test_right_angled_tetrahedron():
    V = np.array([[0, 0, 0], [4, 0, 0], [0, 3, 0], [0, 0, 12]], dtype=np.float64) + 10.0
    T = _outward(V, [(0, 1, 2), (0, 1, 3), (0, 2, 3), (1, 2, 3)])
    q = oracle.shape(V, T)
    assert q["min_angle_deg"] == pytest.approx(math.degrees(math.atan(0.25)), abs=1e-12)
    assert q["edge_min"] == pytest.approx(3.0, rel=1e-14)
    assert q["edge_max"] == pytest.approx(math.sqrt(160.0), rel=1e-14)


def _law_of_cosines(V, T):
    P = V[T]
    l = np.stack([np.linalg.norm(P[:, 1] - P[:, 2], axis=1), np.linalg.norm(P[:, 2] - P[:, 0], axis=1),
                  np.linalg.norm(P[:, 0] - P[:, 1], axis=1)], axis=1)
    ang = []
    for k in range(3):
        a, b, c = l[:, k], l[:, (k + 1) % 3], l[:, (k + 2) % 3]
        ang.append(np.degrees(np.arccos(np.clip((b * b + c * c - a * a) / (2 * b * c), -1, 1))))
    return np.min(ang), l.min(), l.max()


def test_sheared_icosphere_matches_law_of_cosines():
    V, T = icosphere(3, 5.0)
    M = np.array([[1.0, 0.6, 0.0], [0.0, 1.0, 0.0], [0.2, 0.0, 0.7]])
    W = V @ M.T + 20.0
    q = oracle.shape(W, T, radius=5.0)
    amin, emin, emax = _law_of_cosines(W, T)
    assert q["min_angle_deg"] == pytest.approx(amin, abs=1e-6)  # arccos near small angles
    assert q["edge_min"] == pytest.approx(emin, rel=1e-13)
    assert q["edge_max"] == pytest.approx(emax, rel=1e-13)


def test_rotation_and_scale_invariance():
    V, T = icosphere(2, 4.0)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    if np.linalg.det(Q) < 0:
        Q[:, 0] = -Q[:, 0]
    W = V @ np.diag([1.0, 0.8, 1.3])
    q0 = oracle.shape(W, T)
    q1 = oracle.shape(2.5 * W @ Q.T + 7.0, T)
    assert q1["min_angle_deg"] == pytest.approx(q0["min_angle_deg"], abs=1e-10)
    assert q1["edge_min"] == pytest.approx(2.5 * q0["edge_min"], rel=1e-12)
    assert q1["edge_max"] == pytest.approx(2.5 * q0["edge_max"], rel=1e-12)
