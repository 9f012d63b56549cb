"""Seeded input generators: icosphere mesh and OU velocity-gradient tables."""
import numpy as np
import pytest

from paper_2403_01161_amd.inputs import (box_center, icosphere, icosphere_counts,
                                         ou_gradient_table, simple_shear)


@pytest.mark.parametrize("level", [0, 1, 2, 3, 4])
def test_icosphere_topology(level):
    V, T = icosphere(level, 2.5, (1.0, 2.0, 3.0))
    nv, nt = icosphere_counts(level)
    assert V.shape == (nv, 3) and T.shape == (nt, 3)
    edges = set()
    for a, b, c in T:
        for u, v in ((a, b), (b, c), (c, a)):
            edges.add((min(u, v), max(u, v)))
    assert nv - len(edges) + nt == 2  # Euler characteristic of a sphere
    # every directed edge appears exactly once: closed and consistently oriented
    directed = [(int(u), int(v)) for a, b, c in T for u, v in ((a, b), (b, c), (c, a))]
    assert len(set(directed)) == len(directed) == 3 * nt
    assert all((v, u) in set(directed) for u, v in directed)
    np.testing.assert_allclose(np.linalg.norm(V - [1.0, 2.0, 3.0], axis=1), 2.5, rtol=1e-14)
    # outward: every face normal points away from the centre
    c = V[T].mean(axis=1) - [1.0, 2.0, 3.0]
    n = np.cross(V[T[:, 1]] - V[T[:, 0]], V[T[:, 2]] - V[T[:, 0]])
    assert np.all(np.einsum("ij,ij->i", n, c) > 0)


def test_icosphere_paper_mesh_size():
    # Sec. 3.2: a 20480-triangle mesh; the level-5 icosphere has exactly that many.
    assert icosphere_counts(5) == (10242, 20480)


def test_box_center():
    np.testing.assert_array_equal(box_center((32, 8, 5)), [15.5, 3.5, 2.0])


def test_simple_shear():
    A = simple_shear(0.25)
    assert A.reshape(3, 3)[0, 1] == 0.25 and np.count_nonzero(A) == 1


def test_ou_statistics():
    T, G, n = 50.0, 0.3, 200000
    A = ou_gradient_table(n, T, G, seed=7)
    assert A.shape == (n, 9)
    tr = A[:, 0] + A[:, 4] + A[:, 8]
    assert np.max(np.abs(tr)) < 1e-15
    rms = np.sqrt(np.mean(np.sum(A * A, axis=1)))
    assert abs(rms / G - 1.0) < 0.05
    a = A[:, 1]
    lag1 = np.corrcoef(a[:-1], a[1:])[0, 1]
    assert abs(lag1 - np.exp(-1.0 / T)) < 0.01
    # same seed -> same table; different seed -> different table
    np.testing.assert_array_equal(A[:100], ou_gradient_table(100, T, G, seed=7))
    assert not np.allclose(A[:100], ou_gradient_table(100, T, G, seed=8))
