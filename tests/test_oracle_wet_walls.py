"""Oracle wet-node velocity walls (Sec. 3.1, the Zou-He conditions in the 3D
form of Hecht and Harting): a fluid at rest between resting walls stays at
rest exactly, edges and corners included (the buried-link rules and
f_0 = 12 f_b return the rest weights); plane Couette flow between two moving
walls is steady and exact at every node, the wall nodes included; and at
every face node (one wall) the reconstructed populations carry exactly the
imposed velocity u_w = A (x - x_c), whatever the flow inside."""
import numpy as np

import oracle

from .test_oracle_physics import _grid, _traceless


def test_rest_stays_at_rest():
    L = (9, 10, 11)
    o = oracle.Oracle(L, 0.8, walls="wet", init_rest=True)
    o.step(np.zeros(9), 30)
    f = o.populations().reshape(-1, 19)
    w = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)  # D3Q19 rest weights (index 0 rest, 1-6 axes)
    assert np.abs(f - w[None, :]).max() <= 1e-15
    o.close()


def test_couette_exact_with_wet_walls():
    L = (4, 12, 4)
    g = 1e-3
    A = np.zeros(9)
    A[1] = g
    o = oracle.Oracle(L, 0.8, A0=A, periodic=(1, 0, 1), walls="wet")
    o.step(A, 300)
    rho, u = o.fields()
    x, y, z = _grid(L)
    assert np.abs(u[0] - g * (y - (L[1] - 1) / 2)).max() < 1e-15
    assert np.abs(u[1:]).max() < 1e-15
    assert np.abs(rho - 1.0).max() < 1e-14
    o.close()


def test_face_nodes_carry_wall_velocity():
    L = (10, 11, 12)
    A = _traceless(2e-3, 6)
    o = oracle.Oracle(L, 0.9, A0=A, walls="wet")
    o.step(A, 7)
    rho, u = o.fields()
    x, y, z = _grid(L)
    X = np.stack([x, y, z]).astype(float) - ((np.array(L) - 1) / 2)[:, None, None, None]
    uw = np.einsum("ab,b...->a...", A.reshape(3, 3), X)
    nwall = sum(((c == 0) | (c == n - 1)).astype(int) for c, n in zip((x, y, z), L))
    face = nwall == 1
    assert face.sum() > 0
    assert np.abs(u[:, face] - uw[:, face]).max() <= 1e-15
    o.close()
