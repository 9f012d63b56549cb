"""Pins of the oracle's viscosity ratio (Sec. 2: the droplet phase has
viscosity chi mu; Eq. tau_to_nu ties each viscosity to a relaxation time).

* The inside indicator, defined by the winding number, against geometry
  that does not use solid angles: the half-space test of a convex
  polyhedron (an icosphere), and, for a star-shaped non-convex mesh, the
  distance from the centre to the surface along the ray through each node
  (ray-triangle intersection).
* The winding number itself: 1 at the centre, 0 far away, -1 for the
  reversed orientation.
* One collision step with chi != 1 equals, node by node, the step of a
  one-fluid run whose tau is the outer one outside the droplet and the inner
  one (nu_in = chi nu, so tau_in - 1/2 = chi (tau - 1/2)) inside.
"""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere


def _offset_center(L):
    # off the lattice's symmetry planes, so that no node sits on the surface
    return np.asarray(box_center(L)) + np.array([0.137, -0.291, 0.073])


def test_winding_number_special_points():
    V, T = icosphere(2, 5.0, (10.0, 10.0, 10.0))
    assert abs(oracle.winding(V, T, (10.0, 10.0, 10.0)) - 1.0) < 1e-12
    assert abs(oracle.winding(V, T, (10.3, 9.1, 11.2)) - 1.0) < 1e-12
    assert abs(oracle.winding(V, T, (30.0, 10.0, 10.0))) < 1e-12
    assert abs(oracle.winding(V, T, (10.0, 16.0, 10.0))) < 1e-12
    assert abs(oracle.winding(V, T[:, ::-1], (10.0, 10.0, 10.0)) + 1.0) < 1e-12


def test_indicator_convex_mesh_half_spaces():
    L = (24, 22, 26)
    c = _offset_center(L)
    V, T = icosphere(3, 6.3, c)
    ind = oracle.indicator(L, V, T)
    # a point is inside a convex polyhedron iff it is behind every face plane
    a, b, cc = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, cc - a)
    z, y, x = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    P = np.stack([x, y, z], -1).reshape(-1, 3).astype(float)
    s = P @ n.T - (n * a).sum(1)[None]
    inside = (s < 0).all(1)
    margin = np.abs(s / np.linalg.norm(n, axis=1)[None]).min(1)
    assert margin.min() > 1e-6  # no node on the surface
    assert (ind.reshape(-1).astype(bool) == inside).all()
    assert inside.sum() > 700


def _star_mesh(c, R):
    V, T = icosphere(3, 1.0, (0.0, 0.0, 0.0))
    u = V / np.linalg.norm(V, axis=1, keepdims=True)
    rad = R * (1.0 + 0.35 * (u[:, 0] ** 2 - u[:, 2] ** 2) + 0.25 * u[:, 1] * u[:, 2] - 0.2 * u[:, 0] * u[:, 1] * u[:, 2])
    return c + u * rad[:, None], T


def _ray_radius(V, T, c, d):
    """Distance from c along the unit direction d to the mesh (Moller-Trumbore)."""
    a, b, e = V[T[:, 0]] - c, V[T[:, 1]] - c, V[T[:, 2]] - c
    e1, e2 = b - a, e - a
    h = np.cross(d, e2)
    det = (e1 * h).sum(1)
    f = 1.0 / det
    s = -a
    uu = f * (s * h).sum(1)
    q = np.cross(s, e1)
    vv = f * (q @ d)
    t = f * (e2 * q).sum(1)
    hit = (uu >= 0) & (vv >= 0) & (uu + vv <= 1) & (t > 0)
    return t[hit].min(), t[hit].max()


def test_indicator_star_shaped_mesh_ray_distance():
    L = (30, 30, 30)
    c = _offset_center(L)
    V, T = _star_mesh(c, 7.0)
    ind = oracle.indicator(L, V, T)
    checked = 0
    lo, hi = np.floor(V.min(0)).astype(int) - 1, np.ceil(V.max(0)).astype(int) + 1
    for z in range(lo[2], hi[2] + 1):
        for y in range(lo[1], hi[1] + 1):
            for x in range(lo[0], hi[0] + 1):
                p = np.array([x, y, z], float) - c
                r = np.linalg.norm(p)
                t0, t1 = _ray_radius(V, T, c, p / r)
                assert abs(t1 - t0) < 1e-9  # star-shaped: one crossing per ray
                if abs(r - t0) < 1e-6:
                    continue
                assert ind[z, y, x] == (r < t0), (x, y, z, r, t0)
                checked += 1
    assert ind.sum() > 1000 and checked > 5000
    # nothing outside the mesh's bounding box
    mask = np.zeros_like(ind, dtype=bool)
    mask[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = True
    assert ind[~mask].sum() == 0


def test_one_step_takes_the_inner_tau_inside():
    L = (20, 20, 20)
    c = _offset_center(L)
    V, T = icosphere(2, 5.2, c)
    tau, chi = 0.9, 3.5
    tau_in = 0.5 + chi * (tau - 0.5)   # nu = (tau - 1/2)/3, nu_in = chi nu
    rng = np.random.default_rng(7)
    kw = dict(radius=5.2, vertices=V, triangles=T, periodic=(1, 1, 1), reg_max_iter=0, sigma=0.02)
    base = oracle.Oracle(L, tau, **kw)
    f0 = base.populations()
    f0 = f0 + 1e-3 * rng.standard_normal(f0.shape) * f0
    runs = {}
    for name, t, x in (("chi", tau, chi), ("out", tau, 1.0), ("in", tau_in, 1.0)):
        o = oracle.Oracle(L, t, chi=x, **kw)
        o.set_populations(f0)
        if name == "chi":
            ind = o.indicator().reshape(-1)
        o.step(np.zeros(9))
        runs[name] = o.populations()
        o.close()
    base.close()
    assert 100 < ind.sum() < ind.size
    cv, _, _ = oracle.lattice()
    z, y, x = np.meshgrid(np.arange(L[2]), np.arange(L[1]), np.arange(L[0]), indexing="ij")
    for i in range(19):
        src = (((x - cv[i, 0]) % L[0]) + L[0] * (((y - cv[i, 1]) % L[1]) + L[1] * ((z - cv[i, 2]) % L[2]))).reshape(-1)
        want = np.where(ind[src] == 1, runs["in"][:, i], runs["out"][:, i])
        assert np.array_equal(runs["chi"][:, i], want), i
    # the two one-fluid runs do differ inside
    assert np.abs(runs["in"] - runs["out"]).max() > 1e-6


def test_chi_one_and_no_mesh_are_the_one_fluid_step():
    L = (12, 12, 12)
    A = np.zeros(9)
    A[1] = 1e-3
    ref = oracle.Oracle(L, 0.8, A0=A)
    ref.step(A, 3)
    o = oracle.Oracle(L, 0.8, A0=A, chi=4.0)
    o.step(A, 3)
    assert np.array_equal(o.populations(), ref.populations())
    ref.close()
    o.close()


def test_chi_rejected_with_mrt():
    with pytest.raises(oracle.OracleError):
        oracle.Oracle((8, 8, 8), 0.8, chi=2.0, collision="mrt")
