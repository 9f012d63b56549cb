"""Overlapped step (step variant bit 7): the lattice update of step n + 1 in
two launches on two streams, the rows outside the row box beside the IB half
of step n and the rows inside it. The result must not change:

* FP64 against the oracle at the round-off bars of the plain step, in the
  linear and row layouts, around a periodic corner (the box wraps), with the
  MRT collision, one population copy and the deterministic spreading;
* FP32 against the same handle without bit 7 after an OU run: equal values
  with the deterministic spreading (only the launches differ, not the
  arithmetic of any node), equal to FP32 rounding with the atomics;
* the lattice timing counts a sweep of two launches once;
* ensembles refuse the bit.
"""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere, ou_gradient_table, simple_shear

pytestmark = pytest.mark.gpu

OVERLAP = 128
F64_TOL = dict(tol_r=1e-11, tol_u=1e-11, tol_rho=1e-13)


@pytest.fixture(scope="module")
def ib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01161_amd import ibmlb
    ibmlb.lib()
    return ibmlb


def _traceless(scale, seed):
    A = np.random.default_rng(seed).standard_normal((3, 3))
    A -= np.trace(A) / 3 * np.eye(3)
    return (scale * A / np.linalg.norm(A)).ravel()


def _compare(sim, ref, tol_r, tol_u, tol_rho):
    dr = np.abs(sim.vertices() - ref.vertices()).max()
    rho_g, u_g = sim.fields()
    rho_r, u_r = ref.fields()
    du = np.abs(u_g - u_r).max() / np.abs(u_r).max()
    drho = np.abs(rho_g - rho_r).max()
    print(f"  max|dr| {dr:.2e}, max|du|/max|u| {du:.2e}, max|drho| {drho:.2e}", flush=True)
    assert dr <= tol_r and du <= tol_u and drho <= tol_rho


CASES = {
    "linear_walls_ragged": dict(L=(19, 17, 21), R=3.2, steps=30, A=_traceless(3e-3, 2), variant=33,
                                kw=dict(tau=0.9, sigma=0.02)),
    "rows_walls_ragged": dict(L=(19, 17, 21), R=3.2, steps=30, A=_traceless(3e-3, 3), variant=57,
                              kw=dict(tau=0.9, sigma=0.02)),
    "periodic_corner": dict(L=(12, 13, 16), R=2.5, steps=25, A=np.zeros(9), center=(0.3, 12.6, 0.0), variant=33,
                            kw=dict(tau=0.8, sigma=0.03, periodic=(1, 1, 1))),
    "periodic_corner_rows": dict(L=(12, 13, 16), R=2.5, steps=25, A=np.zeros(9), center=(11.8, 0.4, 15.7),
                                 variant=57, kw=dict(tau=0.8, sigma=0.03, periodic=(1, 1, 1))),
    "mrt": dict(L=(17, 16, 18), R=3.2, steps=30, A=_traceless(3e-3, 4), variant=33,
                kw=dict(tau=0.9, sigma=0.02, collision="mrt")),
    "one_copy": dict(L=(19, 17, 21), R=3.2, steps=31, A=_traceless(3e-3, 8), variant=96,
                     kw=dict(tau=0.9, sigma=0.02), sim=dict(populations=1)),
    "deterministic": dict(L=(18, 19, 17), R=3.2, steps=30, A=simple_shear(2e-3), variant=33,
                          kw=dict(tau=0.9, sigma=0.02), sim=dict(deterministic=True)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_f64_matches_oracle(ib, case):
    c = CASES[case]
    L = c["L"]
    V, T = icosphere(2, c["R"], c.get("center", box_center(L)))
    kw = dict(radius=c["R"], vertices=V, triangles=T, A0=c["A"], **c["kw"])
    v = c["variant"] | OVERLAP
    print(f"case {case}: L={L} nv={len(V)} FP64, variant {v}", flush=True)
    sim = ib.Simulation(L, storage="f64", **kw, **c.get("sim", {}))
    sim.set_variant(v)
    ref = oracle.Oracle(L, **kw)
    sim.step(c["A"], c["steps"])
    ref.step(c["A"], c["steps"])
    _compare(sim, ref, **F64_TOL)
    sim.close()
    ref.close()


def _ou_case(n):
    L = (48, 48, 48)
    V, T = icosphere(3, 8.0, box_center(L))
    table = ou_gradient_table(n + 1, 50.0, 4e-3, seed=23)
    kw = dict(tau=0.9, sigma=(1 / 6) * 4e-3 * 8.0 / 0.1, radius=8.0, vertices=V, triangles=T, A0=table[0])
    return L, kw, table


def _run(ib, L, kw, table, v, **sim_kw):
    sim = ib.Simulation(L, storage="f32", **kw, **sim_kw)
    sim.set_variant(v)
    for k in range(3):  # three calls: each starts and ends without the overlap
        sim.step_table(table[1 + 100 * k:101 + 100 * k])
    rho, u = sim.fields()
    out = (sim.vertices(), rho, u, sim.observables()["D"])
    sim.close()
    return out


@pytest.mark.parametrize("variant", [33, 57, 2 | 8 | 32])
def test_f32_equals_the_plain_step(ib, variant):
    """With the deterministic spreading both runs are reproducible bit for bit,
    so the overlapped one must equal the plain one exactly."""
    L, kw, table = _ou_case(300)
    print(f"case 48^3 FP32 deterministic, 300 OU steps, variant {variant} with and without bit 7", flush=True)
    r0, rho0, u0, D0 = _run(ib, L, kw, table, variant, deterministic=True)
    r1, rho1, u1, D1 = _run(ib, L, kw, table, variant | OVERLAP, deterministic=True)
    print(f"  max|dr| {np.abs(r0 - r1).max():.1e}, max|du| {np.abs(u0 - u1).max():.1e}, D {D0:.6f}", flush=True)
    assert np.array_equal(r0, r1)
    assert np.array_equal(rho0, rho1) and np.array_equal(u0, u1)
    assert D0 == D1


def test_f32_atomics_agree_with_the_plain_step(ib):
    """With the spreading's float atomics the order of the additions varies
    from run to run: equal to FP32 rounding, at the bars of the deterministic
    spreading against the atomics."""
    L, kw, table = _ou_case(300)
    print("case 48^3 FP32 atomics, 300 OU steps, variant 57 with and without bit 7", flush=True)
    r0, _, u0, D0 = _run(ib, L, kw, table, 57)
    r1, _, u1, D1 = _run(ib, L, kw, table, 57 | OVERLAP)
    dr = np.abs(r0 - r1).max()
    du = np.abs(u0 - u1).max() / np.abs(u0).max()
    print(f"  max|dr| {dr:.2e}, max|du|/max|u| {du:.2e}, dD/D {abs(D0 - D1) / D0:.2e}", flush=True)
    assert dr <= 2e-5 and du <= 2e-4 and abs(D0 - D1) <= 1e-5 * D0


def test_timing_counts_each_sweep_once(ib):
    L, kw, table = _ou_case(40)
    sim = ib.Simulation(L, storage="f32", **kw)
    sim.set_variant(33 | OVERLAP)
    sim.timing(True)
    sim.step_table(table[1:41])
    ms, n = sim.timing_read()
    print(f"case 48^3 timing: {n} sweeps, {ms:.3f} ms", flush=True)
    assert n == 40 and ms > 0
    sim.close()


def test_ensemble_refuses_the_overlap(ib):
    L = (24, 24, 24)
    V, T = icosphere(2, 3.0, box_center(L))
    cfg = dict(L=L, tau=0.9, sigma=0.02, radius=3.0, vertices=V, triangles=T)
    ens = ib.Ensemble([cfg, cfg])
    ens.set_variant(33)
    with pytest.raises(ib.IbmLbError) as e:
        ens.set_variant(33 | OVERLAP)
    assert e.value.code == ib.EINVAL
    ens.close()
