"""GPU MRT collision against the FP64 oracle's MRT (same basis and rates),
with two population copies and with one (in place), and in ensembles (each
member with its own rates); its variants (linear, row and in-place layouts)
bit-identical to each other on a lattice-only box; its limits (ensembles of
one collision, no adjoint)."""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere

pytestmark = pytest.mark.gpu

ROWS, SPLIT, AA = 16, 32, 64


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


def _case(L=(19, 17, 21)):
    A = _traceless(3e-3, 2)
    V, T = icosphere(2, 3.2, box_center(L))
    return A, dict(tau=0.9, sigma=0.02, radius=3.2, vertices=V, triangles=T, A0=A)


@pytest.mark.parametrize("storage,mrt_s,tol", [
    ("f64", None, (1e-11, 1e-11, 1e-13)),
    ("f64", [1.5, 1.1, 1.7, 1.3, 1.0], (1e-11, 1e-11, 1e-13)),
    ("f32", None, (2e-5, 2e-4, 1e-6)),
])
def test_mrt_droplet_matches_oracle(ib, storage, mrt_s, tol):
    L = (19, 17, 21)
    A, kw = _case(L)
    print(f"case MRT droplet {storage} rates {mrt_s}", flush=True)
    sim = ib.Simulation(L, storage=storage, collision="mrt", mrt_s=mrt_s, **kw)
    ref = oracle.Oracle(L, collision="mrt", mrt_s=mrt_s, **kw)
    sim.step(A, 30)
    ref.step(A, 30)
    dr = np.abs(sim.vertices() - ref.vertices()).max()
    rho_g, u_g = sim.fields()
    rho_r, u_r = ref.fields()
    du = np.abs(u_g - u_r).max() / np.abs(u_r).max()
    drho = np.abs(rho_g - rho_r).max()
    print(f"  max|dr| {dr:.2e}  du {du:.2e}  drho {drho:.2e}", flush=True)
    assert dr <= tol[0] and du <= tol[1] and drho <= tol[2]
    assert abs(sim.observables()["mass"] - ref.observables()["mass"]) <= 1e-9 * ref.observables()["mass"]
    sim.close()
    ref.close()


@pytest.mark.parametrize("pops,variant,steps", [(1, AA | SPLIT | 1, 31), (2, AA | SPLIT | 8, 30)])
def test_mrt_in_place_matches_oracle(ib, pops, variant, steps):
    """In-place streaming with MRT: one population copy (an odd step count
    leaves it in the odd mapping until the reads), or in-place variants on a
    two-copy handle."""
    L = (19, 17, 21)
    A, kw = _case(L)
    rates = [1.5, 1.1, 1.7, 1.3, 1.0]
    print(f"case MRT in place: populations {pops}, variant {variant}, {steps} steps", flush=True)
    sim = ib.Simulation(L, storage="f64", collision="mrt", mrt_s=rates, populations=pops, **kw)
    sim.set_variant(variant)
    ref = oracle.Oracle(L, collision="mrt", mrt_s=rates, **kw)
    sim.step(A, steps)
    ref.step(A, steps)
    dr = np.abs(sim.vertices() - ref.vertices()).max()
    rho_g, u_g = sim.fields()
    rho_r, u_r = ref.fields()
    du = np.abs(u_g - u_r).max() / np.abs(u_r).max()
    drho = np.abs(rho_g - rho_r).max()
    print(f"  max|dr| {dr:.2e}, max|du|/max|u| {du:.2e}, max|drho| {drho:.2e}", flush=True)
    assert dr <= 1e-11 and du <= 1e-11 and drho <= 1e-13
    sim.close()
    ref.close()


def test_mrt_equal_rates_match_bgk(ib):
    L = (19, 17, 21)
    A, kw = _case(L)
    s = 1 / kw["tau"]
    out = []
    for coll, rates in (("bgk", None), ("mrt", [s] * 5)):
        sim = ib.Simulation(L, storage="f64", collision=coll, mrt_s=rates, **kw)
        sim.step(A, 30)
        out.append((sim.vertices(), sim.fields()[1]))
        sim.close()
    assert np.abs(out[0][0] - out[1][0]).max() <= 1e-11
    assert np.abs(out[0][1] - out[1][1]).max() <= 1e-11 * np.abs(out[0][1]).max()


def test_mrt_variants_bit_identical(ib):
    L, A = (40, 9, 11), _traceless(2e-3, 3)
    states = {}
    for v in (1, 0, 3, 5, 7, 8, 9, SPLIT | 1, ROWS | 1, ROWS | 9, ROWS, ROWS | 3, AA | 1, AA | 3, AA | 8 | 1):
        sim = ib.Simulation(L, 0.8, storage="f32", A0=A, collision="mrt", periodic=(1, 0, 0))
        sim.set_variant(v)
        sim.step(A, 7)
        states[v] = sim.save().cpu().numpy().copy()
        sim.close()
    for v, st in states.items():
        assert np.array_equal(st, states[1]), f"variant {v}"


def test_mrt_limits(ib):
    L = (12, 10, 9)
    A, kw = _case((19, 17, 21))
    sim = ib.Simulation(L, 0.8, storage="f32", A0=A, collision="mrt", populations=1)
    with pytest.raises(ib.IbmLbError):
        sim.set_variant(1)  # one copy: in-place variants only
    v = sim.autotune(2)
    assert v & AA
    sim.close()
    with pytest.raises(ib.IbmLbError):  # BGK and MRT members together
        ib.Ensemble([dict(L=(8, 8, 8), tau=0.8, collision="mrt"), dict(L=(8, 8, 8), tau=0.8)], storage="f32")
    sim = ib.Simulation((19, 17, 21), storage="f64", collision="mrt", **kw)
    sim.step(A, 2)
    with pytest.raises(ib.IbmLbError):
        sim.objective_grad()
    sim.close()


def test_mrt_ensemble_matches_oracle(ib):
    """MRT members with different rates, with and without a droplet, through
    the batched kernels (the autotuner's choice and the row layout) against
    the oracle in FP64."""
    from paper_2403_01161_amd.inputs import ou_gradient_table
    specs = [((16, 16, 16), 0.9, 0.02, 3.0, [1.5, 1.1, 1.7, 1.3, 1.0]),
             ((20, 14, 18), 1.0, 0.01, 2.6, None),
             ((13, 9, 11), 0.7, 0.0, None, [1.2, 1.9, 1.1, 1.6, 1.4])]
    members = []
    for i, (L, tau, sigma, R, rates) in enumerate(specs):
        kw = dict(L=L, tau=tau, sigma=sigma, collision="mrt", mrt_s=rates)
        if R is not None:
            V, T = icosphere(2, R, box_center(L))
            kw.update(vertices=V, triangles=T, radius=R)
        members.append(kw)
    tabs = np.stack([ou_gradient_table(25, 15.0, 3e-3, seed=200 + i) for i in range(len(members))])
    for i, m in enumerate(members):
        m["A0"] = tabs[i, 0]
    for variant in (None, ROWS | 1):
        print(f"case MRT ensemble, variant {variant}", flush=True)
        ens = ib.Ensemble(members, storage="f64")
        if variant is not None:
            ens.set_variant(variant)
        ens.step(tabs[:, :12])
        ens.step(tabs[:, 12:])
        for i, m in enumerate(members):
            kw = dict(m)
            L = kw.pop("L")
            ref = oracle.Oracle(L, **kw)
            ref.step_table(tabs[i])
            mem = ens.member(i)
            if mem.nv:
                assert np.abs(mem.vertices() - ref.vertices()).max() < 1e-11, i
            rho_g, u_g = mem.fields()
            rho_r, u_r = ref.fields()
            assert np.abs(u_g - u_r).max() <= 1e-11 * max(np.abs(u_r).max(), 1e-30), i
            assert np.abs(rho_g - rho_r).max() < 1e-13, i
            ref.close()
        ens.close()
