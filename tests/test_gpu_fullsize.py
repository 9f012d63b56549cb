"""GPU parity at the benchmarked sizes, in the launch configuration bench.py
times (the autotuner's variant), against the FP64 oracle.

* 128^3 single droplet (R 16, 10242 vertices, OU gradient), FP32 storage:
  every vertex and every node's rho and u after 12 steps; and after 8 steps
  with each option of the step (MRT collision, viscosity ratio 4, wet-node
  walls, deterministic spreading).
* 256^3 single droplet (R 32, 40962 vertices), FP32 storage: every vertex,
  and rho and u on every node of sampled z-planes (through the walls and the
  droplet) after 4 steps.
* The 64-droplet ensemble (boxes 48^3 / 64^3 / 96^3, 2562-vertex meshes), run
  batched with graph replays; members of each box size against their own
  oracle runs after 10 steps.

The oracle runs with the same seeded gradient tables; the tolerances are the
FP32-storage bars of the small parity tests (FP32 rounding of the stored
deviations and of the relative positions).
"""
import numpy as np
import pytest

import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL_R = 2e-5      # vertex positions, absolute lattice units
TOL_U = 2e-4      # max |du| / max |u|
TOL_RHO = 1e-6    # absolute density


@pytest.fixture(scope="module")
def ib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01161_amd import ibmlb
    ibmlb.lib()
    return ibmlb


def _single(ib, w, nsteps, planes=None, options=None, gpu_only=None):
    import bench
    from paper_2403_01161_amd.inputs import ou_gradient_table
    table = ou_gradient_table(nsteps + 1, w["corr"], w["G"], seed=w["seed"])
    kw = dict(tau=w["tau"], sigma=w["sigma"], radius=w["R"], vertices=w["V"], triangles=w["T"], A0=table[0],
              **(options or {}))
    print(f"case full size L={w['L']} nv={len(w['V'])} steps={nsteps} {options or ''} {gpu_only or ''}", flush=True)
    sim = ib.Simulation(w["L"], storage="f32", **kw, **(gpu_only or {}))
    variant = sim.autotune(3)
    print(f"  variant {variant}: {bench.describe_variant(variant)}", flush=True)
    sim.step_table(table[:nsteps])
    ref = oracle.Oracle(w["L"], **kw)
    ref.step_table(table[:nsteps])
    dr = np.abs(sim.vertices() - ref.vertices()).max()
    assert dr <= TOL_R, f"max |dr| = {dr:.3e}"
    rho_g, u_g = sim.fields()
    rho_r, u_r = ref.fields()
    if planes is not None:
        rho_g, rho_r = rho_g[planes], rho_r[planes]
        u_g, u_r = u_g[:, planes], u_r[:, planes]
    du = np.abs(u_g - u_r).max() / np.abs(u_r).max()
    drho = np.abs(rho_g - rho_r).max()
    print(f"  max|dr| {dr:.2e}  max|du|/max|u| {du:.2e}  max|drho| {drho:.2e}", flush=True)
    assert du <= TOL_U and drho <= TOL_RHO
    og, orf = sim.observables(), ref.observables()
    assert abs(og["D"] - orf["D"]) <= 1e-3 * max(orf["D"], 1e-6) + 1e-7
    assert abs(og["mass"] - orf["mass"]) <= 1e-9 * orf["mass"]
    sim.close()


def test_single_droplet_128(ib):
    import bench
    _single(ib, bench.workload("f32"), 12)


@pytest.mark.parametrize("options,gpu_only", [
    (dict(collision="mrt"), None),
    (dict(chi=4.0), None),
    (dict(walls="wet"), None),
    (None, dict(deterministic=True)),
], ids=["mrt", "chi4", "wet_walls", "deterministic"])
def test_single_droplet_128_options(ib, options, gpu_only):
    """The 128^3 droplet with each option of the step (MRT collision,
    viscosity ratio 4, wet-node walls, deterministic spreading) in the
    autotuner's variant, after 8 steps."""
    import bench
    _single(ib, bench.workload("f32"), 8, options=options, gpu_only=gpu_only)


def test_single_droplet_256_sampled_planes(ib):
    import bench
    w = bench.precision_workload()
    # z-planes: both walls, through the droplet, and between
    _single(ib, w, 4, planes=[0, 1, 64, 100, 127, 128, 156, 200, 254, 255])


def test_ensemble_members_full_size(ib):
    import bench
    from paper_2403_01161_amd.inputs import ou_gradient_table
    members, rms = bench.ensemble_workload()
    n, nsteps = len(members), 10
    tabs = np.stack([ou_gradient_table(nsteps, 2000.0, rms[d], seed=1000 + d) for d in range(n)])
    for d in range(n):
        members[d]["A0"] = tabs[d, 0]
    print(f"case ensemble of {n} droplets, {nsteps} steps", flush=True)
    ens = ib.Ensemble(members, storage="f32")
    ens.autotune(2)
    ens.set_graph(4)
    ens.step(tabs)
    # one member of each box size
    picks = {}
    for d, m in enumerate(members):
        picks.setdefault(m["L"][0], d)
    for side, d in sorted(picks.items()):
        kw = dict(members[d])
        L = kw.pop("L")
        ref = oracle.Oracle(L, **kw)
        ref.step_table(tabs[d])
        mem = ens.member(d)
        dr = np.abs(mem.vertices() - ref.vertices()).max()
        rho_g, u_g = mem.fields()
        rho_r, u_r = ref.fields()
        du = np.abs(u_g - u_r).max() / np.abs(u_r).max()
        drho = np.abs(rho_g - rho_r).max()
        print(f"  member {d} ({side}^3): max|dr| {dr:.2e}  du {du:.2e}  drho {drho:.2e}", flush=True)
        assert dr <= TOL_R and du <= TOL_U and drho <= TOL_RHO
    ens.close()
