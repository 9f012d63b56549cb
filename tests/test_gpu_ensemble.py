"""GPU ensembles: independent droplets advanced by batched launches.

Each member of a heterogeneous ensemble (different box sizes, periodicity,
tau, sigma, meshes and gradient tables) is compared with the FP64 oracle run
on its own, and FP32 ensembles with the same members run one at a time.
"""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere, ou_gradient_table

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01161_amd import ibmlb
    ibmlb.lib()
    return ibmlb


def _members():
    out = []
    specs = [((16, 16, 16), (0, 0, 0), 0.9, 0.02, 3.0, 2, None),
             ((20, 14, 18), (0, 0, 0), 1.0, 0.01, 2.6, 2, None),
             ((12, 13, 16), (1, 1, 1), 0.8, 0.03, 2.5, 2, (0.3, 12.6, 0.0)),
             ((13, 9, 11), (0, 0, 0), 0.7, 0.0, 1.0, None, None)]
    for L, per, tau, sigma, R, level, centre in specs:
        kw = dict(L=L, periodic=per, tau=tau, sigma=sigma, radius=R)
        if level is not None:
            V, T = icosphere(level, R, box_center(L) if centre is None else centre)
            kw.update(vertices=V, triangles=T)
        out.append(kw)
    return out


def _tables(n, nsteps, scale=3e-3):
    tabs = np.stack([ou_gradient_table(nsteps, 15.0, scale, seed=100 + i) for i in range(n)])
    if n > 2:
        tabs[2] = 0.0  # the periodic member has no walls to impose a gradient
    return tabs


def test_ensemble_wet_walls_match_oracle_fp64(ib):
    """Members with the wet-node walls (two of them, one with a droplet) beside
    link-wall and periodic members, FP64 against the oracle."""
    members = _members()
    members[0]["walls"] = "wet"
    members[3]["walls"] = "wet"
    tabs = _tables(len(members), 20)
    for i, m in enumerate(members):
        m["A0"] = tabs[i, 0]
    ens = ib.Ensemble(members, storage="f64")
    ens.step(tabs[:, :9])
    ens.step(tabs[:, 9:])
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
        du = np.abs(u_g - u_r).max() / max(np.abs(u_r).max(), 1e-30)
        print(f"  member {i} ({m.get('walls', 'link')} walls): max|du|/max|u| {du:.1e}", flush=True)
        assert du <= 1e-11, i
        assert np.abs(rho_g - rho_r).max() < 1e-13, i
        ref.close()
    ens.close()


def test_ensemble_members_match_oracle_fp64(ib):
    members = _members()
    tabs = _tables(len(members), 25)
    for i, m in enumerate(members):
        m["A0"] = tabs[i, 0]
    ens = ib.Ensemble(members, storage="f64")
    ens.step(tabs[:, :12])
    ens.step(tabs[:, 12:])
    obs = ens.observables()
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
        orf = ref.observables()
        assert obs[i]["step"] == 25
        assert abs(obs[i]["mass"] - orf["mass"]) <= 1e-12 * orf["mass"], i
        if mem.nv:
            assert abs(obs[i]["D"] - orf["D"]) < 1e-10, i
            assert obs[i]["reg_iters"] == orf["reg_iters"], i


def test_ensemble_equals_solo_runs_fp32(ib):
    members = _members()[:3]
    tabs = _tables(len(members), 30)
    for i, m in enumerate(members):
        m["A0"] = tabs[i, 0]
    ens = ib.Ensemble(members, storage="f32")
    ens.step(tabs)
    for i, m in enumerate(members):
        kw = dict(m)
        L, tau = kw.pop("L"), kw.pop("tau")
        solo = ib.Simulation(L, tau, storage="f32", **kw)
        solo.step_table(tabs[i])
        # same kernels, same arithmetic; only the order of float atomics differs
        assert np.abs(ens.member(i).vertices() - solo.vertices()).max() < 1e-5, i
        assert abs(ens.member(i).observables()["D"] - solo.observables()["D"]) < 1e-5, i


def test_ensemble_autotune_keeps_state(ib):
    members = _members()[:2]
    tabs = _tables(2, 20)
    for i, m in enumerate(members):
        m["A0"] = tabs[i, 0]
    a = ib.Ensemble(members, storage="f64")
    b = ib.Ensemble(members, storage="f64")
    a.step(tabs[:, :10])
    b.step(tabs[:, :10])
    b.autotune(3)
    a.step(tabs[:, 10:])
    b.step(tabs[:, 10:])
    for i in range(2):
        assert np.abs(a.member(i).vertices() - b.member(i).vertices()).max() < 1e-12


def test_ensemble_rejects_mixed_storage(ib):
    import ctypes as C
    members = _members()[:2]
    cfgs = (ib.Config * 2)()
    keep = []
    for i, (m, st) in enumerate(zip(members, ("f32", "f64"))):
        kw = dict(m)
        cfg, k = ib.make_config(kw.pop("L"), kw.pop("tau"), storage=st, **kw)
        cfgs[i] = cfg
        keep.append(k)
    h = C.c_void_p()
    assert ib.lib().ibm_lb_batch_init(cfgs, 2, None, C.byref(h)) == ib.EINVAL


def _graph_vs_launches(ib, members, storage, tabs, chunks, graph_steps):
    """Member states after each chunk, with graph replays and with plain launches."""
    out = []
    for g in (graph_steps, 0):
        ens = ib.Ensemble(members, storage=storage)
        ens.set_graph(g)
        states, obs = [], []
        done = 0
        for c in chunks:
            ens.step(tabs[:, done:done + c])
            done += c
            # synchronising reads between replays
            obs.append(ens.observables())
            states.append([ens.member(i).save().cpu().numpy().copy() for i in range(len(members))])
        ens.close()
        out.append((states, obs))
    return out


def test_ensemble_graph_replays_match_launches(ib):
    # lattice-only members: no atomics, so graph replays and plain launches
    # must agree bit for bit after every call (chunks mix whole graphs, a
    # remainder of plain launches and an odd count that flips the parity)
    specs = [((16, 12, 10), (0, 0, 0)), ((20, 9, 8), (1, 0, 0)), ((9, 9, 8), (0, 1, 1))]
    members = []
    for i, (L, per) in enumerate(specs):
        members.append(dict(L=L, periodic=per, tau=0.85))
    tabs = _tables(len(specs), 64, scale=2e-3)
    tabs[1:] = 0.0  # the periodic members carry no gradient
    for m, t in zip(members, tabs):
        m["A0"] = t[0]
    (sg, _), (sl, _) = _graph_vs_launches(ib, members, "f32", tabs, [8, 8, 13, 9, 16], 8)
    for call, (a, b) in enumerate(zip(sg, sl)):
        for i in range(len(specs)):
            assert np.array_equal(a[i], b[i]), f"call {call}, member {i}"
    # the same with the wet-node walls on the member walled on every face
    members[0]["walls"] = "wet"
    (sg, _), (sl, _) = _graph_vs_launches(ib, members, "f32", tabs, [8, 8, 13, 9, 16], 8)
    for call, (a, b) in enumerate(zip(sg, sl)):
        for i in range(len(specs)):
            assert np.array_equal(a[i], b[i]), f"wet walls: call {call}, member {i}"


def test_ensemble_graph_replays_with_droplets(ib):
    members = _members()
    tabs = _tables(len(members), 40)
    for i, m in enumerate(members):
        m["A0"] = tabs[i, 0]
    (sg, og), (sl, ol) = _graph_vs_launches(ib, members, "f64", tabs, [8, 8, 11, 8], 8)
    for call in range(len(og)):
        for i, m in enumerate(members):
            if "vertices" in m:
                assert abs(og[call][i]["D"] - ol[call][i]["D"]) <= 1e-11
                assert og[call][i]["reg_iters"] == ol[call][i]["reg_iters"]
            assert abs(og[call][i]["mass"] - ol[call][i]["mass"]) <= 1e-9 * abs(ol[call][i]["mass"])
