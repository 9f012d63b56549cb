"""GPU: every lattice-kernel variant computes the same step.

The variants differ only in how nodes map to work-groups (linear blocks, an
XCD-grouped block order, whole x-rows per work-group with the x-moving
populations exchanged through LDS), in cache hints and in where populations
are stored between steps (two copies, or one copy streamed in place with
alternating index mappings), never in the per-node arithmetic. Without a
droplet the step has no atomics, so every variant must reproduce the default
variant's state bit for bit, on boxes with walls,
periodic axes, rows longer than a work-group and ragged last work-groups.
With a droplet, a few variants are checked against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere

pytestmark = pytest.mark.gpu

NVAR = 32
ROWS = 16
BS = (128, 256, 512, 64)


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


def _row_ok(v, Lx):
    return not (v & ROWS) or Lx <= 512


def _state_after(ib, L, periodic, storage, variant, A, nsteps, populations=2):
    sim = ib.Simulation(L, tau=0.8, periodic=periodic, storage=storage, A0=A, init="linear",
                        populations=populations)
    sim.set_variant(variant)
    sim.step(A, nsteps)
    out = sim.save().cpu().numpy().copy()
    sim.close()
    return out


BOXES = [((13, 9, 11), (0, 0, 0)),     # odd sizes, walls on every side
         ((16, 12, 10), (1, 0, 0)),    # periodic along x (rows wrap through LDS)
         ((40, 8, 9), (1, 0, 1)),      # several rows per work-group, ragged tail
         ((130, 8, 8), (0, 1, 0)),     # a row longer than 128 threads
         ((8, 8, 8), (1, 1, 1))]       # fully periodic


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16dev"])
@pytest.mark.parametrize("L,periodic", BOXES)
def test_lattice_variants_bit_identical(ib, storage, L, periodic):
    A = _traceless(2e-3, 7) if not all(periodic) else np.zeros(9)
    print(f"case L={L} periodic={periodic} storage={storage}", flush=True)
    ref = _state_after(ib, L, periodic, storage, 1, A, 7)
    for v in range(NVAR):
        if not _row_ok(v, L[0]):
            continue
        got = _state_after(ib, L, periodic, storage, v, A, 7)
        assert np.array_equal(got, ref), f"variant {v} differs from variant 1"


def test_row_layout_rejects_long_rows(ib):
    sim = ib.Simulation((520, 8, 8), tau=0.8, storage="f32", init="rest")
    with pytest.raises(ib.IbmLbError):
        sim.set_variant(ROWS | 1)
    sim.set_variant(8 | 1)  # linear layouts take any row length
    sim.step(np.zeros(9), 2)
    sim.close()
    sim = ib.Simulation((8, 8, 8), tau=0.8, storage="f32")
    for bad in (4 * NVAR, -1, AA | ROWS | 1):
        with pytest.raises(ib.IbmLbError):
            sim.set_variant(bad)
    sim.close()


SPLIT = 32  # smoothing finish as a launch of its own
AA = 64     # in-place streaming, one population copy


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16dev"])
@pytest.mark.parametrize("L,periodic", BOXES)
def test_in_place_variants_bit_identical(ib, storage, L, periodic):
    # an odd and an even number of in-place steps (the odd count leaves the
    # copy in the second mapping, settled by save)
    A = _traceless(2e-3, 7) if not all(periodic) else np.zeros(9)
    print(f"case in-place L={L} periodic={periodic} storage={storage}", flush=True)
    for nsteps in (7, 8):
        ref = _state_after(ib, L, periodic, storage, 1, A, nsteps)
        for v in range(ROWS):
            got = _state_after(ib, L, periodic, storage, AA | v, A, nsteps)
            assert np.array_equal(got, ref), f"variant {AA | v}, {nsteps} steps"


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16dev"])
@pytest.mark.parametrize("L,periodic", BOXES)
def test_one_copy_handles_bit_identical(ib, storage, L, periodic):
    # one population copy: in-place variants only, the same states
    A = _traceless(2e-3, 7) if not all(periodic) else np.zeros(9)
    print(f"case one copy L={L} periodic={periodic} storage={storage}", flush=True)
    for nsteps in (7, 8):
        ref = _state_after(ib, L, periodic, storage, 1, A, nsteps)
        for v in (AA, AA | SPLIT | 1, AA | 8 | 4):
            got = _state_after(ib, L, periodic, storage, v, A, nsteps, populations=1)
            assert np.array_equal(got, ref), f"variant {v}, {nsteps} steps"


def test_one_copy_handle_rules(ib):
    A = _traceless(2e-3, 8)
    sim = ib.Simulation((12, 10, 9), tau=0.8, storage="f32", A0=A, populations=1)
    for bad in (1, SPLIT | 1, ROWS | 1):
        with pytest.raises(ib.IbmLbError):
            sim.set_variant(bad)
    sim.step(A, 3)
    before = sim.save().cpu().numpy().copy()
    v = sim.autotune(2)
    assert v & AA
    assert np.array_equal(sim.save().cpu().numpy(), before)  # the tuner restores the state
    sim.close()
    with pytest.raises(ib.IbmLbError):
        ib.Ensemble([dict(L=(8, 8, 8), tau=0.8, populations=1)], storage="f32")


def test_in_place_switching_mid_run(ib):
    # in-place runs of odd and even lengths interleaved with two-copy runs,
    # row-layout runs and reads, against one two-copy run
    L, periodic = (16, 12, 10), (1, 0, 0)
    A = _traceless(2e-3, 9)
    ref = _state_after(ib, L, periodic, "f32", 1, A, 23)
    sim = ib.Simulation(L, tau=0.8, periodic=periodic, storage="f32", A0=A, init="linear")
    for v, k in [(AA | 1, 3), (1, 4), (AA | 8 | 1, 5), (ROWS | 1, 1), (AA, 2), (AA | 1, 1), (9, 2), (AA | 3, 5)]:
        sim.set_variant(v)
        sim.step(A, k)
        if v == AA | 1:
            sim.fields()  # a read between in-place steps (after an odd count in total)
    got = sim.save().cpu().numpy().copy()
    sim.close()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("variant,nsteps", [(1, 30), (9, 30), (ROWS | 1, 30), (ROWS | 8, 30), (ROWS | 4 | 8 | 1, 30),
                                            (ROWS | 6, 30), (SPLIT | 1, 30), (SPLIT | ROWS | 8 | 1, 30),
                                            (AA | SPLIT | 1, 30), (AA | SPLIT | 8 | 1, 29), (AA | 4, 31)])
def test_droplet_variants_match_oracle(ib, variant, nsteps):
    L = (19, 17, 21)
    A = _traceless(3e-3, 2)
    V, T = icosphere(2, 3.2, box_center(L))
    kw = dict(tau=0.9, sigma=0.02, radius=3.2, vertices=V, triangles=T, A0=A)
    print(f"case droplet L={L} variant={variant} steps={nsteps}", flush=True)
    sim = ib.Simulation(L, storage="f64", **kw)
    sim.set_variant(variant)
    ref = oracle.Oracle(L, **kw)
    sim.step(A, nsteps)
    ref.step(A, nsteps)
    dr = np.abs(sim.vertices() - ref.vertices()).max()
    rho_g, u_g = sim.fields()
    rho_r, u_r = ref.fields()
    du = np.abs(u_g - u_r).max() / np.abs(u_r).max()
    assert dr <= 1e-11, f"max |dr| = {dr:.3e}"
    assert du <= 1e-11, f"max|du|/max|u| = {du:.3e}"
    assert np.abs(rho_g - rho_r).max() <= 1e-13
    sim.close()


def _ensemble_states(ib, members, tabs, variant):
    ens = ib.Ensemble(members, storage="f32")
    ens.set_variant(variant)
    ens.step(tabs)
    out = [ens.member(i).save().cpu().numpy().copy() for i in range(len(members))]
    ens.close()
    return out


def test_droplet_one_copy_matches_oracle(ib):
    L = (19, 17, 21)
    A = _traceless(3e-3, 2)
    V, T = icosphere(2, 3.2, box_center(L))
    kw = dict(tau=0.9, sigma=0.02, radius=3.2, vertices=V, triangles=T, A0=A)
    sim = ib.Simulation(L, storage="f64", populations=1, **kw)
    ref = oracle.Oracle(L, **kw)
    for k in (5, 8, 18):  # a read after every call, odd and even totals
        sim.step(A, k)
        ref.step(A, k)
        assert np.abs(sim.vertices() - ref.vertices()).max() <= 1e-11
        rho_g, u_g = sim.fields()
        rho_r, u_r = ref.fields()
        assert np.abs(u_g - u_r).max() <= 1e-11 * np.abs(u_r).max()
        assert np.abs(rho_g - rho_r).max() <= 1e-13
        assert abs(sim.observables()["D"] - ref.observables()["D"]) <= 1e-11
    sim.close()


def test_droplet_in_place_adjoint_unchanged(ib):
    # the forward run in place, then one adjoint segment from its checkpoint:
    # the same objective and gradients as with two copies (and with one copy,
    # where the recompute returns to natural order after every step)
    L = (19, 17, 21)
    A = np.tile(_traceless(3e-3, 4), (7, 1))
    V, T = icosphere(2, 3.2, box_center(L))
    out = []
    for v, pops in ((SPLIT | 1, 2), (AA | SPLIT | 1, 2), (AA | SPLIT, 1)):
        print(f"case adjoint after variant {v}, {pops} copies", flush=True)
        sim = ib.Simulation(L, tau=0.9, sigma=0.02, radius=3.2, vertices=V, triangles=T, A0=A[0], storage="f64",
                            populations=pops)
        sim.set_variant(v)
        ck = sim.save()
        sim.step_table(A)
        D, rbar = sim.objective_grad()
        _, rb0, dA, ds = sim.adjoint_segment(ck, A, None, rbar)
        out.append((D, rb0.cpu().numpy(), dA.cpu().numpy(), float(ds[0])))
        sim.close()
    D1, r1, a1, s1 = out[0]
    for D2, r2, a2, s2 in out[1:]:
        # equal up to the order of the float atomics of spreading (run to run)
        assert abs(D1 - D2) < 1e-13
        assert abs(s1 - s2) <= 1e-10 * abs(s1)
        assert np.abs(r1 - r2).max() <= 1e-10 * np.abs(r1).max()
        assert np.abs(a1 - a2).max() <= 1e-10 * np.abs(a1).max()


def test_ensemble_variants_bit_identical(ib):
    # lattice-only members of mixed sizes and periodicity: rows of 48, 20,
    # 96 and 9 nodes, so the row layout packs different row counts per
    # work-group for each member
    specs = [((48, 8, 9), (0, 0, 0)), ((20, 14, 9), (1, 0, 0)), ((96, 8, 8), (0, 1, 1)), ((9, 9, 8), (0, 0, 0))]
    members = []
    tabs = np.zeros((len(specs), 6, 9))
    for i, (L, per) in enumerate(specs):
        A = _traceless(2e-3, 20 + i)
        tabs[i, :] = A
        members.append(dict(L=L, periodic=per, tau=0.85, A0=A))
    print("case ensemble variants", flush=True)
    ens = ib.Ensemble(members, storage="f32")
    with pytest.raises(ib.IbmLbError):
        ens.set_variant(AA | 1)  # single droplets only
    ens.close()
    ref = _ensemble_states(ib, members, tabs, 1)
    for v in range(NVAR):
        if v & ROWS and BS[(v >> 1) & 3] < 96:
            ens = ib.Ensemble(members, storage="f32")
            with pytest.raises(ib.IbmLbError):
                ens.set_variant(v)
            ens.close()
            continue
        got = _ensemble_states(ib, members, tabs, v)
        for i in range(len(specs)):
            assert np.array_equal(got[i], ref[i]), f"variant {v}, member {i}"
