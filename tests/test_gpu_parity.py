"""GPU parity: the HIP library (through its C-ABI) against the FP64 oracle.

Element-wise comparison of vertex positions and of the rho/u fields on the
same seeded inputs, at sizes that span several 8^3 tiles with ragged tails,
for FP64 storage (round-off tolerance) and FP32 storage (tolerance from FP32
rounding of populations stored as deviations).
"""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere, simple_shear

pytestmark = pytest.mark.gpu


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


def _pair(ib, storage, L, R=None, level=2, center=None, **kw):
    if R is not None:
        V, T = icosphere(level, R, box_center(L) if center is None else center)
        kw.update(vertices=V, triangles=T, radius=R)
    print(f"case L={L} storage={storage} nv={0 if R is None else len(kw['vertices'])}", flush=True)
    init = kw.pop("init", "linear")
    sim = ib.Simulation(L, storage=storage, init=init, **kw)
    ref = oracle.Oracle(L, init_rest=(init == "rest"), **kw)
    return sim, ref


def _compare(sim, ref, tol_r, tol_u, tol_rho):
    if sim.nv:
        dr = np.abs(sim.vertices() - ref.vertices()).max()
        assert dr <= tol_r, f"max |dr| = {dr:.3e}"
    rho_g, u_g = sim.fields()
    rho_r, u_r = ref.fields()
    du = np.abs(u_g - u_r).max() / max(np.abs(u_r).max(), 1e-30)
    drho = np.abs(rho_g - rho_r).max()
    assert du <= tol_u, f"max|du|/max|u| = {du:.3e}"
    assert drho <= tol_rho, f"max |drho| = {drho:.3e}"
    return du


F64_TOL = dict(tol_r=1e-11, tol_u=1e-11, tol_rho=1e-13)
# FP32 populations (deviations) and FP32 positions: rounding ~ 6e-8 relative
F32_TOL = dict(tol_r=2e-5, tol_u=2e-4, tol_rho=1e-6)


@pytest.mark.parametrize("storage,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_lattice_only_walls_ragged(ib, storage, tol):
    A = _traceless(2e-3, 1)
    sim, ref = _pair(ib, storage, (13, 9, 11), tau=0.8, A0=A, init="linear")
    sim.step(A, 40)
    ref.step(A, 40)
    _compare(sim, ref, **tol)


@pytest.mark.parametrize("storage,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_patch_windows_beyond_capacity(ib, storage, tol):
    """A coarse mesh on a large droplet (162 vertices in three patches, R 9):
    each patch's stencils span about 22 x 22 x 13 nodes, beyond the LDS
    windows of the interpolation (2048 nodes) and of the spreading (1456), so
    both kernels take their direct global-memory paths."""
    L = (27, 26, 28)
    A = _traceless(2e-3, 5)
    sim, ref = _pair(ib, storage, L, R=9.0, level=2, tau=0.9, sigma=0.02, A0=A)
    sim.step(A, 25)
    ref.step(A, 25)
    _compare(sim, ref, **tol)


@pytest.mark.parametrize("storage,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_droplet_walls_ragged(ib, storage, tol):
    L = (19, 17, 21)
    A = _traceless(3e-3, 2)
    sim, ref = _pair(ib, storage, L, R=3.2, level=2, tau=0.9, sigma=0.02, A0=A)
    sim.step(A, 30)
    ref.step(A, 30)
    _compare(sim, ref, **tol)


def test_droplet_periodic_wrap(ib):
    """Droplet centred on a periodic box corner: every stencil wraps."""
    L = (12, 13, 16)
    sim, ref = _pair(ib, "f64", L, R=2.5, level=2, center=(0.3, 12.6, 0.0), tau=0.8,
                     sigma=0.03, periodic=(1, 1, 1), init="rest")
    sim.step(np.zeros(9), 25)
    ref.step(np.zeros(9), 25)
    _compare(sim, ref, **F64_TOL)


def test_droplet_couette_mixed(ib):
    L = (16, 24, 16)
    A = simple_shear(2e-3)
    sim, ref = _pair(ib, "f64", L, R=4.0, level=3, tau=1.0, sigma=0.01, A0=A, periodic=(1, 0, 1))
    sim.step(A, 40)
    ref.step(A, 40)
    _compare(sim, ref, **F64_TOL)
    og, orf = sim.observables(), ref.observables()
    for key in ("volume", "D", "theta_deg", "beta"):
        assert abs(og[key] - orf[key]) <= 1e-9 * max(1.0, abs(orf[key])), key
    np.testing.assert_allclose(og["eigval"], orf["eigval"], rtol=1e-11)
    assert abs(og["mass"] - orf["mass"]) <= 1e-12 * orf["mass"]
    assert og["reg_iters"] == orf["reg_iters"]


def test_step_table_matches_oracle(ib):
    from paper_2403_01161_amd.inputs import ou_gradient_table
    L = (16, 16, 16)
    table = ou_gradient_table(30, 20.0, 4e-3, seed=9)
    sim, ref = _pair(ib, "f64", L, R=3.0, level=2, tau=0.9, sigma=0.02, A0=table[0])
    sim.step_table(table)
    ref.step_table(table)
    _compare(sim, ref, **F64_TOL)
    og, orf = sim.observables(), ref.observables()
    assert abs(og["beta"] - orf["beta"]) < 1e-9


def test_device_table_equals_host_table(ib):
    import torch
    from paper_2403_01161_amd.inputs import ou_gradient_table
    L = (16, 16, 16)
    table = ou_gradient_table(12, 20.0, 4e-3, seed=3)
    a, _ = _pair(ib, "f64", L, R=3.0, level=2, tau=0.9, sigma=0.02, A0=table[0])
    b, _ = _pair(ib, "f64", L, R=3.0, level=2, tau=0.9, sigma=0.02, A0=table[0])
    a.step_table(table)
    dev = torch.from_numpy(table).to("cuda:0")
    b.step_table(dev)
    np.testing.assert_allclose(a.vertices(), b.vertices(), rtol=0, atol=1e-13)


def test_no_smoothing_and_printed_sign(ib):
    L = (16, 16, 16)
    for kw in (dict(reg_max_iter=0), dict(reg_sign=-1)):
        sim, ref = _pair(ib, "f64", L, R=3.0, level=2, tau=0.9, sigma=0.02, **kw)
        sim.step(np.zeros(9), 15)
        ref.step(np.zeros(9), 15)
        _compare(sim, ref, **F64_TOL)


def test_checkpoint_roundtrip(ib):
    L = (16, 16, 16)
    A = _traceless(2e-3, 4)
    sim, _ = _pair(ib, "f64", L, R=3.0, level=2, tau=0.9, sigma=0.02, A0=A)
    other, _ = _pair(ib, "f64", L, R=3.0, level=2, tau=0.9, sigma=0.02, A0=A)
    sim.step(A, 20)
    ck = sim.save()
    sim.step(A, 20)
    other.load(ck)
    assert other.observables()["step"] == 20
    other.step(A, 20)
    np.testing.assert_allclose(other.vertices(), sim.vertices(), rtol=0, atol=1e-13)
    assert other.observables()["step"] == 40


def test_domain_error_is_sticky(ib):
    """An off-centre droplet in an extensional flow drifts outward until its
    stencil crosses a wall: EDOMAIN at the next synchronising call, and on
    every call after it."""
    L = (12, 12, 12)
    A = np.diag([5e-3, -2.5e-3, -2.5e-3]).ravel()
    sim, _ = _pair(ib, "f32", L, R=2.0, level=2, center=(7.0, 5.5, 5.5), tau=0.8, sigma=0.001,
                   A0=A)
    sim.step(A, 300)
    with pytest.raises(ib.IbmLbError) as e:
        sim.observables()
    assert e.value.code == ib.EDOMAIN
    with pytest.raises(ib.IbmLbError) as e:
        sim.step(A, 1)
    assert e.value.code == ib.EDOMAIN


@pytest.mark.parametrize("droplet", [False, True])
def test_nonfinite_error_is_sticky(ib, droplet):
    """A gradient far outside the lattice's range (wall speeds near 100 lattice
    units per step) drives densities non-positive and then non-finite. The
    kernels only raise the device flag and exit; ENONFINITE comes at the next
    synchronising call and on every call after it, and a new handle runs."""
    L = (12, 12, 12)
    A = np.zeros(9)
    A[1] = 20.0
    kw = dict(tau=0.8)
    if droplet:
        V, T = icosphere(2, 2.5, box_center(L))
        kw.update(sigma=0.01, radius=2.5, vertices=V, triangles=T)
    print(f"case nonfinite droplet={droplet}", flush=True)
    sim = ib.Simulation(L, storage="f32", **kw)
    sim.step(A, 20)
    with pytest.raises(ib.IbmLbError) as e:
        sim.observables()
    assert e.value.code == ib.ENONFINITE
    with pytest.raises(ib.IbmLbError) as e:
        sim.step(np.zeros(9), 1)
    assert e.value.code == ib.ENONFINITE
    sim.close()
    fresh = ib.Simulation(L, storage="f32", **kw)
    fresh.step(np.zeros(9), 5)
    assert np.isfinite(fresh.observables()["mass"])
    fresh.close()


@pytest.mark.parametrize("storage", ["f16dev", "bf16dev"])
def test_16bit_storage_soft_gate(ib, storage):
    L = (24, 24, 24)
    g = 2e-3
    A = simple_shear(g)
    kw = dict(tau=1.0, sigma=(1 / 6) * g * 4.0 / 0.1, A0=A)
    sim, ref = _pair(ib, storage, L, R=4.0, level=3, **kw)
    sim.step(A, 200)
    ref.step(A, 200)
    og, orf = sim.observables(), ref.observables()
    rho_g, u_g = sim.fields()
    assert np.isfinite(u_g).all()
    print(f"{storage}: D gpu {og['D']:.6f} oracle {orf['D']:.6f}")
    assert abs(og["D"] - orf["D"]) <= 0.05 * orf["D"]


@pytest.mark.slow
def test_plain_method_fp64_1000_steps(ib):
    """Plain-method workload in FP64: 32^3, tau 1, R = 5 (642 vertices),
    simple shear with Ca = 0.05, 1000 steps; D, theta, u, r, mass."""
    L = (32, 32, 32)
    g = 1e-3
    A = simple_shear(g)
    sim, ref = _pair(ib, "f64", L, R=5.0, level=3, tau=1.0, sigma=(1 / 6) * g * 5.0 / 0.05, A0=A)
    sim.step(A, 1000)
    ref.step(A, 1000)
    og, orf = sim.observables(), ref.observables()
    assert abs(og["D"] - orf["D"]) <= 1e-9
    assert abs(og["theta_deg"] - orf["theta_deg"]) <= 1e-6
    assert abs(og["mass"] - orf["mass"]) <= 1e-12 * orf["mass"]
    _compare(sim, ref, tol_r=1e-9, tol_u=1e-9, tol_rho=1e-12)


def test_fp32_plain_geometry_200_steps(ib):
    L = (32, 32, 32)
    g = 1e-3
    A = simple_shear(g)
    sim, ref = _pair(ib, "f32", L, R=5.0, level=3, tau=1.0, sigma=(1 / 6) * g * 5.0 / 0.05, A0=A)
    sim.step(A, 200)
    ref.step(A, 200)
    og, orf = sim.observables(), ref.observables()
    assert abs(og["D"] - orf["D"]) <= 1e-2 * orf["D"]
    assert abs(og["theta_deg"] - orf["theta_deg"]) <= 0.5
    _compare(sim, ref, tol_r=1e-4, tol_u=1e-3, tol_rho=1e-5)


@pytest.mark.parametrize("storage,tol", [("f64", F64_TOL), ("f32", F32_TOL)])
def test_several_smoothing_iterations_every_step(ib, storage, tol):
    """A tolerance no smoothing iteration meets: every step runs to the cap of
    4 iterations. On the GPU the force kernel's first work-group then runs
    iterations 2-4 itself and spreads every vertex with direct atomics."""
    L = (19, 17, 21)
    A = _traceless(3e-3, 2)
    sim, ref = _pair(ib, storage, L, R=3.2, level=2, tau=0.9, sigma=0.02, A0=A, reg_tol=1e-12, reg_max_iter=4)
    sim.step(A, 20)
    ref.step(A, 20)
    _compare(sim, ref, **tol)
    og, orf = sim.observables(), ref.observables()
    assert og["reg_iters"] == orf["reg_iters"] == 4


def test_smoothing_iterations_vary_between_steps(ib):
    """A tolerance met after one to a few iterations, so that steps with one
    iteration (the patch path) and with more (the first work-group's path)
    alternate (the oracle takes 1 iteration in 21 of the 30 steps and 2-6 in
    the others); FP64 against the oracle, iteration counts equal every step."""
    L = (19, 17, 21)
    A = _traceless(3e-3, 5)
    sim, ref = _pair(ib, "f64", L, R=3.2, level=2, tau=0.9, sigma=0.02, A0=A, reg_tol=3e-3)
    counts = []
    for _ in range(30):
        sim.step(A, 1)
        ref.step(A, 1)
        og, orf = sim.observables(), ref.observables()
        assert og["reg_iters"] == orf["reg_iters"]
        counts.append(og["reg_iters"])
    print(f"  iteration counts {np.bincount(counts)}", flush=True)
    assert min(counts) == 1 and max(counts) > 1
    _compare(sim, ref, **F64_TOL)


def test_viscosity_ratio_several_smoothing_iterations(ib):
    """The same path with a viscosity ratio: the first work-group also crosses
    every triangle with the lattice rows; indicator and fields against the
    oracle (FP64)."""
    L = (16, 18, 16)
    A = simple_shear(2e-3)
    sim, ref = _pair(ib, "f64", L, R=3.5, level=2, tau=0.9, sigma=0.02, A0=A, chi=4.0, reg_tol=1e-12,
                     reg_max_iter=3)
    sim.step(A, 20)
    ref.step(A, 20)
    assert np.array_equal(sim.indicator(), ref.indicator())
    _compare(sim, ref, **F64_TOL)
