"""GPU discrete adjoint for the other shape objectives, lambda_max (the
largest eigenvalue of S) and beta (Eq. beta with the strain of the last
gradient row, whose direct dependence on that row is part of dJ/dA),
against central differences of the FP64 oracle with the smoothing
iteration counts frozen at the nominal run's (the bar of the D objective:
1e-3 relative). Also dJ/dA0 through the linear initial state."""
import numpy as np
import pytest

import oracle
from paper_2403_01161_amd.inputs import box_center, icosphere

from .test_gpu_adjoint import BAR, H, _nominal, _oracle, _rel, _shear_ou, _small_spec

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01161_amd import ibmlb
    ibmlb.lib()
    return ibmlb


def _J(spec, sigma, V, A, counts, objective):
    o = _oracle(spec, sigma, V)
    o.freeze_iters(counts)
    o.step_table(A)
    if objective == "D":
        j = o.observables()["D"]
    elif objective == "lambda_max":
        j = o.observables()["eigval"][0]
    else:
        # the strain of the (possibly perturbed) last gradient row
        j = oracle.shape(o.vertices(), spec["triangles"], A=A[-1], radius=spec["radius"])["beta"]
    o.close()
    return j


@pytest.mark.parametrize("objective", ["lambda_max", "beta"])
def test_shape_objective_adjoint_matches_oracle_fd(ib, objective):
    import torch
    spec = _small_spec(50)
    V = icosphere(3, 4.0, box_center(spec["L"]))[0]
    nst, gamma = 30, 3e-3
    A = _shear_ou(nst, gamma, 1e-3, 10.0, seed=17)
    spec["A0"] = A[0]
    sigma = (spec["tau"] - 0.5) / 3 * 4.0 * gamma / 0.1
    counts, _, _ = _nominal(spec, sigma, V, A)
    Vt = torch.tensor(V, dtype=torch.float64, requires_grad=True)
    sg = torch.tensor(sigma, dtype=torch.float64, requires_grad=True)
    At = torch.tensor(A, dtype=torch.float64, device="cuda", requires_grad=True)
    print(f"case adjoint objective {objective}", flush=True)
    J = ib.deformation(sg, At, Vt, K=12, objective=objective, **spec)
    J.backward()
    J0 = _J(spec, sigma, V, A, counts, objective)
    assert abs(float(J.detach()) - J0) <= 1e-10 * max(abs(J0), 1e-3)
    hs = H * sigma
    fd = (_J(spec, sigma + hs, V, A, counts, objective)
          - _J(spec, sigma - hs, V, A, counts, objective)) / (2 * hs)
    print(f"  dJ/dsigma adj={float(sg.grad):.9e} fd={fd:.9e}", flush=True)
    assert _rel(float(sg.grad), fd) < BAR
    rng = np.random.default_rng(23)
    dA = At.grad.cpu().numpy()
    for k in range(2):
        d = rng.standard_normal(A.shape) * np.abs(A).max()
        fd = (_J(spec, sigma, V, A + H * d, counts, objective)
              - _J(spec, sigma, V, A - H * d, counts, objective)) / (2 * H)
        ad = float((dA * d).sum())
        print(f"  direction {k}: adj={ad:.9e} fd={fd:.9e}", flush=True)
        assert _rel(ad, fd) < BAR
    dv = rng.standard_normal(V.shape) * 0.05
    fd = (_J(spec, sigma, V + H * dv, A, counts, objective)
          - _J(spec, sigma, V - H * dv, A, counts, objective)) / (2 * H)
    ad = float((Vt.grad.numpy() * dv).sum())
    print(f"  initial positions: adj={ad:.9e} fd={fd:.9e}", flush=True)
    assert _rel(ad, fd) < BAR


def test_initial_gradient_adjoint_matches_oracle_fd(ib):
    """dJ/dA0 through the linear initial state (the equilibrium of u = A0 (x - x_c) and its
    Chapman-Enskog part) against oracle central differences in A0, two seeded directions."""
    import torch
    spec = _small_spec(50)
    V = icosphere(3, 4.0, box_center(spec["L"]))[0]
    nst, gamma = 30, 3e-3
    A = _shear_ou(nst, gamma, 1e-3, 10.0, seed=29)
    spec["A0"] = A[0]
    sigma = (spec["tau"] - 0.5) / 3 * 4.0 * gamma / 0.1
    counts, _, _ = _nominal(spec, sigma, V, A)
    A0t = torch.tensor(A[0], dtype=torch.float64, requires_grad=True)
    At = torch.tensor(A, dtype=torch.float64, device="cuda")
    kw = {k: v for k, v in spec.items() if k != "A0"}
    print("case adjoint initial state A0", flush=True)
    J = ib.deformation(torch.tensor(sigma, dtype=torch.float64), At, V, K=12, A0=A0t, **kw)
    J.backward()
    g = A0t.grad.numpy()
    rng = np.random.default_rng(31)
    for k in range(2):
        d = rng.standard_normal(9) * np.abs(A[0]).max()
        Jp = _J(dict(spec, A0=A[0] + H * d), sigma, V, A, counts, "D")
        Jm = _J(dict(spec, A0=A[0] - H * d), sigma, V, A, counts, "D")
        fd = (Jp - Jm) / (2 * H)
        ad = float(g @ d)
        print(f"  direction {k}: adj={ad:.9e} fd={fd:.9e}", flush=True)
        assert _rel(ad, fd) < BAR
    # a rest initial state does not depend on A0
    sim = ib.Simulation(kw["L"], kw["tau"], sigma=sigma, radius=4.0, vertices=V, triangles=kw["triangles"],
                        storage="f64", init="rest", A0=A[0])
    assert np.array_equal(sim.adjoint_initial(torch.ones(19 * sim.N, dtype=torch.float64, device="cuda")),
                          np.zeros(9))
    sim.close()
