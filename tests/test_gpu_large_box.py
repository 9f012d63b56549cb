"""GPU: a box above 2^31 / 19 nodes (500^3, FP32 populations), where every
population plane offset i N + n exceeds 32 bits for the later planes. The
oracle cannot run this size; a property that holds at any size stands in:
from the Chapman-Enskog state of plane Couette flow u_x = g (y - y_c),
periodic along x and z, with the y walls moving with that flow, the flow is
steady: the linear field is an exact solution of the link-wise moving-wall
scheme (the FP64 oracle keeps it to 1e-15). After a few steps the velocity
at sampled nodes, including the last planes and the walls, equals
A (x - x_c) to FP32 rounding of the stored deviations, and the mass is
unchanged."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_couette_steady_at_500_cubed():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_01161_amd import ibmlb
    L = (500, 500, 500)
    A = np.array([0.0, 1e-4, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0])
    print("case 500^3 Couette flow, f32", flush=True)
    sim = ibmlb.Simulation(L, 0.8, storage="f32", A0=A, periodic=(1, 0, 1))
    m0 = sim.observables()["mass"]
    sim.step(A, 3)
    ob = sim.observables()
    rho, u = sim.fields()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    assert abs(ob["mass"] - m0) <= 1e-9 * m0
    xc = (np.array(L) - 1) / 2.0
    rng = np.random.default_rng(0)
    pts = np.concatenate([rng.integers(0, 500, size=(2000, 3)),
                          [[0, 0, 0], [499, 499, 499], [250, 0, 499], [499, 250, 0], [3, 497, 499]]])
    G = A.reshape(3, 3)
    umax = 0.0
    for x, y, z in pts:
        want = G @ (np.array([x, y, z]) - xc)
        got = u[:, z, y, x]
        umax = max(umax, np.abs(got - want).max())
        assert np.abs(got - want).max() <= 1e-7, (x, y, z, got, want)
        assert abs(rho[z, y, x] - 1.0) <= 1e-5
    print(f"  max |u - A(x - x_c)| at {len(pts)} nodes: {umax:.2e}", flush=True)
