"""The allocation-free vertex read, ibm_lb_read_vertices_noalloc, against
ibm_lb_read_vertices through the C-ABI: bit-identical output on two calls in
a row, the second on a handle with a smaller mesh (the library's staging
array keeps the last call's contents), in FP64 and FP32 storage, into a
caller buffer filled with NaN; a lattice without a mesh; and the size limit
(EINVAL above IBM_LB_NOALLOC_MAX_VERTICES, the allocating read still works)."""
import numpy as np
import pytest

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


def _droplet(ib, storage, L, level, R):
    V, T = icosphere(level, R, box_center(L))
    print(f"case noalloc storage={storage} L={L} nv={len(V)}", flush=True)
    A = simple_shear(2e-3)
    sim = ib.Simulation(L, 0.9, storage=storage, sigma=0.01, radius=R, vertices=V, triangles=T, A0=A)
    sim.step(A, 5)
    return sim, A


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_noalloc_read_equals_read_vertices(ib, storage):
    big, A = _droplet(ib, storage, (40, 40, 40), 5, 12.0)   # 10242 vertices
    small, _ = _droplet(ib, storage, (16, 16, 16), 2, 3.0)  # 162 vertices
    for sim in (big, small, big):
        ref = sim.vertices()
        out = np.full((sim.nv, 3), np.nan)
        got = sim.read_vertices_noalloc(out)
        assert got is out
        assert np.array_equal(out, ref)
        sim.step(A, 2)
        assert np.array_equal(sim.read_vertices_noalloc(), sim.vertices())
    big.close()
    small.close()


def test_noalloc_read_without_mesh(ib):
    sim = ib.Simulation((8, 8, 8), 0.8, storage="f32")
    assert sim.read_vertices_noalloc().shape == (0, 3)
    sim.close()


def test_noalloc_read_size_limit(ib):
    L = (80, 80, 80)
    V, T = icosphere(8, 30.0, box_center(L))  # 655362 vertices
    assert len(V) > ib.NOALLOC_MAX_VERTICES
    print(f"case noalloc limit nv={len(V)}", flush=True)
    sim = ib.Simulation(L, 0.9, storage="f32", sigma=0.01, radius=30.0, vertices=V, triangles=T)
    with pytest.raises(ib.IbmLbError) as e:
        sim.read_vertices_noalloc()
    assert e.value.code == ib.EINVAL
    assert np.abs(sim.vertices() - V).max() < 1e-5
    sim.close()
