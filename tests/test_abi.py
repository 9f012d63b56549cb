"""The C-ABI library loads, exports every declared entry point, and rejects
bad configurations on the host (no GPU needed: validation runs before any
HIP call)."""
import os
import re

import numpy as np
import pytest

from paper_2403_01161_amd.inputs import box_center, icosphere

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^[A-Za-z_][\w \*]*?\b(ibm_lb_\w+)\s*\(", src, re.M))
    return names


@pytest.fixture(scope="module")
def ib():
    from paper_2403_01161_amd import ibmlb
    if not os.path.exists(ibmlb.LIB_PATH):
        pytest.skip("libibmlb.so not built")
    ibmlb.lib()
    return ibmlb


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("ibm_lb_init", "ibm_lb_step", "ibm_lb_observables", "ibm_lb_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(ib):
    lib = ib.lib()
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert set(ib.EXPORTS) <= _declared()


def test_strerror(ib):
    lib = ib.lib()
    assert lib.ibm_lb_strerror(0) == b"ok"
    assert lib.ibm_lb_strerror(-4) == b"vertex stencil outside the box"


def _cfg(ib, **kw):
    L = kw.pop("L", (16, 16, 16))
    V, T = icosphere(2, 3.0, box_center(L))
    args = dict(L=L, tau=0.9, sigma=0.01, radius=3.0, vertices=V, triangles=T)
    args.update(kw)
    return ib.make_config(**args)


def _size_rc(ib, cfg):
    import ctypes as C
    n = C.c_size_t()
    rc = ib.lib().ibm_lb_workspace_size(C.byref(cfg), C.byref(n))
    return rc, n.value


def test_valid_config_sizes(ib):
    cfg, keep = _cfg(ib)
    rc, n = _size_rc(ib, cfg)
    assert rc == 0
    N = 16 ** 3
    assert n >= 2 * 19 * N * 4 + 6 * N * 4
    cfg64, keep = _cfg(ib, storage="f64")
    assert _size_rc(ib, cfg64)[1] > n
    cfg16, keep = _cfg(ib, storage="bf16dev")
    assert _size_rc(ib, cfg16)[1] < n
    # one population copy: 19 N s bytes less (up to the 256-byte alignment)
    cfg1, keep = _cfg(ib, populations=1)
    rc1, n1 = _size_rc(ib, cfg1)
    assert rc1 == 0 and abs((n - n1) - 19 * N * 4) <= 256


def test_ensemble_rejects_one_copy_members(ib):
    import ctypes as C
    cfgs = (ib.Config * 2)()
    keep = []
    for i, pops in enumerate((2, 1)):
        c, k = ib.make_config((8, 8, 8), 0.8, populations=pops)
        cfgs[i] = c
        keep.append(k)
    b = C.c_void_p()
    assert ib.lib().ibm_lb_batch_init(cfgs, 2, None, C.byref(b)) == ib.EINVAL
    assert not b.value


def test_deterministic_spreading_sizes(ib):
    """The deterministic spreading stages 76 B (FP64: 136 B) per vertex and a
    32 B window per 64-vertex patch; ensembles refuse it."""
    import ctypes as C
    for storage, rec in (("f32", 76), ("f64", 136)):
        cfg, keep = _cfg(ib, storage=storage)
        n0 = _size_rc(ib, cfg)[1]
        cfg.deterministic = 1
        rc, n1 = _size_rc(ib, cfg)
        nv = cfg.n_vertices
        extra = rec * nv + 32 * ((nv + 63) // 64)
        assert rc == 0 and abs((n1 - n0) - extra) <= 512, (storage, n1 - n0, extra)  # 256-byte alignment
    cfgs = (ib.Config * 1)()
    c, k = ib.make_config((8, 8, 8), 0.8, deterministic=1)
    cfgs[0] = c
    b = C.c_void_p()
    assert ib.lib().ibm_lb_batch_init(cfgs, 1, None, C.byref(b)) == ib.EINVAL
    assert not b.value


@pytest.mark.parametrize("bad", [
    dict(L=(7, 16, 16)), dict(tau=0.5), dict(sigma=-1.0), dict(radius=0.0), dict(rho0=0.0),
    dict(storage=7), dict(init=5), dict(reg_sign=2), dict(reg_max_iter=-1),
    dict(f16_scale=3.0, storage="f16dev"), dict(A0=[np.nan] + [0] * 8), dict(populations=3),
    dict(collision=2), dict(collision="mrt", mrt_s=[2.0, 1, 1, 1, 1]),
    dict(walls=2), dict(walls="wet", populations=1), dict(deterministic=2),
])
def test_invalid_parameters(ib, bad):
    cfg, keep = _cfg(ib, **bad)
    assert _size_rc(ib, cfg)[0] == ib.EINVAL
    import ctypes as C
    h = C.c_void_p()
    assert ib.lib().ibm_lb_init(C.byref(cfg), C.byref(h)) == ib.EINVAL
    assert not h.value
    assert len(ib.lib().ibm_lb_last_error()) > 0


def test_invalid_meshes(ib):
    L = (16, 16, 16)
    V, T = icosphere(2, 3.0, box_center(L))
    cases = {
        "inward": (V, T[:, ::-1].copy()),
        "open": (V, T[1:].copy()),
        "index": (V, np.where(T == 5, len(V), T).astype(np.int32)),
        "wall": (V + [5.5, 0, 0], T),
        "nan": (np.where(np.arange(V.size).reshape(V.shape) == 4, np.nan, V), T),
    }
    for name, (v, t) in cases.items():
        cfg, keep = ib.make_config(L, 0.9, 0.01, 3.0, v, t)
        assert _size_rc(ib, cfg)[0] == ib.EINVAL, name
    # the same stencil is fine on a periodic axis
    cfg, keep = ib.make_config(L, 0.9, 0.01, 3.0, V + [5.5, 0, 0], T, periodic=(1, 0, 0))
    assert _size_rc(ib, cfg)[0] == 0


def test_box_size_limits(ib):
    # 500^3 (above 2^31 / 19 nodes: population offsets need 64 bits) is valid;
    # more than 2^31 - 1 nodes is not
    cfg, keep = ib.make_config((500, 500, 500), 0.8)
    rc, n = _size_rc(ib, cfg)
    assert rc == 0 and n >= 2 * 19 * 4 * 500 ** 3
    cfg, keep = ib.make_config((1300, 1300, 1300), 0.8)
    assert _size_rc(ib, cfg)[0] == ib.EINVAL


def test_lattice_only_config(ib):
    cfg, keep = ib.make_config((8, 9, 10), 0.8)
    assert _size_rc(ib, cfg)[0] == 0
