"""ctypes front-end of the plain FP64 CPU oracle (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg use
this package. It shares no code with the HIP library; the two meet only on
the seeded inputs of ``paper_2403_01161_amd.inputs``.

Arrays returned here use the external layouts of the tests:
rho as (Lz, Ly, Lx), u as (3, Lz, Ly, Lx), vertices as (nv, 3).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibmlb_oracle.so")

OBS_N = 38
FLAG_DEGENERATE, FLAG_E_ZERO, FLAG_REG_CAP = 1, 2, 4
ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -4: "EDOMAIN", -5: "ENONFINITE"}

_lib = None


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where}: {ERRORS.get(code, code)}")
        self.code = code


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


class _Params(C.Structure):
    _fields_ = [("L", C.c_int * 3), ("periodic", C.c_int * 3), ("tau", C.c_double),
                ("sigma", C.c_double), ("radius", C.c_double), ("rho0", C.c_double),
                ("nv", C.c_int), ("nt", C.c_int), ("verts", C.POINTER(C.c_double)),
                ("tris", C.POINTER(C.c_int)), ("reg_alpha", C.c_double),
                ("reg_gamma", C.c_double), ("reg_tol", C.c_double),
                ("reg_max_iter", C.c_int), ("reg_sign", C.c_int), ("init_rest", C.c_int),
                ("A0", C.c_double * 9), ("wall_bc", C.c_int), ("collision", C.c_int),
                ("mrt_s", C.c_double * 5), ("chi", C.c_double)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp, ip, i = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_int
        L.ibo_phi.restype = C.c_double
        L.ibo_phi.argtypes = [C.c_double]
        L.ibo_lattice.argtypes = [ip, dp, ip]
        L.ibo_equilibrium.argtypes = [C.c_double, dp, dp]
        L.ibo_guo_source.argtypes = [C.c_double, dp, dp, dp]
        L.ibo_forces.argtypes = [i, dp, i, ip, C.c_double, dp]
        L.ibo_spread.argtypes = [ip, ip, i, dp, dp, dp]
        L.ibo_interp.argtypes = [ip, ip, i, dp, dp, dp]
        L.ibo_hc.argtypes = [i, i, ip, C.c_double, C.c_double, C.c_double, i, i, dp, ip]
        L.ibo_eig3.argtypes = [dp, dp, dp]
        L.ibo_mrt_basis.argtypes = [dp, dp]
        L.ibo_mrt_basis.restype = None
        L.ibo_shape.argtypes = [i, dp, i, ip, dp, C.c_double, dp]
        L.ibo_winding.restype = C.c_double
        L.ibo_winding.argtypes = [i, dp, i, ip, dp]
        L.ibo_indicator.argtypes = [ip, i, dp, i, ip, C.POINTER(C.c_ubyte)]
        L.ibo_get_indicator.argtypes = [C.c_void_p, C.POINTER(C.c_ubyte)]
        L.ibo_create.argtypes = [C.POINTER(_Params), C.POINTER(C.c_void_p)]
        L.ibo_destroy.argtypes = [C.c_void_p]
        L.ibo_destroy.restype = None
        L.ibo_step.argtypes = [C.c_void_p, dp, i, i]
        L.ibo_observables.argtypes = [C.c_void_p, dp]
        L.ibo_get_vertices.argtypes = [C.c_void_p, dp]
        L.ibo_set_vertices.argtypes = [C.c_void_p, dp]
        L.ibo_fields.argtypes = [C.c_void_p, dp, dp]
        L.ibo_get_populations.argtypes = [C.c_void_p, dp]
        L.ibo_set_populations.argtypes = [C.c_void_p, dp]
        L.ibo_freeze_iters.argtypes = [C.c_void_p, ip, i]
        L.ibo_last_iters.argtypes = [C.c_void_p]
        L.ibo_last_iters.restype = C.c_int
        L.ibo_nodes.argtypes = [C.c_void_p]
        L.ibo_nodes.restype = C.c_long
        _lib = L
    return _lib


def _check(rc, where):
    if rc != 0:
        raise OracleError(rc, where)


# ---------------------------------------------------------------- primitives
def lattice():
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().ibo_lattice(_ip(c), _dp(w), _ip(opp))
    return c.reshape(19, 3), w, opp


def phi(r):
    return lib().ibo_phi(float(r))


def equilibrium(rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    lib().ibo_equilibrium(float(rho), _dp(u), _dp(out))
    return out


def guo_source(tau, u, F):
    u = np.ascontiguousarray(u, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib().ibo_guo_source(float(tau), _dp(u), _dp(F), _dp(out))
    return out


def forces(r, tris, sigma):
    r = np.ascontiguousarray(r, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    out = np.zeros_like(r)
    lib().ibo_forces(len(r), _dp(r), len(t), _ip(t), float(sigma), _dp(out))
    return out


def spread(L, periodic, r, phi_k):
    """F as (N, 3) node-major, node n = x + Lx (y + Ly z)."""
    Li = np.array(L, dtype=np.int32)
    Pi = np.array(periodic, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.float64)
    p = np.ascontiguousarray(phi_k, dtype=np.float64)
    F = np.zeros((int(np.prod(L)), 3))
    _check(lib().ibo_spread(_ip(Li), _ip(Pi), len(r), _dp(r), _dp(p), _dp(F)), "spread")
    return F


def interp(L, periodic, r, u_nodes):
    """u_nodes (N, 3) node-major -> U (nv, 3)."""
    Li = np.array(L, dtype=np.int32)
    Pi = np.array(periodic, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.float64)
    u = np.ascontiguousarray(u_nodes, dtype=np.float64)
    U = np.zeros_like(r)
    _check(lib().ibo_interp(_ip(Li), _ip(Pi), len(r), _dp(r), _dp(u), _dp(U)), "interp")
    return U


def hc(r, tris, alpha=0.1, gamma=0.51, tol=0.01, max_iter=50, sign=1):
    r = np.array(r, dtype=np.float64, copy=True)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    capped = np.zeros(1, dtype=np.int32)
    it = lib().ibo_hc(len(r), len(t), _ip(t), alpha, gamma, tol, max_iter, sign, _dp(r), _ip(capped))
    if it < 0:
        raise OracleError(it, "hc")
    return r, it, bool(capped[0])


def eig3(S):
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(9)
    ev = np.zeros(3)
    vec = np.zeros(9)
    lib().ibo_eig3(_dp(S), _dp(ev), _dp(vec))
    return ev, vec.reshape(3, 3)


def _obs_dict(o):
    return {"step": int(o[0]), "volume": o[1], "centroid": o[2:5].copy(),
            "S": o[5:14].reshape(3, 3).copy(), "eigval": o[14:17].copy(),
            "eigvec": o[17:26].reshape(3, 3).copy(), "D": o[26], "beta": o[27],
            "theta_deg": o[28], "mass": o[29], "momentum": o[30:33].copy(),
            "reg_iters": int(o[33]), "flags": int(o[34]), "min_angle_deg": o[35], "edge_min": o[36],
            "edge_max": o[37]}


def mrt_basis():
    """(M [19, 19], squared row norms [19]) of the MRT moment basis."""
    M, n2 = np.zeros(19 * 19), np.zeros(19)
    lib().ibo_mrt_basis(_dp(M), _dp(n2))
    return M.reshape(19, 19), n2


def shape(r, tris, A=None, radius=1.0):
    r = np.ascontiguousarray(r, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    A = np.zeros(9) if A is None else np.ascontiguousarray(A, dtype=np.float64).reshape(9)
    out = np.zeros(OBS_N)
    _check(lib().ibo_shape(len(r), _dp(r), len(t), _ip(t), _dp(A), float(radius), _dp(out)), "shape")
    return _obs_dict(out)


def winding(r, tris, p):
    """Winding number of the closed mesh about the point p."""
    r = np.ascontiguousarray(r, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    q = np.ascontiguousarray(p, dtype=np.float64).reshape(3)
    return float(lib().ibo_winding(len(r), _dp(r), len(t), _ip(t), _dp(q)))


def _up(a):
    return a.ctypes.data_as(C.POINTER(C.c_ubyte))


def indicator(L, r, tris):
    """Inside indicator of the closed mesh (absolute coordinates) on the
    lattice L, as uint8 [Lz, Ly, Lx]."""
    Lv = np.ascontiguousarray(L, dtype=np.int32)
    r = np.ascontiguousarray(r, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    out = np.zeros(int(np.prod(Lv)), dtype=np.uint8)
    lib().ibo_indicator(_ip(Lv), len(r), _dp(r), len(t), _ip(t), _up(out))
    return out.reshape(int(Lv[2]), int(Lv[1]), int(Lv[0]))


# ---------------------------------------------------------------- simulation
class Oracle:
    """The coupled IB-LB timestep in plain FP64 loops."""

    def __init__(self, L, tau, sigma=0.0, radius=1.0, vertices=None, triangles=None,
                 periodic=(0, 0, 0), rho0=1.0, reg_alpha=0.1, reg_gamma=0.51, reg_tol=0.01,
                 reg_max_iter=50, reg_sign=1, init_rest=False, A0=None, collision="bgk", mrt_s=None,
                 walls="link", chi=1.0):
        p = _Params()
        self.L = tuple(int(v) for v in L)
        for a in range(3):
            p.L[a] = self.L[a]
            p.periodic[a] = int(periodic[a])
        p.tau, p.sigma, p.radius, p.rho0 = float(tau), float(sigma), float(radius), float(rho0)
        if vertices is None:
            self._v = np.zeros((0, 3))
            self._t = np.zeros((0, 3), dtype=np.int32)
        else:
            self._v = np.ascontiguousarray(vertices, dtype=np.float64)
            self._t = np.ascontiguousarray(triangles, dtype=np.int32)
        p.nv, p.nt = len(self._v), len(self._t)
        p.verts = _dp(self._v)
        p.tris = _ip(self._t)
        p.reg_alpha, p.reg_gamma, p.reg_tol = reg_alpha, reg_gamma, reg_tol
        p.reg_max_iter, p.reg_sign, p.init_rest = int(reg_max_iter), int(reg_sign), int(init_rest)
        A0 = np.zeros(9) if A0 is None else np.asarray(A0, dtype=np.float64).reshape(9)
        for k in range(9):
            p.A0[k] = A0[k]
        p.collision = {"bgk": 0, "mrt": 1}[collision]
        p.wall_bc = {"link": 0, "wet": 1, "wet_printed": 2}[walls]
        for k, v in enumerate(mrt_s if mrt_s is not None else [0.0] * 5):
            p.mrt_s[k] = float(v)
        p.chi = float(chi)
        h = C.c_void_p()
        _check(lib().ibo_create(C.byref(p), C.byref(h)), "create")
        self._h = h
        self.nv = p.nv
        self.N = int(np.prod(self.L))

    def close(self):
        if getattr(self, "_h", None):
            lib().ibo_destroy(self._h)
            self._h = None

    __del__ = close

    def step(self, A, nsteps=1):
        A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
        _check(lib().ibo_step(self._h, _dp(A), int(nsteps), 0), "step")

    def step_table(self, A_table):
        A = np.ascontiguousarray(A_table, dtype=np.float64).reshape(-1, 9)
        _check(lib().ibo_step(self._h, _dp(A), len(A), 1), "step_table")

    def observables(self):
        out = np.zeros(OBS_N)
        _check(lib().ibo_observables(self._h, _dp(out)), "observables")
        return _obs_dict(out)

    def vertices(self):
        out = np.zeros((self.nv, 3))
        lib().ibo_get_vertices(self._h, _dp(out))
        return out

    def set_vertices(self, r):
        r = np.ascontiguousarray(r, dtype=np.float64)
        lib().ibo_set_vertices(self._h, _dp(r))

    def fields(self):
        rho = np.zeros(self.N)
        u = np.zeros((self.N, 3))
        _check(lib().ibo_fields(self._h, _dp(rho), _dp(u)), "fields")
        Lx, Ly, Lz = self.L
        return rho.reshape(Lz, Ly, Lx), u.T.reshape(3, Lz, Ly, Lx).copy()

    def freeze_iters(self, counts):
        """The next len(counts) steps run exactly counts[j] smoothing iterations."""
        c = np.ascontiguousarray(counts, dtype=np.int32)
        _check(lib().ibo_freeze_iters(self._h, _ip(c), len(c)), "freeze_iters")

    def last_iters(self):
        return int(lib().ibo_last_iters(self._h))

    def indicator(self):
        """Inside indicator of the current mesh, uint8 [Lz, Ly, Lx]: the nodes
        that the next step relaxes with the inner relaxation time."""
        out = np.zeros(self.N, dtype=np.uint8)
        _check(lib().ibo_get_indicator(self._h, _up(out)), "indicator")
        Lx, Ly, Lz = self.L
        return out.reshape(Lz, Ly, Lx)

    def populations(self):
        f = np.zeros((self.N, 19))
        lib().ibo_get_populations(self._h, _dp(f))
        return f

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(self.N, 19)
        lib().ibo_set_populations(self._h, _dp(f))
