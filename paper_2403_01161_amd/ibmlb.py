"""Python binding of the gfx950 IB-LB droplet library (libibmlb.so).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C-ABI of include/ibm_lb.h. PyTorch supplies device memory (the
workspace tensor) and the HIP stream. There is no CPU fallback: if the
library has not been built, importing the handle classes raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # loads the HIP runtime the library binds to

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibmlb.so")

OK, EINVAL, ENOMEM, EDEVICE, EDOMAIN, ENONFINITE = 0, -1, -2, -3, -4, -5
NOALLOC_MAX_VERTICES = 262144  # IBM_LB_NOALLOC_MAX_VERTICES
F64, F32, F16DEV, BF16DEV = 0, 1, 2, 3
STORAGE = {"f64": F64, "f32": F32, "f16dev": F16DEV, "bf16dev": BF16DEV}
INIT_LINEAR, INIT_REST = 0, 1
OBS_DEGENERATE, OBS_E_ZERO, OBS_REG_CAP = 1, 2, 4
FIELD_RHO, FIELD_U = 0, 1

_lib = None


OBJECTIVES = {"D": 0, "lambda_max": 1, "beta": 2}


class IbmLbError(RuntimeError):
    def __init__(self, code, where, detail=""):
        super().__init__(f"{where}: {_lib.ibm_lb_strerror(code).decode() if _lib else code}"
                         + (f" ({detail})" if detail else ""))
        self.code = code


class Config(C.Structure):
    _fields_ = [("L", C.c_int32 * 3), ("periodic", C.c_int32 * 3), ("tau", C.c_double),
                ("sigma", C.c_double), ("radius", C.c_double), ("rho0", C.c_double),
                ("n_vertices", C.c_int32), ("n_triangles", C.c_int32),
                ("vertices", C.POINTER(C.c_double)), ("triangles", C.POINTER(C.c_int32)),
                ("reg_alpha", C.c_double), ("reg_gamma", C.c_double), ("reg_tol", C.c_double),
                ("reg_max_iter", C.c_int32), ("reg_sign", C.c_int32), ("storage", C.c_int32),
                ("init", C.c_int32), ("A0", C.c_double * 9), ("f16_scale", C.c_double),
                ("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("populations", C.c_int32), ("collision", C.c_int32), ("mrt_s", C.c_double * 5),
                ("walls", C.c_int32), ("chi", C.c_double), ("deterministic", C.c_int32)]


class Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("volume", C.c_double), ("centroid", C.c_double * 3),
                ("S", C.c_double * 9), ("eigval", C.c_double * 3), ("eigvec", C.c_double * 9),
                ("D", C.c_double), ("beta", C.c_double), ("theta_deg", C.c_double),
                ("mass", C.c_double), ("momentum", C.c_double * 3), ("reg_iters", C.c_int32),
                ("flags", C.c_int32), ("min_angle_deg", C.c_double), ("edge_min", C.c_double),
                ("edge_max", C.c_double)]


EXPORTS = ["ibm_lb_workspace_size", "ibm_lb_init", "ibm_lb_step", "ibm_lb_step_table",
           "ibm_lb_observables", "ibm_lb_read_vertices", "ibm_lb_read_field", "ibm_lb_read_indicator",
           "ibm_lb_state_bytes", "ibm_lb_save", "ibm_lb_load", "ibm_lb_autotune", "ibm_lb_set_variant",
           "ibm_lb_timing_enable",
           "ibm_lb_timing_read", "ibm_lb_destroy", "ibm_lb_strerror", "ibm_lb_last_error",
           "ibm_lb_batch_init", "ibm_lb_batch_step", "ibm_lb_batch_observables", "ibm_lb_batch_member",
           "ibm_lb_batch_autotune", "ibm_lb_batch_set_variant", "ibm_lb_batch_set_graph",
           "ibm_lb_batch_destroy", "ibm_lb_objective_grad", "ibm_lb_shape_objective_grad",
           "ibm_lb_adjoint_segment", "ibm_lb_adjoint_initial", "ibm_lb_read_vertices_noalloc"]


def lib():
    """Load libibmlb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, dp, i32 = C.c_void_p, C.POINTER(C.c_double), C.c_int32
        L.ibm_lb_workspace_size.argtypes = [C.POINTER(Config), C.POINTER(C.c_size_t)]
        L.ibm_lb_init.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.ibm_lb_step.argtypes = [vp, dp, i32]
        L.ibm_lb_step_table.argtypes = [vp, vp, i32, i32]
        L.ibm_lb_observables.argtypes = [vp, C.POINTER(Obs)]
        L.ibm_lb_read_vertices.argtypes = [vp, dp]
        L.ibm_lb_read_vertices_noalloc.argtypes = [vp, dp]
        L.ibm_lb_read_field.argtypes = [vp, i32, dp]
        L.ibm_lb_read_indicator.argtypes = [vp, C.POINTER(C.c_uint8)]
        L.ibm_lb_state_bytes.argtypes = [vp]
        L.ibm_lb_state_bytes.restype = C.c_size_t
        L.ibm_lb_save.argtypes = [vp, vp, C.c_size_t]
        L.ibm_lb_load.argtypes = [vp, vp, C.c_size_t]
        L.ibm_lb_autotune.argtypes = [vp, i32, C.POINTER(C.c_int32)]
        L.ibm_lb_set_variant.argtypes = [vp, i32]
        L.ibm_lb_timing_enable.argtypes = [vp, i32]
        L.ibm_lb_timing_read.argtypes = [vp, dp, C.POINTER(C.c_int64)]
        L.ibm_lb_destroy.argtypes = [vp]
        L.ibm_lb_destroy.restype = None
        L.ibm_lb_batch_init.argtypes = [C.POINTER(Config), i32, vp, C.POINTER(vp)]
        L.ibm_lb_batch_step.argtypes = [vp, dp, i32]
        L.ibm_lb_batch_observables.argtypes = [vp, C.POINTER(Obs)]
        L.ibm_lb_batch_member.argtypes = [vp, i32, C.POINTER(vp)]
        L.ibm_lb_batch_autotune.argtypes = [vp, i32, C.POINTER(C.c_int32)]
        L.ibm_lb_batch_set_variant.argtypes = [vp, i32]
        L.ibm_lb_batch_set_graph.argtypes = [vp, i32]
        L.ibm_lb_batch_destroy.argtypes = [vp]
        L.ibm_lb_batch_destroy.restype = None
        L.ibm_lb_objective_grad.argtypes = [vp, dp, vp]
        L.ibm_lb_shape_objective_grad.argtypes = [vp, i32, dp, vp, dp]
        L.ibm_lb_adjoint_segment.argtypes = [vp, vp, C.c_size_t, vp, i32, i32, vp, vp, vp, vp, vp, vp]
        L.ibm_lb_adjoint_initial.argtypes = [vp, vp, dp]
        L.ibm_lb_strerror.argtypes = [C.c_int]
        L.ibm_lb_strerror.restype = C.c_char_p
        L.ibm_lb_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc, where):
    if rc != OK:
        raise IbmLbError(rc, where, lib().ibm_lb_last_error().decode())


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_config(L, tau, sigma=0.0, radius=1.0, vertices=None, triangles=None, periodic=(0, 0, 0),
                storage="f32", init="linear", A0=None, rho0=1.0, reg_alpha=0.1, reg_gamma=0.51,
                reg_tol=0.01, reg_max_iter=50, reg_sign=1, f16_scale=0.0, populations=2, collision="bgk",
                mrt_s=None, walls="link", chi=1.0, deterministic=False):
    """Fill an ibm_lb_config; returns (config, keep-alive arrays)."""
    cfg = Config()
    for a in range(3):
        cfg.L[a] = int(L[a])
        cfg.periodic[a] = int(periodic[a])
    cfg.tau, cfg.sigma, cfg.radius, cfg.rho0 = float(tau), float(sigma), float(radius), float(rho0)
    if vertices is None:
        V = np.zeros((0, 3))
        T = np.zeros((0, 3), dtype=np.int32)
    else:
        V = np.ascontiguousarray(vertices, dtype=np.float64)
        T = np.ascontiguousarray(triangles, dtype=np.int32)
    cfg.n_vertices, cfg.n_triangles = len(V), len(T)
    cfg.vertices = _dp(V) if len(V) else None
    cfg.triangles = T.ctypes.data_as(C.POINTER(C.c_int32)) if len(T) else None
    cfg.reg_alpha, cfg.reg_gamma, cfg.reg_tol = reg_alpha, reg_gamma, reg_tol
    cfg.reg_max_iter, cfg.reg_sign = int(reg_max_iter), int(reg_sign)
    cfg.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    cfg.init = {"linear": INIT_LINEAR, "rest": INIT_REST}[init] if isinstance(init, str) else int(init)
    A0 = np.zeros(9) if A0 is None else np.asarray(A0, dtype=np.float64).reshape(9)
    for k in range(9):
        cfg.A0[k] = A0[k]
    cfg.f16_scale = float(f16_scale)
    cfg.populations = int(populations)
    cfg.collision = {"bgk": 0, "mrt": 1}[collision] if isinstance(collision, str) else int(collision)
    for k, v in enumerate(mrt_s if mrt_s is not None else [0.0] * 5):
        cfg.mrt_s[k] = float(v)
    cfg.walls = {"link": 0, "wet": 1}[walls] if isinstance(walls, str) else int(walls)
    cfg.chi = float(chi)
    cfg.deterministic = int(deterministic)
    return cfg, (V, T)


def workspace_size(cfg):
    n = C.c_size_t()
    _check(lib().ibm_lb_workspace_size(C.byref(cfg), C.byref(n)), "ibm_lb_workspace_size")
    return n.value


def _obs_dict(o):
    return {"step": o.step, "volume": o.volume, "centroid": np.array(o.centroid[:]),
            "S": np.array(o.S[:]).reshape(3, 3), "eigval": np.array(o.eigval[:]),
            "eigvec": np.array(o.eigvec[:]).reshape(3, 3), "D": o.D, "beta": o.beta,
            "theta_deg": o.theta_deg, "mass": o.mass, "momentum": np.array(o.momentum[:]),
            "reg_iters": o.reg_iters, "flags": o.flags, "min_angle_deg": o.min_angle_deg,
            "edge_min": o.edge_min, "edge_max": o.edge_max}


class Simulation:
    """One droplet (or a bare lattice) advanced on the GPU.

    Device memory comes from a torch uint8 tensor on `device`; the work is
    enqueued on torch's current stream of that device (or `stream`).
    """

    def __init__(self, L, tau, sigma=0.0, radius=1.0, vertices=None, triangles=None,
                 periodic=(0, 0, 0), storage="f32", init="linear", A0=None, device="cuda:0",
                 stream=None, **kw):
        lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        cfg, keep = make_config(L, tau, sigma, radius, vertices, triangles, periodic, storage, init,
                                A0, **kw)
        nbytes = workspace_size(cfg)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        cfg.workspace = self.workspace.data_ptr()
        cfg.workspace_bytes = nbytes
        cfg.stream = self.stream.cuda_stream
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ibm_lb_init(C.byref(cfg), C.byref(h)), "ibm_lb_init")
        self._h = h
        self.L = tuple(int(v) for v in L)
        self.N = int(np.prod(self.L))
        self.nv = cfg.n_vertices
        self.storage = cfg.storage

    def close(self):
        if getattr(self, "_h", None):
            lib().ibm_lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, A, nsteps=1):
        A = np.ascontiguousarray(A, dtype=np.float64).reshape(9)
        _check(lib().ibm_lb_step(self._h, _dp(A), int(nsteps)), "ibm_lb_step")

    def step_table(self, A_table):
        """A_table: host array [n, 9] or a float64 CUDA tensor [n, 9] (kept alive by the caller
        until the next synchronising call)."""
        if isinstance(A_table, torch.Tensor) and A_table.is_cuda:
            assert A_table.dtype == torch.float64 and A_table.is_contiguous()
            n = A_table.numel() // 9
            _check(lib().ibm_lb_step_table(self._h, A_table.data_ptr(), n, 1), "ibm_lb_step_table")
        else:
            A = np.ascontiguousarray(A_table, dtype=np.float64).reshape(-1, 9)
            _check(lib().ibm_lb_step_table(self._h, A.ctypes.data, len(A), 0), "ibm_lb_step_table")

    def observables(self):
        o = Obs()
        _check(lib().ibm_lb_observables(self._h, C.byref(o)), "ibm_lb_observables")
        return _obs_dict(o)

    def vertices(self):
        out = np.zeros((self.nv, 3))
        _check(lib().ibm_lb_read_vertices(self._h, _dp(out)), "ibm_lb_read_vertices")
        return out

    def read_vertices_noalloc(self, out=None):
        """ibm_lb_read_vertices_noalloc into `out` (float64 [nv][3], C order;
        a new array if None)."""
        if out is None:
            out = np.zeros((self.nv, 3))
        assert out.dtype == np.float64 and out.shape == (self.nv, 3) and out.flags.c_contiguous
        _check(lib().ibm_lb_read_vertices_noalloc(self._h, _dp(out)), "ibm_lb_read_vertices_noalloc")
        return out

    def fields(self):
        Lx, Ly, Lz = self.L
        rho = np.zeros(self.N)
        u = np.zeros(3 * self.N)
        _check(lib().ibm_lb_read_field(self._h, FIELD_RHO, _dp(rho)), "ibm_lb_read_field")
        _check(lib().ibm_lb_read_field(self._h, FIELD_U, _dp(u)), "ibm_lb_read_field")
        return rho.reshape(Lz, Ly, Lx), u.reshape(3, Lz, Ly, Lx)

    def indicator(self):
        """Inside indicator of the current mesh (viscosity ratio only), uint8 [Lz, Ly, Lx]."""
        Lx, Ly, Lz = self.L
        out = np.zeros(self.N, dtype=np.uint8)
        _check(lib().ibm_lb_read_indicator(self._h, out.ctypes.data_as(C.POINTER(C.c_uint8))),
               "ibm_lb_read_indicator")
        return out.reshape(Lz, Ly, Lx)

    def state_bytes(self):
        return lib().ibm_lb_state_bytes(self._h)

    def save(self, dst=None):
        n = self.state_bytes()
        if dst is None:
            dst = torch.empty(n, dtype=torch.uint8, device=self.device)
        _check(lib().ibm_lb_save(self._h, dst.data_ptr(), n), "ibm_lb_save")
        return dst

    def load(self, src):
        _check(lib().ibm_lb_load(self._h, src.data_ptr(), src.numel()), "ibm_lb_load")

    def autotune(self, reps=20):
        """Pick the fastest lattice-kernel variant for this configuration."""
        v = C.c_int32()
        _check(lib().ibm_lb_autotune(self._h, int(reps), C.byref(v)), "ibm_lb_autotune")
        return v.value

    def set_variant(self, variant):
        """Select a step variant directly (0 <= variant < 128: lattice layout and options in
        bits 0-4, the smoothing's finish in the force kernel in bit 5, in-place streaming in
        bit 6; see ibm_lb_set_variant)."""
        _check(lib().ibm_lb_set_variant(self._h, int(variant)), "ibm_lb_set_variant")

    def timing(self, enable=True):
        _check(lib().ibm_lb_timing_enable(self._h, int(enable)), "ibm_lb_timing_enable")

    def timing_read(self):
        ms = C.c_double()
        n = C.c_int64()
        _check(lib().ibm_lb_timing_read(self._h, C.byref(ms), C.byref(n)), "ibm_lb_timing_read")
        return ms.value, n.value

    # ---- adjoint
    def objective_grad(self, objective="D", with_last_row=False):
        """J of the current mesh and dJ/dr as a float64 CUDA tensor [nv, 3] (caller vertex order);
        J is D, "lambda_max" or "beta" (with the strain of the last gradient row). With
        with_last_row, also J's direct derivative by the last gradient row (numpy [9])."""
        rbar = torch.empty((self.nv, 3), dtype=torch.float64, device=self.device)
        v = C.c_double()
        dlast = np.zeros(9)
        _check(lib().ibm_lb_shape_objective_grad(self._h, OBJECTIVES[objective], C.byref(v), rbar.data_ptr(),
                                                 _dp(dlast)),
               "ibm_lb_shape_objective_grad")
        return (v.value, rbar, dlast) if with_last_row else (v.value, rbar)

    def adjoint_initial(self, fbar0):
        """dJ/dA0 (numpy [9]) through the linear initial state from the adjoint of the step-0
        population deviations (float64 CUDA tensor [19 N])."""
        assert fbar0.dtype == torch.float64 and fbar0.is_cuda and fbar0.numel() == 19 * self.N
        out = np.zeros(9)
        _check(lib().ibm_lb_adjoint_initial(self._h, fbar0.contiguous().data_ptr(), _dp(out)),
               "ibm_lb_adjoint_initial")
        return out

    def adjoint_segment(self, ckpt, A, fbar_end, rbar_end, fbar_begin=None, rbar_begin=None, dA=None,
                        dsigma=None):
        """Reverse one segment that starts at checkpoint `ckpt` (a tensor written by save) and runs
        the gradient rows A (float64 CUDA tensor [n, 9] or host array). fbar_end: float64 CUDA
        tensor [19 N] or None (zero); rbar_end: float64 CUDA tensor [nv, 3]. Returns
        (fbar_begin, rbar_begin, dA [n, 9], dsigma [1]); dsigma is accumulated into."""
        dev = self.device
        if isinstance(A, torch.Tensor) and A.is_cuda:
            A = A.contiguous()
            assert A.dtype == torch.float64
            n, a_ptr, on_dev = A.numel() // 9, A.data_ptr(), 1
        else:
            A = np.ascontiguousarray(A, dtype=np.float64).reshape(-1, 9)
            n, a_ptr, on_dev = len(A), A.ctypes.data, 0
        if fbar_begin is None:
            fbar_begin = torch.empty(19 * self.N, dtype=torch.float64, device=dev)
        if rbar_begin is None:
            rbar_begin = torch.empty((self.nv, 3), dtype=torch.float64, device=dev)
        if dA is None:
            dA = torch.empty((n, 9), dtype=torch.float64, device=dev)
        if dsigma is None:
            dsigma = torch.zeros(1, dtype=torch.float64, device=dev)
        for t in (fbar_begin, rbar_begin, dA, dsigma) + ((fbar_end,) if fbar_end is not None else ()) + (rbar_end,):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
        assert dA.numel() == 9 * n and fbar_begin.numel() == 19 * self.N and rbar_end.numel() == 3 * self.nv
        _check(lib().ibm_lb_adjoint_segment(self._h, ckpt.data_ptr(), ckpt.numel(), a_ptr, n, on_dev,
                                            None if fbar_end is None else fbar_end.data_ptr(),
                                            rbar_end.data_ptr(), fbar_begin.data_ptr(), rbar_begin.data_ptr(),
                                            dA.data_ptr(), dsigma.data_ptr()),
               "ibm_lb_adjoint_segment")
        return fbar_begin, rbar_begin, dA, dsigma


class _Member:
    """Read access to one ensemble member (the ensemble owns the handle)."""

    def __init__(self, ens, h, L, nv):
        self._ens, self._h, self.L, self.nv = ens, h, L, nv
        self.N = int(np.prod(L))
        self.device = ens.device

    observables = Simulation.observables
    vertices = Simulation.vertices
    fields = Simulation.fields
    state_bytes = Simulation.state_bytes
    save = Simulation.save


class Ensemble:
    """Independent droplets advanced together: one batched lattice launch and
    one set of batched IB launches per step. `members` is a list of keyword
    dicts for make_config (L, tau, sigma, radius, vertices, triangles, ...);
    all members share `storage`."""

    def __init__(self, members, storage="f32", device="cuda:0", stream=None):
        lib()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        n = len(members)
        cfgs = (Config * n)()
        self._keep, self.workspaces, self._shapes = [], [], []
        for i, kw in enumerate(members):
            kw = dict(kw)
            L, tau = kw.pop("L"), kw.pop("tau")
            cfg, keep = make_config(L, tau, storage=storage, **kw)
            nbytes = workspace_size(cfg)
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            cfg.workspace, cfg.workspace_bytes = ws.data_ptr(), nbytes
            cfgs[i] = cfg
            self._keep.append(keep)
            self.workspaces.append(ws)
            self._shapes.append((tuple(int(v) for v in L), cfg.n_vertices))
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().ibm_lb_batch_init(cfgs, n, self.stream.cuda_stream, C.byref(h)), "ibm_lb_batch_init")
        self._h = h
        self.n = n

    def close(self):
        if getattr(self, "_h", None):
            lib().ibm_lb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def autotune(self, reps=10):
        v = C.c_int32()
        _check(lib().ibm_lb_batch_autotune(self._h, int(reps), C.byref(v)), "ibm_lb_batch_autotune")
        return v.value

    def set_variant(self, variant):
        _check(lib().ibm_lb_batch_set_variant(self._h, int(variant)), "ibm_lb_batch_set_variant")

    def set_graph(self, steps):
        """Replay runs of `steps` batched steps as captured HIP graphs (0: plain launches)."""
        _check(lib().ibm_lb_batch_set_graph(self._h, int(steps)), "ibm_lb_batch_set_graph")

    def step(self, A_tables):
        """A_tables: host array [n, nsteps, 9]."""
        A = np.ascontiguousarray(A_tables, dtype=np.float64)
        assert A.ndim == 3 and A.shape[0] == self.n and A.shape[2] == 9
        _check(lib().ibm_lb_batch_step(self._h, _dp(A), A.shape[1]), "ibm_lb_batch_step")

    def observables(self):
        out = (Obs * self.n)()
        _check(lib().ibm_lb_batch_observables(self._h, out), "ibm_lb_batch_observables")
        return [_obs_dict(o) for o in out]

    def member(self, i):
        h = C.c_void_p()
        _check(lib().ibm_lb_batch_member(self._h, int(i), C.byref(h)), "ibm_lb_batch_member")
        L, nv = self._shapes[i]
        return _Member(self, h, L, nv)



class DeformationFunction(torch.autograd.Function):
    """J = D(r^T): the deformation of a droplet started from a fresh initial
    state and driven by the gradient rows A[n, 9], differentiable with
    respect to sigma, A and the initial vertex positions.

    Forward: run the HIP timestep, saving a checkpoint every K steps.
    Backward: for each segment, last first, reload its checkpoint, recompute
    it and sweep the discrete adjoint (ibm_lb_adjoint_segment), chaining the
    adjoint state (fbar, rbar) from segment to segment. The smoothing
    iteration counts are those the forward took."""

    @staticmethod
    def forward(ctx, sigma, A, vertices, spec, K, objective="D", A0=None):
        spec = dict(spec)
        ctx.a0 = A0 is not None
        if ctx.a0:
            ctx.a0dev, ctx.a0shape = A0.device, A0.shape
            spec["A0"] = A0.detach().cpu().numpy().reshape(9)
        sim = Simulation(sigma=float(sigma), vertices=vertices.detach().cpu().numpy(), **spec)
        ctx.adev = A.device
        A = A.detach().to(device=sim.device, dtype=torch.float64).contiguous()
        n = A.shape[0]
        ckpts = []
        for s0 in range(0, n, K):
            ckpts.append(sim.save())
            sim.step_table(A[s0:s0 + K])
        D, rbar, dlast = sim.objective_grad(objective, with_last_row=True)
        ctx.sim, ctx.ckpts, ctx.K, ctx.rbar, ctx.A, ctx.dlast = sim, ckpts, K, rbar, A, dlast
        ctx.sigma_shape, ctx.sdev, ctx.vdev = sigma.shape, sigma.device, vertices.device
        return torch.tensor(D, dtype=torch.float64, device=sim.device)

    @staticmethod
    def backward(ctx, gD):
        sim, A, K = ctx.sim, ctx.A, ctx.K
        n = A.shape[0]
        rbar = (ctx.rbar * gD).contiguous()
        rnext = torch.empty_like(rbar)
        fbar = None
        fbuf = torch.empty(19 * sim.N, dtype=torch.float64, device=sim.device)
        dA = torch.empty_like(A)
        dsig = torch.zeros(1, dtype=torch.float64, device=sim.device)
        for idx in reversed(range(len(ctx.ckpts))):
            s0, s1 = idx * K, min(n, idx * K + K)
            sim.adjoint_segment(ctx.ckpts[idx], A[s0:s1], fbar, rbar, fbuf, rnext, dA[s0:s1], dsig)
            fbar = fbuf
            rbar, rnext = rnext, rbar
        # the objective's own dependence on the last gradient row (beta)
        dA[-1] += torch.from_numpy(ctx.dlast).to(dA.device).reshape(dA[-1].shape) * gD
        dA0 = None
        if ctx.a0:
            # fbar now holds the adjoint of the step-0 populations (gD already in the seed)
            g0 = sim.adjoint_initial(fbar) if fbar is not None else np.zeros(9)
            dA0 = torch.from_numpy(g0).to(ctx.a0dev).reshape(ctx.a0shape)
        return (dsig.reshape(ctx.sigma_shape).to(ctx.sdev), dA.to(ctx.adev), rbar.to(ctx.vdev), None, None, None,
                dA0)


def deformation(sigma, A, vertices, K=50, objective="D", **spec):
    """Differentiable droplet shape objective J(r^T): the deformation D
    (default), "lambda_max" or "beta" (with the strain of the last gradient row);
    spec holds the Simulation keywords other than sigma and vertices (L, tau,
    radius, triangles, ...). A torch tensor A0 in spec (9 values) is
    differentiated too, through the linear initial state."""
    if not isinstance(sigma, torch.Tensor):
        sigma = torch.tensor(float(sigma), dtype=torch.float64)
    if not isinstance(vertices, torch.Tensor):
        vertices = torch.as_tensor(np.asarray(vertices, dtype=np.float64))
    A0 = spec.pop("A0", None)
    if isinstance(A0, torch.Tensor):
        return DeformationFunction.apply(sigma, A, vertices, spec, int(K), objective, A0)
    if A0 is not None:
        spec["A0"] = A0
    return DeformationFunction.apply(sigma, A, vertices, spec, int(K), objective)
