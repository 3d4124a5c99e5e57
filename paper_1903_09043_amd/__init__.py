"""MI355X (gfx950) all-regime, well-balanced finite-volume step of
arXiv 1903.09043 -- thin Python binding of ``include/ars.h``.

Every step of the method runs in the HIP library ``libars.so`` built in this
directory (``python -m paper_1903_09043_amd.build``); this module only
marshals arguments.  PyTorch provides device memory and the stream.  There is
no CPU fallback: if the library is missing, importing the binding raises.
"""
import ctypes as C
import os

import numpy as np

from . import workloads  # noqa: F401  (problem set-ups)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libars.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONPHYS, EUNSUPPORTED, ESCRATCH, ENOCONV = 0, -1, -2, -3, -4, -5, -6, -7
NOALLOC_MAX_STATE = 131072  # ARS_NOALLOC_MAX_STATE of include/ars.h
TILE3_32x10, TILE3_16x20 = 0, 1
BC_PERIODIC, BC_WALL, BC_OUTFLOW = 0, 1, 2


class ArsError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__(f"{what}: {lib().ars_strerror(status).decode()} ({status})")


class ArsConfig(C.Structure):
    _fields_ = [
        ("dim", C.c_int32),
        ("n", C.c_int32 * 3),
        ("L", C.c_double * 3),
        ("gamma", C.c_double), ("g", C.c_double), ("mu", C.c_double),
        ("kappa", C.c_double), ("K", C.c_double), ("cfl", C.c_double),
        ("low_mach", C.c_int32),
        ("dt_mode", C.c_int32),
        ("bc", (C.c_int32 * 2) * 3),
        ("wall_noslip", C.c_int32),
        ("thermal", C.c_int32 * 2),
        ("T_wall", C.c_double * 2),
        ("energy_form", C.c_int32),
        ("pad_", C.c_int32),
    ]


class ArsTuneResult(C.Structure):
    _fields_ = [("zchunk", C.c_int32), ("wg_per_cu", C.c_int32), ("rows", C.c_int32), ("zc_policy", C.c_int32),
                ("from_cache", C.c_int32), ("n_candidates", C.c_int32), ("ms_per_step", C.c_double),
                ("tile3", C.c_int32), ("pad_", C.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ArsDiag(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("mom", C.c_double * 3), ("e_total", C.c_double), ("e_kin", C.c_double),
        ("e_int", C.c_double), ("e_grav", C.c_double), ("max_u", C.c_double), ("mean_u", C.c_double),
        ("max_mach", C.c_double), ("nu_bot", C.c_double), ("nu_top", C.c_double),
        ("fault_cell", C.c_int64), ("fault", C.c_int32), ("pad_", C.c_int32),
    ]


# (name, restype, argtypes) of every exported entry point of include/ars.h
_VP, _DP, _CP = C.c_void_p, C.POINTER(C.c_double), C.POINTER(ArsConfig)
SIGNATURES = [
    ("ars_validate", C.c_int, [_CP]),
    ("ars_create", C.c_int, [_CP, C.POINTER(_VP)]),
    ("ars_destroy", None, [_VP]),
    ("ars_state_len", C.c_size_t, [_VP]),
    ("ars_workspace_bytes", C.c_size_t, [_VP]),
    ("ars_workspace_init", C.c_int, [_VP, _VP, _VP]),
    ("ars_set_zchunk", C.c_int, [_VP, C.c_int]),
    ("ars_get_zchunk", C.c_int, [_VP]),
    ("ars_init_state", C.c_int, [_VP, C.c_int, _DP, C.c_int, C.c_uint64, _VP, _VP]),
    ("ars_init_state_host", C.c_int, [_VP, C.c_int, _DP, C.c_int, C.c_uint64, _DP]),
    ("ars_init_rb_dT", C.c_int, [_VP, _DP, C.c_int, _VP, _VP, _VP, _VP]),
    ("ars_init_rb_dT_adjoint", C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("ars_compute_dt", C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("ars_step", C.c_int, [_VP, _VP, _VP, _VP, C.c_int, _VP, _VP, _VP, _VP]),
    ("ars_step_noalloc", C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP, _VP]),
    ("ars_step_sched", C.c_int, [_VP, _VP, _VP, _VP, C.c_int, _VP, _VP, _VP]),
    ("ars_step_sched_to", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, C.c_int, _VP, _VP, _VP]),
    ("ars_step_to", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, C.c_int, _VP, _VP, _VP, _VP]),
    ("ars_workspace_bytes_ref", C.c_size_t, [_VP]),
    ("ars_workspace_bytes_imex", C.c_size_t, [_VP]),
    ("ars_step_imex", C.c_int, [_VP, _VP, _VP, _VP, _VP, C.c_int, _VP, _VP, C.c_double, C.c_int,
                                C.POINTER(C.c_int), _VP]),
    ("ars_step_ref", C.c_int, [_VP, _VP, _VP, _VP, _VP, C.c_int, _VP, _VP]),
    ("ars_workspace_bytes_adjoint", C.c_size_t, [_VP]),
    ("ars_step_adjoint", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("ars_workspace_bytes_adjoint_ref", C.c_size_t, [_VP]),
    ("ars_step_adjoint_ref", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("ars_kinetic_energy", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    ("ars_nusselt", C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP, _VP]),
    ("ars_spectrum_len", C.c_int, [_VP]),
    ("ars_workspace_bytes_spectrum", C.c_size_t, [_VP]),
    ("ars_spectrum", C.c_int, [_VP, _VP, C.c_int, _VP, _VP, _VP]),
    ("ars_revolve_plan", C.c_int, [C.c_int, C.c_int, C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int64)]),
    ("ars_revolve_cost", C.c_int64, [C.c_int, C.c_int]),
    ("ars_diagnostics", C.c_int, [_VP, _VP, _VP, C.POINTER(ArsDiag), _VP]),
    ("ars_fault", C.c_int, [_VP, _VP, C.POINTER(C.c_int64), _VP]),
    ("ars_strerror", C.c_char_p, [C.c_int]),
    ("ars_batch_create", C.c_int, [C.c_int, _CP, C.POINTER(_VP)]),
    ("ars_batch_destroy", None, [_VP]),
    ("ars_batch_state_len", C.c_size_t, [_VP]),
    ("ars_batch_state_offset", C.c_size_t, [_VP, C.c_int]),
    ("ars_batch_table_bytes", C.c_size_t, [_VP]),
    ("ars_batch_set_tiling", C.c_int, [_VP, C.c_int, C.POINTER(C.c_int)]),
    ("ars_batch_get_tiling", C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("ars_batch_bind", C.c_int, [_VP, _VP, _VP, _VP, _VP]),
    ("ars_batch_step", C.c_int, [_VP, _VP, C.c_int, _VP]),
    ("ars_batch_capture", C.c_int, [_VP, _VP, C.c_int, _VP]),
    ("ars_batch_replay", C.c_int, [_VP, _VP]),
    ("ars_batch_read", C.c_int, [_VP, _VP, _DP, _DP, C.POINTER(C.c_int64), _VP]),
    ("ars_set_tiling", C.c_int, [_VP, C.c_int, C.c_int]),
    ("ars_set_tile3", C.c_int, [_VP, C.c_int]),
    ("ars_get_tile3", C.c_int, [_VP]),
    ("ars_get_tiling", C.c_int, [_VP, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    ("ars_autotune", C.c_int, [_VP, _VP, _VP, C.c_int, C.c_char_p, _VP, C.POINTER(ArsTuneResult)]),
    ("ars_batch_autotune", C.c_int, [_VP, _VP, _VP, _VP, C.c_int, C.c_char_p, _VP, C.POINTER(ArsTuneResult)]),
]

_lib = None


def lib():
    """Load libars.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1903_09043_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def make_config(cfg: dict) -> ArsConfig:
    c = ArsConfig()
    c.dim = int(cfg["dim"])
    n = list(cfg["n"]) + [1] * (3 - len(cfg["n"]))
    Ls = list(cfg["L"]) + [1.0] * (3 - len(cfg["L"]))
    for a in range(3):
        c.n[a] = int(n[a])
        c.L[a] = float(Ls[a])
    c.gamma = float(cfg.get("gamma", 5.0 / 3.0))
    c.g = float(cfg.get("g", 0.0))
    c.mu = float(cfg.get("mu", 0.0))
    c.kappa = float(cfg.get("kappa", 0.0))
    c.K = float(cfg.get("K", 1.1))
    c.cfl = float(cfg.get("cfl", 0.4))
    c.low_mach = int(cfg.get("low_mach", 1))
    c.dt_mode = int(cfg.get("dt_mode", 0))
    bc = cfg.get("bc", [[BC_PERIODIC, BC_PERIODIC]] * 3)
    for a in range(3):
        for s in range(2):
            c.bc[a][s] = int(bc[a][s]) if a < len(bc) else BC_PERIODIC
    c.wall_noslip = int(cfg.get("wall_noslip", 1))
    th = cfg.get("thermal", [0, 0])
    c.thermal[0], c.thermal[1] = int(th[0]), int(th[1])
    tw = cfg.get("T_wall", [1.0, 1.0])
    c.T_wall[0], c.T_wall[1] = float(tw[0]), float(tw[1])
    c.energy_form = int(cfg.get("energy_form", 0))
    return c


def revolve_plan(n: int, s: int):
    """Binomial checkpointing actions [(op, step, arg)] and the forward steps
    they advance (see ars_revolve_plan in include/ars.h)."""
    L = lib()
    cnt = L.ars_revolve_plan(int(n), int(s), None, 0, None)
    if cnt < 0:
        raise ArsError(cnt, "ars_revolve_plan")
    buf = (C.c_int32 * (4 * cnt))()
    fwd = C.c_int64(0)
    L.ars_revolve_plan(int(n), int(s), buf, cnt, C.byref(fwd))
    acts = [(buf[4 * i], buf[4 * i + 1], buf[4 * i + 2]) for i in range(cnt)]
    return acts, fwd.value


def revolve_cost(n: int, s: int) -> int:
    return lib().ars_revolve_cost(int(n), int(s))


def validate(cfg: dict) -> int:
    c = make_config(cfg)
    return lib().ars_validate(C.byref(c))


def _check(rc, what):
    if rc != OK:
        raise ArsError(rc, what)


def state_shape(cfg: dict):
    return (int(cfg["dim"]) + 2,) + tuple(int(cfg["n"][a]) for a in reversed(range(cfg["dim"])))


class Context:
    """Owns an ars_ctx (host memory only)."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self._c = make_config(cfg)
        h = C.c_void_p()
        _check(lib().ars_create(C.byref(self._c), C.byref(h)), "ars_create")
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.ars_destroy(self.h)
            self.h = None

    @property
    def state_len(self):
        return lib().ars_state_len(self.h)

    @property
    def workspace_bytes(self):
        return lib().ars_workspace_bytes(self.h)

    def init_host(self, problem: int, params=(), seed: int = 0) -> np.ndarray:
        out = np.zeros(state_shape(self.cfg), dtype=np.float64)
        p = np.asarray(list(params) + [0.0], dtype=np.float64)
        _check(lib().ars_init_state_host(self.h, int(problem), p.ctypes.data_as(_DP), len(params),
                                         C.c_uint64(seed), out.ctypes.data_as(_DP)), "ars_init_state_host")
        return out

    def set_zchunk(self, z: int):
        _check(lib().ars_set_zchunk(self.h, int(z)), "ars_set_zchunk")

    def set_tile3(self, tile: int):
        """3D tile of the fused step: TILE3_32x10 (default) or TILE3_16x20."""
        _check(lib().ars_set_tile3(self.h, int(tile)), "ars_set_tile3")

    @property
    def tile3(self) -> int:
        return lib().ars_get_tile3(self.h)

    def set_tiling(self, zchunk: int, wg_per_cu: int = 0):
        _check(lib().ars_set_tiling(self.h, int(zchunk), int(wg_per_cu)), "ars_set_tiling")

    def tiling(self):
        z, w = C.c_int(0), C.c_int(0)
        _check(lib().ars_get_tiling(self.h, C.byref(z), C.byref(w)), "ars_get_tiling")
        return z.value, w.value

    def zchunk(self) -> int:
        return lib().ars_get_zchunk(self.h)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


class Solver:
    """Device state + workspace for one problem; every call goes through the
    C ABI on torch's current stream."""

    def __init__(self, cfg: dict, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("ars.Solver needs a GPU (no CPU fallback)")
        self.torch = torch
        self.ctx = Context(cfg)
        self.cfg = self.ctx.cfg
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device(self.device.type, torch.cuda.current_device())
        shape = state_shape(cfg)
        self.U = torch.zeros(shape, dtype=torch.float64, device=self.device)
        self.tmp = torch.empty_like(self.U)
        self.work = torch.zeros(self.ctx.workspace_bytes, dtype=torch.uint8, device=self.device)
        self.t = torch.zeros(1, dtype=torch.float64, device=self.device)
        self.dt = torch.zeros(1, dtype=torch.float64, device=self.device)
        self._wref = None
        self._wimex = None
        _check(lib().ars_workspace_init(self.ctx.h, _ptr(self.work), self.stream), "ars_workspace_init")

    @property
    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _arg(self, x, n, name):
        """Device pointer of a caller tensor after checking what the C ABI
        assumes of it: FP64, contiguous, on this solver's device, and at
        least n elements (a kernel would otherwise read or write past it)."""
        if x is None:
            return None
        t = self.torch
        if not isinstance(x, t.Tensor) or x.dtype != t.float64 or not x.is_contiguous() or x.device != self.device \
                or x.numel() < n:
            raise ValueError(f"{name}: need a contiguous float64 tensor of >= {n} elements on {self.device}")
        return _ptr(x)

    def init(self, problem: int, params=(), seed: int = 0):
        p = np.asarray(list(params) + [0.0], dtype=np.float64)
        _check(lib().ars_init_state(self.ctx.h, int(problem), p.ctypes.data_as(_DP), len(params),
                                    C.c_uint64(seed), _ptr(self.U), self.stream), "ars_init_state")
        self.t.zero_()
        self.compute_dt()
        return self

    def init_rb_dT(self, params, dT, u0=None):
        """Rayleigh-Benard base (params as for PROB_RB) with the device
        temperature perturbation field dT (and optional initial velocity u0,
        shape (dim, ...)); t = 0 and dt from the new state."""
        p = np.asarray(list(params)[:3] + [0.0], dtype=np.float64)
        n = self.ctx.state_len // (self.cfg["dim"] + 2)
        _check(lib().ars_init_rb_dT(self.ctx.h, p.ctypes.data_as(_DP), min(len(params), 3), self._arg(dT, n, "dT"),
                                    self._arg(u0, self.cfg["dim"] * n, "u0"), _ptr(self.U), self.stream),
               "ars_init_rb_dT")
        self.t.zero_()
        self.compute_dt()
        return self

    def init_rb_dT_adjoint(self, U0, lam, out=None):
        """(dU0/d dT)^T lam at the state U0 built by init_rb_dT."""
        t = self.torch
        n = self.ctx.state_len // (self.cfg["dim"] + 2)
        if out is None:
            out = t.empty(U0.shape[1:], dtype=t.float64, device=self.device)
        L = self.ctx.state_len
        _check(lib().ars_init_rb_dT_adjoint(self.ctx.h, self._arg(U0, L, "U0"), self._arg(lam, L, "lam"),
                                            self._arg(out, n, "out"), self.stream), "ars_init_rb_dT_adjoint")
        return out

    def set_state(self, U):
        self.U.copy_(self.torch.as_tensor(U, dtype=self.torch.float64).to(self.device))
        self.compute_dt()
        return self

    def compute_dt(self):
        _check(lib().ars_compute_dt(self.ctx.h, _ptr(self.U), _ptr(self.work), _ptr(self.dt), self.stream),
               "ars_compute_dt")
        return self.dt

    def step(self, n: int = 1, dt_log=None):
        _check(lib().ars_step(self.ctx.h, _ptr(self.U), _ptr(self.tmp), _ptr(self.work), int(n), _ptr(self.t),
                              _ptr(self.dt), _ptr(dt_log) if dt_log is not None else None, self.stream),
               "ars_step")
        return self

    def capture(self, n: int):
        """Record n steps (one ars_step call: control preparation, n fused
        launches, the copy back after an odd count, the dt finish) into a
        graph on a capture stream.  Nothing runs while recording; every
        graph.replay() then advances this solver's state, t and dt by n
        steps exactly as step(n) would, with one launch from the host."""
        g = self.torch.cuda.CUDAGraph()
        with self.torch.cuda.graph(g):
            self.step(n)
        return g

    def step_sched(self, dt_sched):
        dt_sched = dt_sched.to(self.device, self.torch.float64).contiguous()
        _check(lib().ars_step_sched(self.ctx.h, _ptr(self.U), _ptr(self.tmp), _ptr(self.work), dt_sched.numel(),
                                    _ptr(dt_sched), _ptr(self.t), self.stream), "ars_step_sched")
        return self

    def step_to(self, U_in, U_out, a, b, n, dt_log=None):
        """n CFL steps from U_in (read only) into U_out with the scratch
        states a, b and no copy (ars_step_to); self.U is not touched,
        self.t and self.dt are advanced, dt_log (n doubles) receives the
        dts."""
        L = self.ctx.state_len
        _check(lib().ars_step_to(self.ctx.h, self._arg(U_in, L, "U_in"), self._arg(a, L, "a"), self._arg(b, L, "b"),
                                 self._arg(U_out, L, "U_out"), _ptr(self.work), int(n), _ptr(self.t), _ptr(self.dt),
                                 self._arg(dt_log, int(n), "dt_log"), self.stream), "ars_step_to")
        return U_out

    def step_sched_to(self, U_in, U_out, a, b, dt_sched):
        """len(dt_sched) steps from U_in (read only) into U_out with the
        scratch states a, b and no copy (ars_step_sched_to); self.U is not
        touched, self.t is advanced."""
        dt_sched = dt_sched.to(self.device, self.torch.float64).contiguous()
        L = self.ctx.state_len
        _check(lib().ars_step_sched_to(self.ctx.h, self._arg(U_in, L, "U_in"), self._arg(a, L, "a"),
                                       self._arg(b, L, "b"), self._arg(U_out, L, "U_out"), _ptr(self.work),
                                       dt_sched.numel(), _ptr(dt_sched), _ptr(self.t), self.stream),
               "ars_step_sched_to")
        return U_out

    def step_ref(self, dt_sched):
        if self._wref is None:
            nb = lib().ars_workspace_bytes_ref(self.ctx.h)
            self._wref = self.torch.empty(nb, dtype=self.torch.uint8, device=self.device)
        dt_sched = dt_sched.to(self.device, self.torch.float64).contiguous()
        _check(lib().ars_step_ref(self.ctx.h, _ptr(self.U), _ptr(self.tmp), _ptr(self.work), _ptr(self._wref),
                                  dt_sched.numel(), _ptr(dt_sched), self.stream), "ars_step_ref")
        return self

    def imex_workspace(self):
        """The IMEX step's device workspace (allocated on first use)."""
        if self._wimex is None:
            self._wimex = self.torch.empty(lib().ars_workspace_bytes_imex(self.ctx.h), dtype=self.torch.uint8,
                                           device=self.device)
        return self._wimex

    def step_imex(self, dt_sched, tol=1e-13, max_iter=2000):
        """Implicit acoustic steps (ars_step_imex), dt of step s =
        dt_sched[s]; returns the total solver iterations."""
        t = self.torch
        dt_sched = t.as_tensor(dt_sched, dtype=t.float64).to(self.device).contiguous()
        self.imex_workspace()
        its = C.c_int(0)
        _check(lib().ars_step_imex(self.ctx.h, _ptr(self.U), _ptr(self.tmp), _ptr(self.work), _ptr(self._wimex),
                                   int(dt_sched.numel()), _ptr(dt_sched), _ptr(self.t), float(tol), int(max_iter),
                                   C.byref(its), self.stream), "ars_step_imex")
        return its.value

    def adjoint_workspace(self, ref=False):
        attr = "_wadj_ref" if ref else "_wadj"
        if getattr(self, attr, None) is None:
            f = lib().ars_workspace_bytes_adjoint_ref if ref else lib().ars_workspace_bytes_adjoint
            setattr(self, attr, self.torch.empty(f(self.ctx.h), dtype=self.torch.uint8, device=self.device))
        return getattr(self, attr)

    def step_adjoint(self, U_n, lam_np1, dt, lam_n=None, param_grad=None, ref=False):
        """lam_n = (dU^{n+1}/dU^n)^T lam_np1 at frozen dt (a 1-element device
        tensor); param_grad (2-element device tensor) accumulates the mu and
        kappa derivatives.  ref=True runs the reference (phase-kernel) path.
        Returns lam_n."""
        t = self.torch
        if lam_n is None:
            lam_n = t.empty_like(lam_np1)
        dt = dt.to(self.device, t.float64).reshape(-1)
        w = self.adjoint_workspace(ref)
        L = self.ctx.state_len
        name = "ars_step_adjoint_ref" if ref else "ars_step_adjoint"
        _check(getattr(lib(), name)(self.ctx.h, self._arg(U_n, L, "U_n"), self._arg(lam_np1, L, "lam_np1"),
                                    self._arg(lam_n, L, "lam_n"), self._arg(dt, 1, "dt"),
                                    self._arg(param_grad, 2, "param_grad"), _ptr(w), self.stream), name)
        return lam_n

    def kinetic_energy(self, U=None, grad=None, out=None):
        """Device scalar KE of U (default: the solver state); fills grad (state
        layout) with dKE/dU when given."""
        t = self.torch
        U = self.U if U is None else U
        out = t.zeros(1, dtype=t.float64, device=self.device) if out is None else out
        L = self.ctx.state_len
        _check(lib().ars_kinetic_energy(self.ctx.h, self._arg(U, L, "U"), self._arg(grad, L, "grad"),
                                        self._arg(out, 1, "out"), _ptr(self.work), self.stream),
               "ars_kinetic_energy")
        return out

    def nusselt(self, side=0, U=None, grad=None, out=None):
        """Device scalar Nusselt number at the bottom (side 0) or top (1)
        fixed-T wall; fills grad (state layout) with dNu/dU when given."""
        t = self.torch
        U = self.U if U is None else U
        out = t.zeros(1, dtype=t.float64, device=self.device) if out is None else out
        L = self.ctx.state_len
        _check(lib().ars_nusselt(self.ctx.h, self._arg(U, L, "U"), int(side), self._arg(grad, L, "grad"),
                                 self._arg(out, 1, "out"), _ptr(self.work), self.stream), "ars_nusselt")
        return out

    def spectrum(self, kz=None, U=None, out=None):
        """Device tensor of the kinetic-energy spectrum of the horizontal
        plane kz (default: the middle plane n_z // 2), ``ars_spectrum``."""
        t = self.torch
        U = self.U if U is None else U
        h = self.ctx.h
        kz = int(self.cfg["n"][int(self.cfg["dim"]) - 1]) // 2 if kz is None else int(kz)
        if getattr(self, "_wspec", None) is None:
            self._wspec = t.empty(lib().ars_workspace_bytes_spectrum(h), dtype=t.uint8, device=self.device)
        ns = lib().ars_spectrum_len(h)
        if out is None:
            out = t.empty(ns, dtype=t.float64, device=self.device)
        _check(lib().ars_spectrum(h, self._arg(U, self.ctx.state_len, "U"), kz, self._arg(out, ns, "out"),
                                  _ptr(self._wspec), self.stream), "ars_spectrum")
        return out

    def diagnostics(self, raise_on_fault=True) -> dict:
        d = ArsDiag()
        rc = lib().ars_diagnostics(self.ctx.h, _ptr(self.U), _ptr(self.work), C.byref(d), self.stream)
        if rc not in (OK, ENONPHYS) or (rc == ENONPHYS and raise_on_fault):
            raise ArsError(rc, f"ars_diagnostics (fault cell {d.fault_cell})")
        return dict(mass=d.mass, mom=list(d.mom), e_total=d.e_total, e_kin=d.e_kin, e_int=d.e_int,
                    e_grav=d.e_grav, max_u=d.max_u, mean_u=d.mean_u, max_mach=d.max_mach, nu_bot=d.nu_bot,
                    nu_top=d.nu_top, fault=d.fault, fault_cell=d.fault_cell)

    def autotune(self, trial_steps: int = 10, cache_path=None) -> dict:
        """Time candidate launch shapes of the fused step on a copy of the
        current state and keep the fastest (``ars_autotune``)."""
        r = ArsTuneResult()
        _check(lib().ars_autotune(self.ctx.h, _ptr(self.U), _ptr(self.work), int(trial_steps),
                                  cache_path.encode() if cache_path else None, self.stream, C.byref(r)),
               "ars_autotune")
        return r.as_dict()

    def fault(self):
        fc = C.c_int64(-1)
        rc = lib().ars_fault(self.ctx.h, _ptr(self.work), C.byref(fc), self.stream)
        return rc, fc.value

    def numpy(self):
        return self.U.detach().cpu().numpy()


class Batch:
    """Many independent 2D problems advanced by one persistent launch
    (``ars_batch_*``).  ``cfgs``: list of config dicts.  ``states`` is one
    flat device array; ``view(k)`` is instance k in state layout."""

    def __init__(self, cfgs, device="cuda"):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("ars.Batch needs a GPU (no CPU fallback)")
        self.torch = torch
        self.cfgs = [dict(c) for c in cfgs]
        self.n = len(self.cfgs)
        arr = (ArsConfig * self.n)(*[make_config(c) for c in self.cfgs])
        h = _VP()
        _check(lib().ars_batch_create(self.n, arr, C.byref(h)), "ars_batch_create")
        self.h = h
        self.device = torch.device(device)
        L = lib()
        self.len = L.ars_batch_state_len(h)
        self.off = [L.ars_batch_state_offset(h, k) for k in range(self.n)]
        self.states = torch.zeros(self.len, dtype=torch.float64, device=self.device)
        self.tmps = torch.zeros_like(self.states)
        self.table = torch.zeros(L.ars_batch_table_bytes(h), dtype=torch.uint8, device=self.device)
        self.bind()

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ars_batch_destroy(h)
            self.h = None

    @property
    def stream(self):
        return C.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def view(self, k):
        shape = state_shape(self.cfgs[k])
        n = int(np.prod(shape))
        return self.states[self.off[k]:self.off[k] + n].view(shape)

    def bind(self):
        _check(lib().ars_batch_bind(self.h, _ptr(self.states), _ptr(self.tmps), _ptr(self.table), self.stream),
               "ars_batch_bind")
        return self

    def set_tiling(self, rows, zc=None):
        z = (C.c_int * self.n)(*[int(v) for v in zc]) if zc is not None else None
        _check(lib().ars_batch_set_tiling(self.h, int(rows), z), "ars_batch_set_tiling")
        return self

    def tiling(self):
        r = C.c_int(0)
        z = (C.c_int * self.n)()
        _check(lib().ars_batch_get_tiling(self.h, C.byref(r), z), "ars_batch_get_tiling")
        return r.value, list(z)

    def autotune(self, trial_steps: int = 5, cache_path=None) -> dict:
        """Time candidate tilings of the batched launch on the current
        states (restored afterwards), apply the fastest and rebind (t = 0)."""
        r = ArsTuneResult()
        _check(lib().ars_batch_autotune(self.h, _ptr(self.states), _ptr(self.tmps), _ptr(self.table),
                                        int(trial_steps), cache_path.encode() if cache_path else None, self.stream,
                                        C.byref(r)), "ars_batch_autotune")
        return r.as_dict()

    def step(self, n):
        _check(lib().ars_batch_step(self.h, _ptr(self.table), int(n), self.stream), "ars_batch_step")
        return self

    def capture(self, n, stream):
        """Capture an n-step launch on ``stream`` (a non-default torch stream)."""
        _check(lib().ars_batch_capture(self.h, _ptr(self.table), int(n), C.c_void_p(stream.cuda_stream)),
               "ars_batch_capture")
        return self

    def replay(self, stream):
        _check(lib().ars_batch_replay(self.h, C.c_void_p(stream.cuda_stream)), "ars_batch_replay")
        return self

    def read(self):
        """(t, next dt, fault cell per instance (-1: none), status)."""
        t = np.zeros(self.n)
        dt = np.zeros(self.n)
        fc = (C.c_int64 * self.n)()
        rc = lib().ars_batch_read(self.h, _ptr(self.table), t.ctypes.data_as(_DP), dt.ctypes.data_as(_DP), fc,
                                  self.stream)
        if rc not in (OK, ENONPHYS):
            raise ArsError(rc, "ars_batch_read")
        return t, dt, np.array(list(fc), dtype=np.int64), rc
