"""CPU oracle of the all-regime well-balanced step (arXiv 1903.09043).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of bench.py.  The product package never imports it.

Thin ctypes wrapper over ``libars_oracle.so`` (built by ``oracle/build.py``).
Every routine is plain serial FP64 C++ (OpenMP only splits independent cell
loops); see ``ars_oracle.cpp`` for the passage of the paper each step follows.

Problem ids for :func:`init` (params in order):
  0 uniform      : rho, u0, u1, u2, p
  1 RB linear T  : T_bottom, T_top, rho of the bottom cell (<=0: T of that cell), amp
                   (hydrostatic base from eq. (well_balanced_formula), seeded
                   temperature perturbation dT = amp * (2 U - 1), U from SplitMix64)
  2 Gresho       : Ma   (Sec. 4.2, p0 = 1 / (gamma Ma^2))
  3 Sod          : -    (Sec. 4.1)
  4 isothermal   : -    (Sec. 4.3, p = rho, T = 1, rho_0 = exp(-g z_0))
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libars_oracle.so")

BC_PERIODIC, BC_WALL, BC_OUTFLOW = 0, 1, 2
TH_ADIABATIC, TH_FIXED = 0, 1
PROB_UNIFORM, PROB_RB, PROB_GRESHO, PROB_SOD, PROB_ISOTHERMAL = 0, 1, 2, 3, 4
OK, EINVAL, ENONPHYS = 0, -1, -4


class OrcConfig(C.Structure):
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


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        cp = C.POINTER(OrcConfig)
        i64p = C.POINTER(C.c_int64)
        L.orc_validate.argtypes = [cp]
        L.orc_max_rate.argtypes = [cp, dp]
        L.orc_max_rate.restype = C.c_double
        L.orc_dt.argtypes = [cp, dp]
        L.orc_dt.restype = C.c_double
        L.orc_step_dt.argtypes = [cp, dp, dp, C.c_double, i64p]
        L.orc_run.argtypes = [cp, dp, C.c_int, dp, dp, dp, i64p, i64p]
        L.orc_tlm.argtypes = [cp, dp, dp, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_adjoint_dense.argtypes = [cp, dp, dp, C.c_double, dp, dp, dp]
        L.orc_init.argtypes = [cp, C.c_int, dp, C.c_int, C.c_uint64, dp]
        L.orc_face.argtypes = [cp, C.c_int] + [C.c_double] * 8 + [C.c_int, dp]
        L.orc_face.restype = None
        L.orc_diag.argtypes = [cp, dp, dp]
        L.orc_diag.restype = None
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_long, C.POINTER(C.c_uint64)]
        L.orc_splitmix64.restype = None
        L.orc_num_threads.restype = C.c_int
        L.orc_imex_system.argtypes = [cp, dp, C.c_double, C.c_int64, i64p, i64p, dp, dp, i64p]
        L.orc_imex_residual.argtypes = [cp, dp, C.c_double, dp, dp]
        L.orc_step_imex_x.argtypes = [cp, dp, dp, C.c_double, dp, i64p]
        _lib = L
    return _lib


def make_config(cfg: dict) -> OrcConfig:
    """Build the C struct from a plain dict (same keys as the product's)."""
    c = OrcConfig()
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
    th = cfg.get("thermal", [TH_ADIABATIC, TH_ADIABATIC])
    c.thermal[0], c.thermal[1] = int(th[0]), int(th[1])
    tw = cfg.get("T_wall", [1.0, 1.0])
    c.T_wall[0], c.T_wall[1] = float(tw[0]), float(tw[1])
    c.energy_form = int(cfg.get("energy_form", 0))
    return c


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def ncell(cfg: dict) -> int:
    n = 1
    for a in range(cfg["dim"]):
        n *= int(cfg["n"][a])
    return n


def nvar(cfg: dict) -> int:
    return int(cfg["dim"]) + 2


def state_shape(cfg: dict):
    """(nvar, n_{D-1}, ..., n_0): var-major SoA, x fastest."""
    return (nvar(cfg),) + tuple(int(cfg["n"][a]) for a in reversed(range(cfg["dim"])))


def validate(cfg: dict) -> int:
    c = make_config(cfg)
    return lib().orc_validate(C.byref(c))


def init(cfg: dict, problem: int, params=(), seed: int = 0) -> np.ndarray:
    c = make_config(cfg)
    U = np.zeros(state_shape(cfg), dtype=np.float64)
    p = np.asarray(list(params) + [0.0], dtype=np.float64)
    rc = lib().orc_init(C.byref(c), int(problem), _dp(p), len(params), C.c_uint64(seed), _dp(U))
    if rc != OK:
        raise ValueError(f"orc_init failed: {rc}")
    return U


def max_rate(cfg: dict, U: np.ndarray) -> float:
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_max_rate(C.byref(c), _dp(U))


def dt(cfg: dict, U: np.ndarray) -> float:
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    return lib().orc_dt(C.byref(c), _dp(U))


def step_dt(cfg: dict, U: np.ndarray, dt_: float):
    """One step with a given dt.  Returns (U_new, status, fault_cell)."""
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.empty_like(U)
    fc = C.c_int64(-1)
    rc = lib().orc_step_dt(C.byref(c), _dp(U), _dp(out), float(dt_), C.byref(fc))
    return out, rc, fc.value


def run(cfg: dict, U: np.ndarray, nsteps: int, dt_sched=None, t0: float = 0.0):
    """n steps (dt from the CFL rule on each input state unless dt_sched).

    Returns dict(U, t, dt_log, status, fault_cell, fault_step)."""
    c = make_config(cfg)
    U = np.array(U, dtype=np.float64, copy=True, order="C")
    log = np.zeros(max(nsteps, 1), dtype=np.float64)
    t = C.c_double(t0)
    fc = C.c_int64(-1)
    fs = C.c_int64(-1)
    sched = None
    if dt_sched is not None:
        sched = np.ascontiguousarray(dt_sched, dtype=np.float64)
    rc = lib().orc_run(C.byref(c), _dp(U), int(nsteps), _dp(sched) if sched is not None else None,
                       _dp(log), C.byref(t), C.byref(fc), C.byref(fs))
    return dict(U=U, t=t.value, dt_log=log[:nsteps], status=rc, fault_cell=fc.value, fault_step=fs.value)


def tlm(cfg: dict, U, dU, dt_: float, dmu: float = 0.0, dkappa: float = 0.0):
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    dUa = np.ascontiguousarray(dU, dtype=np.float64) if dU is not None else None
    out = np.empty_like(U)
    dout = np.empty_like(U)
    rc = lib().orc_tlm(C.byref(c), _dp(U), _dp(dUa) if dUa is not None else None, float(dmu), float(dkappa),
                       float(dt_), _dp(out), _dp(dout))
    return out, dout, rc


def adjoint_dense(cfg: dict, U, lam, dt_: float):
    """Brute-force reverse product (J^T lam, <lam, dU'/dmu>, <lam, dU'/dkappa>)."""
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    out = np.empty_like(U)
    gm = C.c_double(0.0)
    gk = C.c_double(0.0)
    lib().orc_adjoint_dense(C.byref(c), _dp(U), _dp(lam), float(dt_), _dp(out), C.byref(gm), C.byref(gk))
    return out, gm.value, gk.value


def face(cfg: dict, d: int, L, R, phiL=0.0, phiR=0.0, wall=False):
    """Face solver on (rho, u_d, p) pairs -> dict(a, S, ustar, theta, pistar, P)."""
    c = make_config(cfg)
    out = np.zeros(6, dtype=np.float64)
    lib().orc_face(C.byref(c), int(d), float(L[0]), float(L[1]), float(L[2]), float(R[0]), float(R[1]),
                   float(R[2]), float(phiL), float(phiR), int(bool(wall)), _dp(out))
    return dict(zip(["a", "S", "ustar", "theta", "pistar", "P"], out.tolist()))


DIAG_KEYS = ["mass", "mom0", "mom1", "mom2", "e_total", "e_kin", "e_int", "e_grav",
             "max_u", "mean_u", "max_mach", "nu_bot", "nu_top"]


def diag(cfg: dict, U) -> dict:
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros(13, dtype=np.float64)
    lib().orc_diag(C.byref(c), _dp(U), _dp(out))
    return dict(zip(DIAG_KEYS, out.tolist()))


def spectrum(cfg: dict, U, kz: int) -> np.ndarray:
    """Kinetic-energy spectrum of the horizontal plane kz (Sec. 4.5, 3D case:
    the mid-plane spectrum figure; the paper gives no formula).  Reading:
    w_c = sqrt(rho) u_c on the plane (all velocity components), its discrete
    Fourier transform W_c(k) = sum_x w_c(x) exp(-2 pi i k.x / n) (numpy's
    FFT, the library primitive), and E(s) = sum over integer wave vectors k
    with round(|k|) = s of sum_c |W_c(k)|^2 / (2 N^2), N the number of cells
    of the plane; so sum_s E(s) is the plane mean of rho |u|^2 / 2
    (Parseval); one shell per integer s up to the largest round(|k|).  In 2D
    the plane is a line and k = |k_x|."""
    D = cfg["dim"]
    U = np.asarray(U, dtype=np.float64)
    rho = U[0][kz]
    w = [np.sqrt(rho) * (U[1 + c][kz] / rho) for c in range(D)]
    if D == 3:
        ny, nx = rho.shape
        kx = np.rint(np.fft.fftfreq(nx) * nx)
        ky = np.rint(np.fft.fftfreq(ny) * ny)
        kk = np.sqrt(ky[:, None] ** 2 + kx[None, :] ** 2)
        P = sum(np.abs(np.fft.fft2(wc)) ** 2 for wc in w)
        N = nx * ny
    else:
        nx = rho.shape[0]
        kk = np.abs(np.rint(np.fft.fftfreq(nx) * nx))
        P = sum(np.abs(np.fft.fft(wc)) ** 2 for wc in w)
        N = nx
    shell = np.rint(kk).astype(np.int64)
    nshell = int(shell.max()) + 1
    E = np.bincount(shell.ravel(), weights=P.ravel(), minlength=nshell)[:nshell]
    return E / (2.0 * N * N)


def imex_system(cfg: dict, U, dt_: float):
    """Sparse matrix L (scipy CSR) and right-hand side b of the implicit
    acoustic system L x = b of one IMEX step from U with time step dt
    (ars_oracle.cpp, IMEX section); x = [Pi | u_0 | ... | u_{D-1}]."""
    import scipy.sparse as sp
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    D = cfg["dim"]
    n = (D + 1) * ncell(cfg)
    cap = n * (8 * D + 4)
    while True:
        rows = np.zeros(cap, dtype=np.int64)
        cols = np.zeros(cap, dtype=np.int64)
        vals = np.zeros(cap)
        rhs = np.zeros(n)
        nnz = C.c_int64(0)
        rc = lib().orc_imex_system(C.byref(c), _dp(U), float(dt_), cap, rows.ctypes.data_as(C.POINTER(C.c_int64)),
                                   cols.ctypes.data_as(C.POINTER(C.c_int64)), _dp(vals), _dp(rhs), C.byref(nnz))
        if rc == OK:
            break
        if nnz.value <= cap:
            raise ValueError("orc_imex_system failed")
        cap = nnz.value
    k = nnz.value
    return sp.csr_matrix((vals[:k], (rows[:k], cols[:k])), shape=(n, n)), rhs


def imex_residual(cfg: dict, U, dt_: float, x) -> np.ndarray:
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    r = np.zeros_like(x)
    assert lib().orc_imex_residual(C.byref(c), _dp(U), float(dt_), _dp(x), _dp(r)) == OK
    return r


def step_imex(cfg: dict, U, dt_: float):
    """One IMEX step: the implicit system solved by a direct sparse solver
    (the solution is that of the plain definition, a linear solve), then
    the step with its interface values.  Returns (U_new, status, x)."""
    import scipy.sparse.linalg as spl
    Lm, b = imex_system(cfg, U, dt_)
    x = spl.spsolve(Lm.tocsc(), b)
    c = make_config(cfg)
    U = np.ascontiguousarray(U, dtype=np.float64)
    out = np.zeros_like(U)
    fc = C.c_int64(-1)
    rc = lib().orc_step_imex_x(C.byref(c), _dp(U), _dp(np.ascontiguousarray(x)), float(dt_), _dp(out), C.byref(fc))
    return out, rc, x


def run_imex(cfg: dict, U, nsteps: int, dt_):
    """nsteps IMEX steps with a fixed time step (or a list of them)."""
    U = np.array(U, dtype=np.float64)
    sched = list(dt_) if hasattr(dt_, "__len__") else [float(dt_)] * nsteps
    for s in range(nsteps):
        U, rc, _ = step_imex(cfg, U, sched[s])
        if rc != OK:
            return {"U": U, "status": rc, "steps": s + 1}
    return {"U": U, "status": OK, "steps": nsteps}


def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_splitmix64(C.c_uint64(seed), n, out.ctypes.data_as(C.POINTER(C.c_uint64)))
    return out


def num_threads() -> int:
    return lib().orc_num_threads()
