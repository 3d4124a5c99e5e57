"""GPU parity of the HIP step against the CPU oracle (run on an MI355X).

Acceptance (FP64): |gpu - oracle| <= 1e-12 * max(|oracle|, s_v) cell-wise,
s_v the magnitude scale of that variable (tests/parity.py: its largest
value; for the momentum, at least the largest rho c).  The oracle evaluates the quotients of
Sec. 2.1.2 and eq. (low_mach_correction) as printed, the kernels use
reciprocal products, so the two differ by rounding; the fused kernel and the
phase-by-phase reference kernels (two GPU paths with the same expression
trees) are compared bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_09043_amd import workloads as W
from tests import inputs as I
from tests import parity as P

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1903_09043_amd as A
    A.lib()
    return A


def close(cfg, g, o):
    """Parity measure of tests/parity.py (momentum on the acoustic scale);
    the measure with every variable on its own largest value is printed."""
    e = P.rel_err(cfg, g, o)
    say("    parity %.3e (each variable on its own max: %.3e)" % (e, P.strict_err(g, o)))
    return e


def bitwise(g, o):
    return np.array_equal(np.asarray(g), np.asarray(o))


def gpu_run(A, cfg, U0, nsteps, zchunk=None):
    import torch
    S = A.Solver(cfg)
    if zchunk:
        S.ctx.set_zchunk(zchunk)
    S.set_state(U0)
    log = torch.zeros(max(nsteps, 1), dtype=torch.float64, device="cuda")
    S.step(nsteps, dt_log=log)
    torch.cuda.synchronize()
    rc, fc = S.fault()
    return S.numpy(), log.cpu().numpy()[:nsteps], S.t.item(), rc, fc


def test_init_bitwise_and_dt(A):
    """Initial states are built by the same formulas on both sides (bitwise);
    the first CFL time step agrees to rounding (the rate's sound speed is a
    reciprocal product on the GPU, a quotient in the oracle)."""
    import torch
    for make in (W.rb2d_64x32, lambda: W.rb([20, 12, 10], [1.0, 1.0, 1.0], Ra=1e5, seed=3),
                 lambda: W.gresho(n=64)):
        cfg, prob, prm, seed = make()
        say("init/dt", cfg["n"])
        S = A.Solver(cfg).init(prob, prm, seed)
        torch.cuda.synchronize()
        U = S.numpy()
        Uo = O.init(cfg, prob, prm, seed)
        assert bitwise(U, Uo)
        dto = O.dt(cfg, Uo)
        assert abs(S.dt.item() - dto) <= 1e-14 * dto


def test_rb2d_64x32_1000_steps(A):
    """2D RB 64x32, Ra = 1e4, theta on, 1000 steps: the workload of the
    parity requirement."""
    cfg, prob, prm, seed = W.rb2d_64x32()
    Uo0 = O.init(cfg, prob, prm, seed)
    say("rb2d 64x32 gpu")
    U, log, t, rc, fc = gpu_run(A, cfg, Uo0, 1000)
    assert rc == 0
    say("rb2d 64x32 oracle")
    r = O.run(cfg, Uo0, 1000)
    err = close(cfg, U, r["U"])
    say("rb2d 64x32 max rel err", err, "bitwise", bitwise(U, r["U"]))
    assert err <= 1e-12
    np.testing.assert_allclose(log, r["dt_log"], rtol=1e-13)
    assert abs(t - r["t"]) <= 1e-12 * r["t"]


CASES = {
    # name: (cfg, U0-builder, steps, zchunk)
    "rb2d_ragged": (lambda: W.rb([100, 37], [2.0, 1.0], Ra=3e3, seed=11, amp=1e-2), 60, 7),
    "rb2d_thetaoff": (lambda: W.rb([64, 32], [2.0, 1.0], Ra=1e4, seed=1, amp=1e-2, low_mach=0), 60, None),
    "rb3d_ragged": (lambda: W.rb([37, 29, 23], [1.3, 1.0, 1.0], Ra=1e5, seed=4, amp=1e-2), 25, 6),
    "rb3d_thetaoff": (lambda: W.rb([20, 16, 12], [1.0, 1.0, 1.0], Ra=1e5, seed=2, amp=1e-2, low_mach=0), 25, None),
    "gresho_on": (lambda: W.gresho(n=128, Ma=1e-2, low_mach=1), 100, None),
    "gresho_off": (lambda: W.gresho(n=96, Ma=1e-2, low_mach=0), 100, 13),
}


@pytest.mark.parametrize("name", list(CASES))
def test_step_vs_oracle(A, name):
    make, nsteps, zc = CASES[name]
    cfg, prob, prm, seed = make()
    Uo0 = O.init(cfg, prob, prm, seed)
    if cfg["g"] != 0.0:
        # add a velocity field so every flux term is exercised
        rng = np.random.default_rng(7)
        D = cfg["dim"]
        for k in range(D):
            Uo0[1 + k] = 1e-2 * rng.standard_normal(Uo0[0].shape) * Uo0[0]
        Uo0[-1] += 0.5 * sum(Uo0[1 + k] ** 2 for k in range(D)) / Uo0[0]
    say(name, "gpu", cfg["n"])
    U, log, t, rc, fc = gpu_run(A, cfg, Uo0, nsteps, zc)
    assert rc == 0, fc
    say(name, "oracle")
    r = O.run(cfg, Uo0, nsteps)
    err = close(cfg, U, r["U"])
    say(name, "max rel err", err, "bitwise", bitwise(U, r["U"]))
    assert err <= 1e-12


def _periodic3d_cfg(bc):
    return dict(dim=3, n=[33, 26, 19], L=[1.0, 0.8, 0.6], gamma=5.0 / 3.0, g=0.0, mu=2e-3, kappa=3e-3, K=1.1,
                cfl=0.4, low_mach=1, dt_mode=0, bc=bc, wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])


@pytest.mark.parametrize("bc", ["periodic", "outflow"])
def test_3d_random_state(A, bc):
    b = [[0, 0]] * 3 if bc == "periodic" else [[2, 2], [0, 0], [2, 2]]
    cfg = _periodic3d_cfg(b)
    U0 = I.smooth_random(cfg, seed=21)
    say("3d", bc)
    U, log, t, rc, fc = gpu_run(A, cfg, U0, 20, zchunk=5)
    assert rc == 0
    r = O.run(cfg, U0, 20)
    err = close(cfg, U, r["U"])
    say("3d", bc, "max rel err", err, "bitwise", bitwise(U, r["U"]))
    assert err <= 1e-12


def test_sod_2d_outflow(A):
    cfg = dict(dim=2, n=[100, 3], L=[1.0, 1.0], gamma=1.4, g=0.0, mu=0.0, kappa=0.0, K=1.1, cfl=0.4, low_mach=1,
               dt_mode=0, bc=[[2, 2], [0, 0]], wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])
    U0 = O.init(cfg, W.PROB_SOD)
    say("sod")
    U, log, t, rc, fc = gpu_run(A, cfg, U0, 120)
    r = O.run(cfg, U0, 120)
    err = close(cfg, U, r["U"])
    say("sod max rel err", err, "bitwise", bitwise(U, r["U"]))
    assert err <= 1e-12


def test_isothermal_column_2d(A):
    """Sec. 4.3 column in 2D (periodic x, walls in y): stays at rest to the
    round-off level of Table 1, and matches the oracle."""
    for lm in (0, 1):
        cfg = dict(dim=2, n=[4, 128], L=[1.0, 3.0], gamma=5.0 / 3.0, g=1.0, mu=0.0, kappa=0.0, K=1.1, cfl=0.4,
                   low_mach=lm, dt_mode=0, bc=[[0, 0], [1, 1]], wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])
        U0 = O.init(cfg, W.PROB_ISOTHERMAL)
        say("iso", lm)
        U, log, t, rc, fc = gpu_run(A, cfg, U0, 500)
        r = O.run(cfg, U0, 500)
        assert close(cfg, U, r["U"]) <= 1e-12
        assert np.max(np.abs(U[1:3] / U[0])) < 1e-12


def test_fused_equals_reference_path(A):
    """The fused z-march kernel and the phase-by-phase reference kernels give
    the same bits, for several tile/boundary/variant combinations."""
    import torch
    cases = [W.rb([70, 33], [2.0, 1.0], Ra=2e3, seed=5, amp=1e-2),
             W.rb([30, 27, 14], [1.0, 1.0, 1.0], Ra=1e5, seed=6, amp=1e-2),
             W.gresho(n=80, Ma=1e-1, low_mach=0)]
    for cfg, prob, prm, seed in cases:
        say("fused vs ref", cfg["n"])
        S1 = A.Solver(cfg).init(prob, prm, seed)
        S2 = A.Solver(cfg).init(prob, prm, seed)
        sched = torch.full((12,), float(S1.dt.item()), dtype=torch.float64, device="cuda")
        S1.ctx.set_zchunk(5)
        S1.step_sched(sched)
        S2.step_ref(sched)
        torch.cuda.synchronize()
        assert bitwise(S1.numpy(), S2.numpy())


def test_result_independent_of_zchunk_and_tile(A):
    """Vertical shares and both 3D tiles give the same bits."""
    cfg, prob, prm, seed = W.rb([40, 24, 30], [1.0, 1.0, 1.0], Ra=1e5, seed=9, amp=1e-2)
    outs = []
    for tile, zc in ((A.TILE3_32x10, 30), (A.TILE3_32x10, 7), (A.TILE3_32x10, 1), (A.TILE3_16x20, 30),
                     (A.TILE3_16x20, 4)):
        S = A.Solver(cfg).init(prob, prm, seed)
        S.ctx.set_tile3(tile)
        S.ctx.set_zchunk(zc)
        S.step(6)
        outs.append(S.numpy())
    for o in outs[1:]:
        assert bitwise(outs[0], o)


@pytest.mark.parametrize("name", ["rb3d_ragged", "rb3d_thetaoff"])
def test_tile_16x20_vs_oracle(A, name):
    """The second 3D tile (16 x 20 outputs) against the oracle on ragged
    grids with a flow added."""
    make, nsteps, zc = CASES[name]
    cfg, prob, prm, seed = make()
    Uo0 = O.init(cfg, prob, prm, seed)
    rng = np.random.default_rng(7)
    for k in range(3):
        Uo0[1 + k] = 1e-2 * rng.standard_normal(Uo0[0].shape) * Uo0[0]
    Uo0[-1] += 0.5 * sum(Uo0[1 + k] ** 2 for k in range(3)) / Uo0[0]
    import torch
    S = A.Solver(cfg)
    S.ctx.set_tile3(A.TILE3_16x20)
    S.set_state(Uo0)
    S.step(nsteps)
    torch.cuda.synchronize()
    assert S.fault()[0] == 0
    r = O.run(cfg, Uo0, nsteps)
    err = close(cfg, S.numpy(), r["U"])
    say(name, "tile 16x20 max rel err", err)
    assert err <= 1e-12


def test_diagnostics_match_oracle(A):
    """Diagnostics of the oracle's state after 50 steps, on the GPU and in
    the oracle."""
    cfg, prob, prm, seed = W.rb2d_64x32()
    r = O.run(cfg, O.init(cfg, prob, prm, seed), 50)
    assert r["status"] == 0
    S = A.Solver(cfg).set_state(r["U"])
    d = S.diagnostics()
    o = O.diag(cfg, r["U"])
    for k in ("mass", "e_total", "e_kin", "e_int", "e_grav", "max_u", "mean_u", "max_mach", "nu_bot", "nu_top"):
        assert abs(d[k] - o[k]) <= 1e-12 * max(abs(o[k]), 1e-300) + 1e-300, k
    assert abs(d["mom"][0] - o["mom0"]) <= 1e-12 * o["mass"]


def test_fault_latch(A):
    import torch
    cfg = dict(dim=2, n=[16, 12], L=[1.0, 1.0], gamma=5.0 / 3.0, bc=[[0, 0], [0, 0]])
    U0 = O.init(cfg, W.PROB_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1.0])
    U0[0, 5, 9] = -1.0
    S = A.Solver(cfg)
    S.U.copy_(torch.as_tensor(U0).cuda())
    S.dt.fill_(1e-3)
    S.step(1)
    rc, fc = S.fault()
    r = O.run(cfg, U0, 1, dt_sched=[1e-3])
    assert rc == A.ENONPHYS and r["status"] == O.ENONPHYS
    assert fc == r["fault_cell"]
    rc2, _ = S.fault()
    assert rc2 == 0  # latch cleared by the read


def test_full_size_256cubed_one_step(A):
    """3D RB 256^3 (the benchmark workload) in the benchmark's launch
    configuration: from the oracle's state after two oracle steps, one GPU
    step (its CFL step chosen on the device) equals one oracle step on the
    whole grid."""
    import torch
    cfg, prob, prm, seed = W.rb3d_ra1e6()
    say("256^3 oracle init + 2 steps (threads=%d)" % O.num_threads())
    r = O.run(cfg, O.init(cfg, prob, prm, seed), 2)
    assert r["status"] == 0
    U2 = r["U"]
    S = A.Solver(cfg).set_state(U2)
    dt = S.dt.item()
    S.step(1)
    torch.cuda.synchronize()
    U3 = S.numpy()
    say("256^3 oracle step")
    Uo, rc, _ = O.step_dt(cfg, U2, dt)
    assert rc == 0
    dto = O.dt(cfg, U2)
    assert abs(dt - dto) <= 1e-14 * dto
    err = close(cfg, U3, Uo)
    say("256^3 max rel err", err, "bitwise", bitwise(U3, Uo))
    assert err <= 1e-12


@pytest.mark.timeout(1200)
def test_full_size_256cubed_100_steps_from_init(A):
    """3D RB 256^3 from the initial state, in the benchmark's launch
    configuration: 100 GPU steps (CFL time steps chosen on the device)
    against 100 oracle steps on the whole grid, every cell to the 1e-12
    scale-aware tolerance, and the dt log to rounding."""
    import torch
    cfg, prob, prm, seed = W.rb3d_ra1e6()
    S = A.Solver(cfg).init(prob, prm, seed)
    log = torch.zeros(100, dtype=torch.float64, device="cuda")
    S.step(100, dt_log=log)
    torch.cuda.synchronize()
    rc, fc = S.fault()
    assert rc == 0, fc
    U = S.numpy()
    t_gpu = S.t.item()
    del S
    say("256^3 x 100 oracle (threads=%d)" % O.num_threads())
    # ten runs of ten steps (each step's dt from its own state, as in one
    # run of 100), reporting progress: the oracle takes minutes here
    Uo, t, dts = O.init(cfg, prob, prm, seed), 0.0, []
    for k in range(10):
        r = O.run(cfg, Uo, 10, t0=t)
        assert r["status"] == 0
        Uo, t = r["U"], r["t"]
        dts.append(r["dt_log"])
        say("oracle steps", 10 * (k + 1), "t", t)
    np.testing.assert_allclose(log.cpu().numpy(), np.concatenate(dts), rtol=1e-13)
    assert abs(t_gpu - t) <= 1e-13 * t
    err = close(cfg, U, Uo)
    say("256^3 x 100 max rel err", err, "bitwise", bitwise(U, Uo))
    assert err <= 1e-12


@pytest.mark.timeout(900)
@pytest.mark.parametrize("lm", [1, 0])
def test_gresho_1024_full_size(A, lm):
    """2D Gresho vortex 1024^2, Mach 1e-3, periodic, theta on and off: 1000
    GPU steps equal 1000 oracle steps on the whole grid to the 1e-12
    scale-aware tolerance; then 4000 more steps on the GPU (the run length of
    the workload) keep the kinetic energy, more of it with the low-Mach
    correction than without (Sec. 4.2)."""
    import torch
    cfg, prob, prm, seed = W.gresho_1024(low_mach=lm)
    S = A.Solver(cfg).init(prob, prm, seed)
    ke0 = S.diagnostics()["e_kin"]
    log = torch.zeros(1000, dtype=torch.float64, device="cuda")
    S.step(1000, dt_log=log)
    torch.cuda.synchronize()
    U = S.numpy()
    say("gresho 1024 lm", lm, "oracle x 1000 (threads=%d)" % O.num_threads())
    # ten runs of 100 steps with progress (each step's dt from its own state)
    Uo, t, dts = O.init(cfg, prob, prm, seed), 0.0, []
    for k in range(10):
        r = O.run(cfg, Uo, 100, t0=t)
        assert r["status"] == 0
        Uo, t = r["U"], r["t"]
        dts.append(r["dt_log"])
        say("oracle steps", 100 * (k + 1), "t", t)
    np.testing.assert_allclose(log.cpu().numpy(), np.concatenate(dts), rtol=1e-13)
    err = close(cfg, U, Uo)
    say("gresho 1024 lm", lm, "1000 steps max rel err", err, "bitwise", bitwise(U, Uo))
    assert err <= 1e-12
    S.step(4000)
    d = S.diagnostics()
    ratio = d["e_kin"] / ke0
    say("gresho 1024 lm", lm, "t", S.t.item(), "KE(t)/KE(0)", ratio)
    if lm:
        assert ratio > 0.99
        test_gresho_1024_full_size.ratio_on = ratio
    else:
        assert ratio < getattr(test_gresho_1024_full_size, "ratio_on", 1.0)


def test_checkpoint_resume(A, tmp_path):
    """A run of 1000 steps equals 500 steps, a save of the state as raw FP64
    and of t, a load into a fresh solver and 500 more steps, bit for bit
    (dt of the resumed run comes from the loaded state)."""
    import torch
    cfg, prob, prm, seed = W.rb2d_64x32()
    S = A.Solver(cfg).init(prob, prm, seed)
    S.step(1000)
    torch.cuda.synchronize()
    ref, t_ref = S.numpy(), S.t.item()
    S1 = A.Solver(cfg).init(prob, prm, seed)
    S1.step(500)
    torch.cuda.synchronize()
    f = tmp_path / "state.f64"
    S1.numpy().tofile(f)
    np.array([S1.t.item()]).tofile(tmp_path / "t.f64")
    S2 = A.Solver(cfg)
    S2.set_state(np.fromfile(f, dtype=np.float64).reshape(S2.U.shape))
    S2.t.fill_(float(np.fromfile(tmp_path / "t.f64")[0]))
    S2.step(500)
    torch.cuda.synchronize()
    assert bitwise(S2.numpy(), ref) and S2.t.item() == t_ref


def _cfg(dim, n, L, bc, g=0.0, mu=2e-3, kappa=3e-3, thermal=(0, 0), T_wall=(1.0, 1.0), lm=1):
    return dict(dim=dim, n=list(n), L=list(L), gamma=5.0 / 3.0, g=g, mu=mu, kappa=kappa, K=1.1, cfl=0.4,
                low_mach=lm, dt_mode=0, bc=bc, wall_noslip=1, thermal=list(thermal), T_wall=list(T_wall))


DEGENERATE = {
    # one cell wide or tall, narrower than the tile halo, single planes
    "2d_1x7_walls": (lambda: _cfg(2, [1, 7], [0.2, 1.0], [[0, 0], [1, 1]], g=1.0, thermal=(1, 1),
                                  T_wall=(1.0, 0.5)), "rb"),
    "2d_5x1_periodic": (lambda: _cfg(2, [5, 1], [1.0, 0.2], [[0, 0], [0, 0]]), "white"),
    "2d_3x2_outflow": (lambda: _cfg(2, [3, 2], [1.0, 1.0], [[2, 2], [2, 2]], lm=0), "white"),
    "3d_1x1x9_column": (lambda: _cfg(3, [1, 1, 9], [0.1, 0.1, 1.0], [[0, 0], [0, 0], [1, 1]], g=1.0,
                                     thermal=(1, 1), T_wall=(1.0, 0.5)), "rb"),
    "3d_2x3x1_walls": (lambda: _cfg(3, [2, 3, 1], [1.0, 1.0, 0.2], [[0, 0], [0, 0], [1, 1]], g=1.0,
                                    thermal=(1, 0), T_wall=(1.0, 0.5)), "rb"),
    "3d_33x1x4_mixed": (lambda: _cfg(3, [33, 1, 4], [1.0, 0.1, 0.3], [[2, 2], [0, 0], [1, 1]], g=1.0,
                                     thermal=(0, 0)), "rb"),
}


@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_shapes(A, name):
    """Grids one cell wide or tall, narrower than the tile halo, or a single
    plane between two walls: 15 GPU steps against the oracle, and the
    fused kernel against the phase-by-phase reference kernels."""
    import torch
    make, kind = DEGENERATE[name]
    cfg = make()
    if kind == "rb":
        U0 = O.init(cfg, W.PROB_RB, [cfg["T_wall"][0], cfg["T_wall"][1], -1.0, 1e-2], 5)
        rng = np.random.default_rng(3)
        D = cfg["dim"]
        for k in range(D):
            U0[1 + k] = 1e-2 * rng.standard_normal(U0[0].shape) * U0[0]
        U0[-1] += 0.5 * sum(U0[1 + k] ** 2 for k in range(D)) / U0[0]
    else:
        U0 = I.white_random(cfg, seed=4)
    say("degenerate", name, cfg["n"])
    U, log, t, rc, fc = gpu_run(A, cfg, U0, 15, zchunk=1)
    assert rc == 0, fc
    r = O.run(cfg, U0, 15)
    assert r["status"] == 0
    err = close(cfg, U, r["U"])
    say(name, "max rel err", err, "bitwise", bitwise(U, r["U"]))
    assert err <= 1e-12
    S = A.Solver(cfg)
    S.set_state(U0)
    S.step_ref(torch.tensor(log, dtype=torch.float64))
    torch.cuda.synchronize()
    assert bitwise(S.numpy(), U)


NC_CASES = {
    "nc_rb2d_ragged": (lambda: W.rb([100, 37], [2.0, 1.0], Ra=3e3, seed=11, amp=1e-2), 60, 7),
    "nc_rb2d_thetaoff": (lambda: W.rb([64, 32], [2.0, 1.0], Ra=1e4, seed=1, amp=1e-2, low_mach=0), 60, None),
    "nc_rb3d_ragged": (lambda: W.rb([37, 29, 23], [1.3, 1.0, 1.0], Ra=1e5, seed=4, amp=1e-2), 25, 6),
    "nc_rb3d_thetaoff": (lambda: W.rb([20, 16, 12], [1.0, 1.0, 1.0], Ra=1e5, seed=2, amp=1e-2, low_mach=0), 25, None),
}


@pytest.mark.parametrize("name", list(NC_CASES))
def test_nonconservative_energy_vs_oracle(A, name):
    """The non-conservative energy scheme (App. B) on the GPU against the
    oracle, with a flow added to the RB state, and fused == reference
    kernels."""
    import torch
    make, nsteps, zc = NC_CASES[name]
    cfg, prob, prm, seed = make()
    cfg = dict(cfg, energy_form=1)
    Uo0 = O.init(cfg, prob, prm, seed)
    rng = np.random.default_rng(7)
    D = cfg["dim"]
    for k in range(D):
        Uo0[1 + k] = 1e-2 * rng.standard_normal(Uo0[0].shape) * Uo0[0]
    Uo0[-1] += 0.5 * sum(Uo0[1 + k] ** 2 for k in range(D)) / Uo0[0]
    U, log, t, rc, fc = gpu_run(A, cfg, Uo0, nsteps, zc)
    assert rc == 0, fc
    r = O.run(cfg, Uo0, nsteps)
    err = close(cfg, U, r["U"])
    say(name, "max rel err", err, "bitwise", bitwise(U, r["U"]))
    assert err <= 1e-12
    S = A.Solver(cfg)
    S.set_state(Uo0)
    S.step_ref(torch.tensor(log, dtype=torch.float64))
    torch.cuda.synchronize()
    assert bitwise(S.numpy(), U)


def test_step_graph_replay(A):
    """Steps recorded in a graph and replayed equal eager steps bit for bit:
    three replays of a 10-step graph (2D, even count) and of a 7-step graph
    (3D, odd count: the copy back is a node of the graph), each replay
    compared with an eager solver after eager work and synchronisation."""
    import torch
    for make, n in ((W.rb2d_64x32, 10), (lambda: W.rb([20, 12, 10], [1.0, 1.0, 1.0], Ra=1e5, seed=3), 7)):
        cfg, prob, prm, seed = make()
        G = A.Solver(cfg).init(prob, prm, seed)
        E = A.Solver(cfg).init(prob, prm, seed)
        torch.cuda.synchronize()
        say("graph capture", cfg["n"], n)
        g = G.capture(n)
        for r in range(3):
            g.replay()
            torch.cuda.synchronize()
            E.step(n)
            torch.cuda.synchronize()
            say("graph replay", cfg["n"], n, r)
            assert bitwise(G.numpy(), E.numpy())
            assert G.t.item() == E.t.item() and G.dt.item() == E.dt.item()
