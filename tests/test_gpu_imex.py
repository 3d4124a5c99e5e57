"""GPU implicit acoustic (IMEX) step against the oracle (run on an MI355X).

The oracle solves the implicit system for (Pi, u) with a direct sparse
solver, the GPU the eliminated system for Pi to a relative residual of
1e-13 (conjugate gradients when every axis is periodic or walled, as in
every case here but the outflow one, BiCGSTAB otherwise); the states are compared with the scale-aware 1e-12 measure of
tests/parity.py.  Without the low-Mach correction the acoustic
dissipation (taken at t^n) limits the step to about the acoustic one, so
those cases run at 0.8 times the explicit step.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_09043_amd import workloads as W
from tests import parity as PA

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


def _flow(cfg, U, amp=1e-2, seed=7):
    rng = np.random.default_rng(seed)
    D = cfg["dim"]
    U = U.copy()
    for k in range(D):
        U[1 + k] = amp * rng.standard_normal(U[0].shape) * U[0]
    U[-1] += 0.5 * sum(U[1 + k] ** 2 for k in range(D)) / U[0]
    return U


def _outflow_cfg():
    return dict(dim=2, n=[24, 10], L=[1.0, 0.5], gamma=1.4, g=0.0, mu=1e-3, kappa=1e-3, K=1.1, cfl=0.4, low_mach=1,
                dt_mode=0, bc=[[2, 2], [0, 0]], wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])


CASES = {
    # name: (setup, flow amplitude, dt multiple of the explicit CFL step, steps)
    "rb2d_walls": (lambda: W.rb([24, 12], [2.0, 1.0], Ra=1e4, seed=3, amp=1e-2), 1e-2, 4.0, 4),
    "rb2d_thetaoff": (lambda: W.rb([20, 10], [2.0, 1.0], Ra=1e4, seed=1, amp=1e-2, low_mach=0), 1e-2, 0.8, 4),
    # two ragged x tiles and three ragged z tiles of the 2D LDS product, walls at both ends
    "rb2d_walls_ragged_tiles": (lambda: W.rb([70, 37], [2.0, 1.0], Ra=1e4, seed=4, amp=1e-2), 1e-2, 4.0, 3),
    "rb3d_walls": (lambda: W.rb([9, 7, 8], [1.0, 1.0, 1.0], Ra=1e5, seed=2, amp=1e-2), 1e-2, 3.0, 3),
    "gresho_on": (lambda: W.gresho(n=32, Ma=1e-2, low_mach=1), 0.0, 8.0, 4),
    "gresho_off": (lambda: W.gresho(n=24, Ma=1e-2, low_mach=0), 0.0, 0.8, 4),
    "gresho_ma1e-3": (lambda: W.gresho(n=40, Ma=1e-3, low_mach=1), 0.0, 50.0, 3),
}


@pytest.mark.parametrize("name", list(CASES))
def test_imex_vs_oracle(A, name):
    import torch
    make, amp, mult, nst = CASES[name]
    cfg, prob, prm, seed = make()
    U0 = O.init(cfg, prob, prm, seed)
    if amp:
        U0 = _flow(cfg, U0, amp)
    dt = O.dt(cfg, U0) * mult
    say(name, cfg["n"], "dt x", mult)
    S = A.Solver(cfg)
    S.set_state(U0)
    its = S.step_imex([dt] * nst)
    torch.cuda.synchronize()
    assert S.fault()[0] == 0
    r = O.run_imex(cfg, U0, nst, dt)
    assert r["status"] == 0
    err = PA.rel_err(cfg, S.numpy(), r["U"])
    say(name, "iterations", its, "parity", err, "(each variable on its own max: %.3e)" % PA.strict_err(S.numpy(), r["U"]))
    assert err <= 1e-12
    assert abs(S.t.item() - nst * dt) <= 1e-14 * nst * dt


def test_imex_outflow_viscous_vs_oracle(A):
    import torch
    cfg = _outflow_cfg()
    from tests import inputs as I
    U0 = I.smooth_random(cfg, seed=5)
    dt = O.dt(cfg, U0) * 2.0
    S = A.Solver(cfg)
    S.set_state(U0)
    its = S.step_imex([dt] * 3)
    torch.cuda.synchronize()
    r = O.run_imex(cfg, U0, 3, dt)
    err = PA.rel_err(cfg, S.numpy(), r["U"])
    say("outflow viscous iterations", its, "parity", err)
    assert err <= 1e-12


def _periodic_cfg(n, lm=1, mu=2e-3):
    return dict(dim=len(n), n=list(n), L=[1.0, 0.8, 0.9][:len(n)], gamma=1.4, g=0.0, mu=mu, kappa=1.5 * mu, K=1.1,
                cfl=0.4, low_mach=lm, dt_mode=0, bc=[[0, 0]] * len(n), wall_noslip=1, thermal=[0, 0],
                T_wall=[1.0, 1.0])


@pytest.mark.parametrize("name,n,lm,mult", [("periodic3d", (10, 7, 9), 1, 4.0),
                                             ("periodic3d_thetaoff", (6, 9, 7), 0, 0.8),
                                             ("periodic2d_ragged", (37, 29), 1, 8.0),
                                             ("periodic2d_below_stencil", (3, 4), 1, 4.0)])
def test_imex_periodic_cg_vs_oracle(A, name, n, lm, mult):
    """Every side periodic (the conjugate-gradient path, whose operator is a
    periodic star stencil of radius 2): a 3D box, odd sizes that leave
    ragged reduction blocks, and sides of 3 and 4 cells where the stencil
    wraps onto itself."""
    import torch
    from tests import inputs as I
    cfg = _periodic_cfg(n, lm)
    U0 = I.smooth_random(cfg, seed=11)
    dt = O.dt(cfg, U0) * mult
    say(name, cfg["n"], "dt x", mult)
    S = A.Solver(cfg)
    S.set_state(U0)
    its = S.step_imex([dt] * 3)
    torch.cuda.synchronize()
    assert S.fault()[0] == 0
    r = O.run_imex(cfg, U0, 3, dt)
    assert r["status"] == 0
    err = PA.rel_err(cfg, S.numpy(), r["U"])
    say(name, "iterations", its, "parity", err)
    assert err <= 1e-12


@pytest.mark.parametrize("lm,mult", [(1, 100.0), (0, 0.8)])
def test_imex_well_balanced_gpu(A, lm, mult):
    """Isothermal column and inviscid RB base at 100 times the explicit
    step (0.8 without the low-Mach correction): at rest to round-off after
    5 steps on the GPU."""
    import torch
    cfg = dict(dim=2, n=[4, 128], L=[1.0, 3.0], gamma=5.0 / 3.0, g=1.0, mu=0.0, kappa=0.0, K=1.1, cfl=0.4,
               low_mach=lm, dt_mode=0, bc=[[0, 0], [1, 1]], wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])
    S = A.Solver(cfg).init(W.PROB_ISOTHERMAL)
    dt = S.dt.item() * mult
    S.step_imex([dt] * 5)
    torch.cuda.synchronize()
    U = S.numpy()
    say("iso lm", lm, "max|u|", np.max(np.abs(U[1:3] / U[0])))
    assert np.max(np.abs(U[1:3] / U[0])) < 1e-12
    cfg, prob, prm, seed = W.rb([32, 16, 12], [2.0, 1.0, 1.0], Ra=1e5, seed=1, amp=0.0, low_mach=lm)
    cfg = dict(cfg, mu=0.0, kappa=0.0)
    S = A.Solver(cfg).init(prob, prm, seed)
    dt = S.dt.item() * mult
    S.step_imex([dt] * 5)
    torch.cuda.synchronize()
    U = S.numpy()
    say("rb3d base lm", lm, "max|u|", np.max(np.abs(U[1:4] / U[0])))
    assert np.max(np.abs(U[1:4] / U[0])) < 1e-12


def test_imex_unsupported_and_invalid(A):
    """App. B energy form is refused; bad arguments are refused."""
    import torch
    cfg, prob, prm, seed = W.rb([16, 8], [2.0, 1.0], Ra=1e4)
    S = A.Solver(dict(cfg, energy_form=1)).init(prob, prm, seed)
    with pytest.raises(A.ArsError):
        S.step_imex([1e-3])
    S2 = A.Solver(cfg).init(prob, prm, seed)
    with pytest.raises(A.ArsError):
        S2.step_imex([1e-3], tol=0.0)
    torch.cuda.synchronize()
