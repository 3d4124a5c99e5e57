"""Fused adjoint marches (3D, periodic lateral sides) on an MI355X.

(i)   against the oracle's brute-force reverse product on small grids that
      take the fused path (tolerance 1e-10 of the largest entry, as for the
      reference path in tests/test_gpu_adjoint.py);
(ii)  against the reference phase-kernel path on grids of several ragged
      tiles and vertical chunks, and at the adjoint workload's full size
      (3D RB 128^3): the two sum the same chain-rule terms in different
      orders, so they agree to rounding (1e-12 of the largest entry);
(iii) repeatability: two calls give the same bits.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_09043_amd import workloads as W
from tests.test_gpu_adjoint import perturbed, gpu_adjoint
from tests import inputs as I

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


def fused_taken(A, cfg):
    """The fused path needs 17 doubles per cell (plus the partial sums)."""
    ctx = A.Context(cfg)
    ncell = int(np.prod(cfg["n"]))
    return A.lib().ars_workspace_bytes_adjoint(ctx.h) == 17 * 8 * ncell + 2 * 1024 * 8


def small_case(name):
    base = dict(gamma=5.0 / 3.0, K=1.1, cfl=0.4, dt_mode=0, wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])
    if name == "rb3d_walls_7x6x6":
        cfg, prob, prm, seed = W.rb([7, 6, 6], [1.0, 1.0, 1.0], Ra=1e4, seed=21, amp=1e-3)
        return cfg, perturbed(cfg, prob, prm, seed)
    if name == "rb3d_thetaoff_freeslip_adiabatic_top":
        cfg, prob, prm, seed = W.rb([6, 7, 5], [1.0, 1.0, 1.0], Ra=1e4, seed=22, amp=1e-3, low_mach=0)
        cfg = dict(cfg, wall_noslip=0, thermal=[1, 0])
        return cfg, perturbed(cfg, prob, prm, seed)
    if name == "rb3d_inviscid":
        cfg, prob, prm, seed = W.rb([6, 5, 6], [1.0, 1.0, 1.0], Ra=1e4, seed=23, amp=1e-3)
        cfg = dict(cfg, mu=0.0, kappa=0.0)
        return cfg, perturbed(cfg, prob, prm, seed)
    if name == "rb3d_strong_flow":
        cfg, prob, prm, seed = W.rb([5, 6, 7], [1.0, 1.0, 1.0], Ra=1e4, seed=24, amp=1e-3)
        return cfg, perturbed(cfg, prob, prm, seed, amp_u=0.3)
    if name == "periodic3d_g0_thetaoff":
        cfg = dict(base, dim=3, n=[6, 5, 6], L=[1.0, 1.0, 1.0], g=0.0, mu=3e-3, kappa=4e-3, low_mach=0,
                   bc=[[0, 0], [0, 0], [0, 0]])
        return cfg, I.white_random(cfg, seed=25, amp=0.2)
    raise KeyError(name)


SMALL = ["rb3d_walls_7x6x6", "rb3d_thetaoff_freeslip_adiabatic_top", "rb3d_inviscid", "rb3d_strong_flow",
         "periodic3d_g0_thetaoff"]


@pytest.mark.parametrize("name", SMALL)
def test_fused_adjoint_vs_oracle_dense(A, name):
    cfg, U = small_case(name)
    assert fused_taken(A, cfg)
    dt = O.dt(cfg, U)
    rng = np.random.default_rng(31)
    lam = rng.standard_normal(U.shape)
    say(name, "fused adjoint", cfg["n"])
    g, pg = gpu_adjoint(A, cfg, U, lam, dt)
    o, gmu, gk = O.adjoint_dense(cfg, U, lam, dt)
    scale = np.abs(o).max()
    err = np.abs(g - o).max() / scale
    say(name, "lam rel err", err, "mu", pg[0], gmu, "kappa", pg[1], gk)
    assert err <= 1e-10
    if cfg["mu"] > 0 or cfg["kappa"] > 0:
        assert abs(pg[0] - gmu) <= 1e-10 * max(abs(gmu), scale)
        assert abs(pg[1] - gk) <= 1e-10 * max(abs(gk), scale)


def _fused_vs_ref(A, cfg, U, dt, seed):
    import torch
    S = A.Solver(cfg)
    Ud = torch.as_tensor(U).cuda()
    rng = np.random.default_rng(seed)
    ld = torch.as_tensor(rng.standard_normal(U.shape)).cuda()
    dtt = torch.tensor([dt], dtype=torch.float64)
    out = {}
    for ref in (False, True):
        S.adjoint_workspace(ref).fill_(0xFF)
        pg = torch.zeros(2, dtype=torch.float64, device="cuda")
        lam = S.step_adjoint(Ud, ld, dtt, param_grad=pg, ref=ref)
        torch.cuda.synchronize()
        out[ref] = (lam.cpu().numpy(), pg.cpu().numpy())
    f, r = out[False], out[True]
    scale = np.abs(r[0]).max()
    err = np.abs(f[0] - r[0]).max() / scale
    return err, f, r, scale


@pytest.mark.parametrize("case", ["walls_lm", "walls_thetaoff_freeslip", "periodic_g0", "walls_inviscid"])
def test_fused_adjoint_vs_reference_ragged_tiles(A, case):
    """Grids of several ragged tiles in x and y (tiles of 20 x 12 and 30 x 14
    outputs) and several vertical shares per tile."""
    if case == "periodic_g0":
        cfg = dict(dim=3, n=[45, 29, 23], L=[1.5, 1.0, 0.8], gamma=1.4, g=0.0, mu=2e-3, kappa=3e-3, K=1.1, cfl=0.4,
                   low_mach=1, dt_mode=0, bc=[[0, 0], [0, 0], [0, 0]], wall_noslip=1, thermal=[0, 0],
                   T_wall=[1.0, 1.0])
        U = I.white_random(cfg, seed=41, amp=0.2)
    else:
        lm = 0 if case == "walls_thetaoff_freeslip" else 1
        cfg, prob, prm, seed = W.rb([45, 29, 23], [2.0, 1.3, 1.0], Ra=1e5, seed=42, amp=1e-3, low_mach=lm)
        if case == "walls_thetaoff_freeslip":
            cfg = dict(cfg, wall_noslip=0, thermal=[1, 0])
        if case == "walls_inviscid":
            cfg = dict(cfg, mu=0.0, kappa=0.0)
        U = perturbed(cfg, prob, prm, seed, amp_u=0.05)
    assert fused_taken(A, cfg)
    dt = O.dt(cfg, U)
    err, f, r, scale = _fused_vs_ref(A, cfg, U, dt, 43)
    say(case, cfg["n"], "fused vs reference", err, "mu", f[1][0], r[1][0], "kappa", f[1][1], r[1][1])
    assert err <= 1e-12
    if cfg["mu"] > 0:
        assert abs(f[1][0] - r[1][0]) <= 1e-12 * max(abs(r[1][0]), 1e-300)
        assert abs(f[1][1] - r[1][1]) <= 1e-12 * max(abs(r[1][1]), 1e-300)


def test_fused_adjoint_full_size_and_repeatable(A):
    """3D RB 128^3 (the adjoint workload): fused = reference to rounding,
    and two fused calls give the same bits."""
    import torch
    cfg, prob, prm, seed = W.rb3d_ra1e5()
    assert fused_taken(A, cfg)
    S = A.Solver(cfg).init(prob, prm, seed)
    S.step(50)
    torch.cuda.synchronize()
    U = S.numpy()
    dt = float(S.dt.item())
    err, f, r, scale = _fused_vs_ref(A, cfg, U, dt, 44)
    say("128^3 fused vs reference", err, "mu", f[1][0], r[1][0], "kappa", f[1][1], r[1][1])
    assert err <= 1e-12
    assert abs(f[1][0] - r[1][0]) <= 1e-12 * abs(r[1][0])
    assert abs(f[1][1] - r[1][1]) <= 1e-12 * abs(r[1][1])
    err2, f2, _, _ = _fused_vs_ref(A, cfg, U, dt, 44)
    assert np.array_equal(f[0], f2[0]) and np.array_equal(f[1], f2[1])
