"""GPU adjoint step against the oracle (run on an MI355X).

(i)  parity with the oracle's brute-force reverse product (columns of the
     Jacobian from its dual-number tangent-linear step) on small grids:
     lam^n and the mu/kappa derivatives, tolerance 1e-10 relative to the
     largest entry (the two sides sum the chain-rule terms in different
     orders);
(ii) central differences of the GPU forward step at the same frozen dt on a
     larger grid, for seeded directions: <lam^{n+1}, (F(U+h d) - F(U-h d))/2h>
     against <lam^n, d>, tolerance 1e-6 relative.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_09043_amd import workloads as W
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


def perturbed(cfg, prob, prm, seed, amp_u=1e-2):
    U = O.init(cfg, prob, prm, seed)
    rng = np.random.default_rng(seed + 17)
    D = cfg["dim"]
    for k in range(D):
        U[1 + k] = amp_u * rng.standard_normal(U[0].shape) * U[0]
    U[-1] += 0.5 * sum(U[1 + k] ** 2 for k in range(D)) / U[0]
    return U


def gpu_adjoint(A, cfg, U, lam, dt):
    import torch
    S = A.Solver(cfg)
    # poison the workspace: every field the reverse sweep reads must have
    # been written by it in this call (NaN bytes otherwise propagate)
    S.adjoint_workspace().fill_(0xFF)
    Ud = torch.as_tensor(U).cuda()
    ld = torch.as_tensor(lam).cuda()
    pg = torch.zeros(2, dtype=torch.float64, device="cuda")
    out = S.step_adjoint(Ud, ld, torch.tensor([dt], dtype=torch.float64), param_grad=pg)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pg.cpu().numpy()


# the *_bulk cases are wide enough in every direction to hold cells two or
# more cells from every boundary, whose reverse is folded in place
CASES = ["rb2d_walls", "rb2d_thetaoff_freeslip", "rb3d_walls", "periodic2d_inviscid", "outflow2d_viscous",
         "periodic3d_viscous", "rb3d_walls_bulk", "periodic3d_bulk",
         # the non-conservative energy form of App. B (gravity on: with g = 0
         # it coincides with the other form)
         "nc_rb2d_walls", "nc_rb2d_thetaoff_freeslip", "nc_rb3d_walls", "nc_rb3d_walls_bulk", "nc_rb2d_outflow_x"]


def make_case(name):
    if name.startswith("nc_"):
        cfg, U = make_case(name[3:])
        return dict(cfg, energy_form=1), U
    if name == "rb2d_outflow_x":
        # gravity needs walls along its axis; the lateral sides are outflow
        cfg, U = make_case("rb2d_walls")
        return dict(cfg, bc=[[2, 2], cfg["bc"][1]]), U
    if name == "rb2d_walls":
        cfg, prob, prm, seed = W.rb([10, 8], [2.0, 1.0], Ra=2e3, seed=3, amp=1e-3)
        return cfg, perturbed(cfg, prob, prm, seed)
    if name == "rb2d_thetaoff_freeslip":
        cfg, prob, prm, seed = W.rb([9, 7], [2.0, 1.0], Ra=1e3, seed=4, amp=1e-3, low_mach=0)
        cfg = dict(cfg, wall_noslip=0, thermal=[1, 0])
        return cfg, perturbed(cfg, prob, prm, seed)
    if name == "rb3d_walls":
        cfg, prob, prm, seed = W.rb([5, 4, 6], [1.0, 1.0, 1.0], Ra=1e4, seed=5, amp=1e-3)
        return cfg, perturbed(cfg, prob, prm, seed)
    if name == "rb3d_walls_bulk":
        cfg, prob, prm, seed = W.rb([6, 5, 7], [1.0, 1.0, 1.0], Ra=1e4, seed=9, amp=1e-3)
        return cfg, perturbed(cfg, prob, prm, seed)
    base = dict(gamma=5.0 / 3.0, g=0.0, K=1.1, cfl=0.4, dt_mode=0, wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])
    if name == "periodic3d_bulk":
        cfg = dict(base, dim=3, n=[7, 6, 5], L=[1.0, 1.0, 1.0], mu=3e-3, kappa=4e-3, low_mach=1,
                   bc=[[0, 0], [0, 0], [0, 0]])
        return cfg, I.white_random(cfg, seed=10, amp=0.2)
    if name == "periodic2d_inviscid":
        cfg = dict(base, dim=2, n=[8, 7], L=[1.0, 1.0], mu=0.0, kappa=0.0, low_mach=1, bc=[[0, 0], [0, 0]])
        return cfg, I.white_random(cfg, seed=6, amp=0.2)
    if name == "outflow2d_viscous":
        cfg = dict(base, dim=2, n=[9, 6], L=[1.0, 1.0], mu=3e-3, kappa=4e-3, low_mach=1, bc=[[2, 2], [2, 2]])
        return cfg, I.white_random(cfg, seed=7, amp=0.2)
    if name == "periodic3d_viscous":
        cfg = dict(base, dim=3, n=[5, 4, 4], L=[1.0, 1.0, 1.0], mu=3e-3, kappa=4e-3, low_mach=1,
                   bc=[[0, 0], [0, 0], [0, 0]])
        return cfg, I.white_random(cfg, seed=8, amp=0.2)
    raise KeyError(name)


@pytest.mark.parametrize("name", CASES)
def test_adjoint_vs_oracle_dense(A, name):
    cfg, U = make_case(name)
    dt = O.dt(cfg, U)
    rng = np.random.default_rng(11)
    lam = rng.standard_normal(U.shape)
    say(name, "gpu adjoint", cfg["n"])
    g, pg = gpu_adjoint(A, cfg, U, lam, dt)
    say(name, "oracle dense adjoint")
    o, gmu, gk = O.adjoint_dense(cfg, U, lam, dt)
    scale = np.abs(o).max()
    err = np.abs(g - o).max() / scale
    say(name, "lam rel err", err, "mu", pg[0], gmu, "kappa", pg[1], gk)
    assert err <= 1e-10
    if cfg["mu"] > 0 or cfg["kappa"] > 0:
        assert abs(pg[0] - gmu) <= 1e-10 * max(abs(gmu), scale)
        assert abs(pg[1] - gk) <= 1e-10 * max(abs(gk), scale)


@pytest.mark.parametrize("energy_form", [0, 1])
def test_adjoint_vs_central_differences(A, energy_form):
    """3D RB 24x20x16 with walls: the adjoint against central differences of
    the GPU forward step at frozen dt, 10 seeded directions and the two
    transport coefficients, in both energy forms.  The step is piecewise
    smooth (upwind switch, |u*|, min/max): h = 1e-8 of each field's scale
    and a 10 % velocity field keep faces away from those switches while
    rounding stays ~1e-8."""
    import torch
    cfg, prob, prm, seed = W.rb([24, 20, 16], [1.0, 1.0, 1.0], Ra=1e5, seed=9, amp=1e-3)
    cfg = dict(cfg, energy_form=energy_form)
    U = perturbed(cfg, prob, prm, seed, amp_u=1e-1)
    dt = O.dt(cfg, U)
    rng = np.random.default_rng(12)
    lam = rng.standard_normal(U.shape)
    g, pg = gpu_adjoint(A, cfg, U, lam, dt)
    sched = torch.tensor([dt], dtype=torch.float64, device="cuda")

    def fwd(c, X):
        S = A.Solver(c)
        S.U.copy_(torch.as_tensor(X).cuda())
        S.step_sched(sched)
        torch.cuda.synchronize()
        return S.numpy()

    scale = np.abs(U).reshape(U.shape[0], -1).max(axis=1)[:, None, None, None]
    for k in range(10):
        d = rng.standard_normal(U.shape) * scale
        h = 1e-8
        fd = np.sum(lam * (fwd(cfg, U + h * d) - fwd(cfg, U - h * d))) / (2 * h)
        ad = np.sum(g * d)
        say("direction", k, "fd", fd, "adjoint", ad)
        assert abs(fd - ad) <= 1e-6 * max(abs(fd), abs(ad))
    for which, idx in (("mu", 0), ("kappa", 1)):
        hp = 0.1 * cfg[which]
        fd = np.sum(lam * (fwd(dict(cfg, **{which: cfg[which] + hp}), U) -
                           fwd(dict(cfg, **{which: cfg[which] - hp}), U))) / (2 * hp)
        say(which, "fd", fd, "adjoint", pg[idx])
        assert abs(fd - pg[idx]) <= 1e-7 * max(abs(fd), 1e-30)
