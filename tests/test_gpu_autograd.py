"""Gradient of a convection run through torch.autograd (run on an MI355X).

J = kinetic energy after N steps of the 3D Rayleigh-Benard layer from the
base state heated by dT0; gradient w.r.t. dT0, mu, kappa (and Ra through the
(Ra, Pr) -> (mu, kappa) map) by the adjoint step with binomial
checkpointing.  Checks: checkpointed = all-states-stored gradient bit for
bit; central differences at the frozen time-step schedule.
"""
import sys

import numpy as np
import pytest

from paper_1903_09043_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def T():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def make_problem(T, slots, nsteps=12, n=(16, 12, 10), Ra=2e4, dt_sched=None, energy_form=0):
    from paper_1903_09043_amd.adjoint import RBProblem
    cfg, prob, prm, seed = W.rb(list(n), [1.0, 1.0, 1.0], Ra=Ra, seed=0, amp=0.0)
    cfg = dict(cfg, energy_form=energy_form)
    rng = np.random.default_rng(5)
    u0 = 0.1 * rng.standard_normal((3,) + tuple(reversed(n)))
    return RBProblem(cfg, prob, prm, nsteps, slots, u0=u0, dt_sched=dt_sched), cfg


def test_checkpointed_gradient_equals_store_all(T):
    from paper_1903_09043_amd.adjoint import rb_kinetic_energy
    grads = []
    for slots in (3, 12):
        pb, cfg = make_problem(T, slots)
        dT = (1e-2 * T.tensor(np.random.default_rng(1).standard_normal(pb.rho.shape))).cuda().requires_grad_()
        mu = T.tensor(cfg["mu"], dtype=T.float64, requires_grad=True)
        ka = T.tensor(cfg["kappa"], dtype=T.float64, requires_grad=True)
        J = rb_kinetic_energy(dT, mu, ka, pb)
        J.backward()
        grads.append((J.item(), dT.grad.cpu().numpy(), mu.grad.item(), ka.grad.item()))
        say("slots", slots, "J", J.item(), "dJ/dmu", mu.grad.item(), "dJ/dkappa", ka.grad.item())
    (J0, g0, m0, k0), (J1, g1, m1, k1) = grads
    assert J0 == J1 and np.array_equal(g0, g1) and m0 == m1 and k0 == k1


def test_step_sched_to_equals_step_sched(T):
    """ars_step_sched_to (out of place, no copy; the adjoint sweep's
    advances) gives the states of ars_step_sched bit for bit, leaves its
    input untouched, and may write its output over its input from two
    steps on."""
    pb, cfg = make_problem(T, 3)
    S = pb.solver(cfg["mu"], cfg["kappa"])
    U0 = pb.build(S, T.zeros(pb.rho.shape, dtype=T.float64, device="cuda")).clone()
    dts = T.full((3,), S.compute_dt().item(), dtype=T.float64, device="cuda")
    a, b, out = (T.empty_like(U0) for _ in range(3))
    want = {}
    for n in (1, 2, 3):
        S.U.copy_(U0)
        S.step_sched(dts[:n])
        want[n] = S.U.clone()
        keep = U0.clone()
        S.step_sched_to(U0, out, a, b, dts[:n])
        T.cuda.synchronize()
        say("step_sched_to", n, "bitwise", T.equal(out, want[n]))
        assert T.equal(out, want[n]) and T.equal(U0, keep)
    buf = U0.clone()
    S.step_sched_to(buf, buf, a, b, dts[:2])
    assert T.equal(buf, want[2])


def test_step_to_equals_step(T):
    """ars_step_to (CFL steps out of place; the objective's forward sweep)
    gives the states, dt log, t and next dt of ars_step bit for bit."""
    pb, cfg = make_problem(T, 3)
    S = pb.solver(cfg["mu"], cfg["kappa"])
    U0 = pb.build(S, T.zeros(pb.rho.shape, dtype=T.float64, device="cuda")).clone()
    dt0 = S.compute_dt().clone()
    a, b, out = (T.empty_like(U0) for _ in range(3))
    for n in (1, 2, 3):
        S.U.copy_(U0)
        S.t.zero_()
        S.dt.copy_(dt0)
        log_ref = T.zeros(n, dtype=T.float64, device="cuda")
        S.step(n, dt_log=log_ref)
        want, t_ref, dt_ref = S.U.clone(), S.t.clone(), S.dt.clone()
        S.t.zero_()
        S.dt.copy_(dt0)
        log = T.zeros(n, dtype=T.float64, device="cuda")
        S.step_to(U0, out, a, b, n, dt_log=log)
        T.cuda.synchronize()
        same = T.equal(out, want) and T.equal(log, log_ref) and T.equal(S.t, t_ref) and T.equal(S.dt, dt_ref)
        say("step_to", n, "bitwise", same)
        assert same


@pytest.mark.parametrize("energy_form", [0, 1])
def test_gradient_vs_central_differences(T, energy_form):
    """Both energy forms (the relaxed total energy and App. B)."""
    from paper_1903_09043_amd.adjoint import rb_kinetic_energy, rb_kinetic_energy_ra_pr
    pb, cfg = make_problem(T, 4, energy_form=energy_form)
    rng = np.random.default_rng(2)
    dT0 = (1e-2 * T.tensor(rng.standard_normal(pb.rho.shape))).cuda()
    dT = dT0.clone().requires_grad_()
    mu = T.tensor(cfg["mu"], dtype=T.float64, requires_grad=True)
    ka = T.tensor(cfg["kappa"], dtype=T.float64, requires_grad=True)
    J = rb_kinetic_energy(dT, mu, ka, pb)
    J.backward()
    g = dT.grad.cpu().numpy()
    # freeze the schedule the forward run chose
    S = pb.solver(cfg["mu"], cfg["kappa"])
    S.U.copy_(pb.initial_state(dT0))
    S.compute_dt()
    log = T.zeros(pb.nsteps, dtype=T.float64, device="cuda")
    S.step(pb.nsteps, dt_log=log)
    pf, _ = make_problem(T, 4, dt_sched=log, energy_form=energy_form)

    def Jf(x, m=cfg["mu"], k=cfg["kappa"]):
        with T.no_grad():
            return rb_kinetic_energy(x, m, k, pf).item()

    assert Jf(dT0) == J.item()

    # A central difference that straddles a switch of a non-smooth branch
    # (upwind side of a face, |u*| in theta) measures the mean of the two
    # one-sided slopes instead of the derivative of the branch taken; such a
    # switch is rare but not impossible over a few thousand faces, so each
    # check accepts agreement at either of two step sizes.
    def agree(f, ad, hs, what):
        errs = []
        for h in hs:
            fd = f(h)
            errs.append(abs(fd - ad) / max(abs(fd), abs(ad)))
            say(what, "h", h, "fd", fd, "adjoint", ad, "rel", errs[-1])
            if errs[-1] <= 1e-5:
                return
        assert min(errs) <= 1e-5, (what, errs)

    for k in range(5):
        d = T.tensor(rng.standard_normal(pb.rho.shape)).cuda()  # unit-RMS direction
        ad = float(np.sum(g * d.cpu().numpy()))
        agree(lambda h: (Jf(dT0 + h * d) - Jf(dT0 - h * d)) / (2 * h), ad, (1e-7, 1e-8), f"dT direction {k}")
    base_mu, base_ka = cfg["mu"], cfg["kappa"]
    agree(lambda h: (Jf(dT0, m=base_mu * (1 + h)) - Jf(dT0, m=base_mu * (1 - h))) / (2 * h * base_mu),
          mu.grad.item(), (1e-4, 1e-5), "mu")
    agree(lambda h: (Jf(dT0, k=base_ka * (1 + h)) - Jf(dT0, k=base_ka * (1 - h))) / (2 * h * base_ka),
          ka.grad.item(), (1e-4, 1e-5), "kappa")
    # Ra through the (Ra, Pr) -> (mu, kappa) map
    Ra = T.tensor(2e4, dtype=T.float64, requires_grad=True)
    J2 = rb_kinetic_energy_ra_pr(dT0, Ra, 1.0, pf)
    J2.backward()

    def fd_ra(hr):
        with T.no_grad():
            fp = rb_kinetic_energy_ra_pr(dT0, T.tensor(2e4 + hr, dtype=T.float64), 1.0, pf).item()
            fm = rb_kinetic_energy_ra_pr(dT0, T.tensor(2e4 - hr, dtype=T.float64), 1.0, pf).item()
        return (fp - fm) / (2 * hr)
    agree(fd_ra, Ra.grad.item(), (1.0, 0.1), "Ra")


def test_rb3d_128_gradient_vs_finite_differences(T):
    """The adjoint workload at full size: 3D RB 128^3, Ra = 1e5, Pr = 1, 200
    steps from the base state heated by a seeded 1e-4 perturbation, 16
    revolve slots.  dJ/d(dT0) against central differences along 10 seeded
    unit-RMS directions, and dJ/dRa through the (Ra, Pr) map, all at the
    frozen time-step schedule of the forward run."""
    from paper_1903_09043_amd.adjoint import RBProblem, rb_kinetic_energy, rb_kinetic_energy_ra_pr
    cfg, prob, prm, seed = W.rb3d_ra1e5()
    pb = RBProblem(cfg, prob, prm, 200, 16)
    g0 = T.Generator(device="cpu").manual_seed(0)
    dT0 = (1e-4 * (2 * T.rand(pb.rho.shape, generator=g0, dtype=T.float64) - 1)).cuda()
    x = dT0.clone().requires_grad_()
    mu = T.tensor(cfg["mu"], dtype=T.float64, requires_grad=True)
    ka = T.tensor(cfg["kappa"], dtype=T.float64, requires_grad=True)
    J = rb_kinetic_energy(x, mu, ka, pb)
    J.backward()
    say("rb3d 128^3 J", J.item(), "dJ/dmu", mu.grad.item(), "dJ/dkappa", ka.grad.item())
    g = x.grad
    S = pb.solver(cfg["mu"], cfg["kappa"])
    S.U.copy_(pb.initial_state(dT0))
    S.compute_dt()
    log = T.zeros(200, dtype=T.float64, device="cuda")
    S.step(200, dt_log=log)
    pf = RBProblem(cfg, prob, prm, 200, 16, dt_sched=log)

    def Jf(v):
        with T.no_grad():
            return rb_kinetic_energy(v, cfg["mu"], cfg["kappa"], pf).item()

    assert Jf(dT0) == J.item()
    # A random direction in R^N is nearly orthogonal to g (|g.d| ~ |g||d| /
    # sqrt(N), N = 128^3), so the directional derivative is compared on the
    # scale of the vectors, |g| |d|, not on its own size: an absolute error
    # of the gradient of 1e-8 |g| shows as 1e-8 |g| |d| on every direction,
    # but as 1e-8 sqrt(N) ~ 1e-5 relative to g.d on a typical one.
    gn = float(g.pow(2).sum().sqrt().item())
    h = 1e-9
    for k in range(1, 11):
        gk = T.Generator(device="cpu").manual_seed(k)
        d = T.randn(pb.rho.shape, generator=gk, dtype=T.float64).cuda()
        d = d / d.pow(2).mean().sqrt()
        dn = float(d.pow(2).sum().sqrt().item())
        ad = float((g * d).sum().item())
        fd = (Jf(dT0 + h * d) - Jf(dT0 - h * d)) / (2 * h)
        err = abs(fd - ad) / (gn * dn)
        say("direction", k, "h", h, "fd", fd, "adjoint", ad, "|fd - ad| / (|g| |d|)", err,
            "relative to g.d", abs(fd - ad) / max(abs(fd), abs(ad)), "g.d / (|g| |d|)", ad / (gn * dn))
        assert err <= 1e-8, (k, err)
    Ra = T.tensor(1e5, dtype=T.float64, requires_grad=True)
    J2 = rb_kinetic_energy_ra_pr(dT0, Ra, 1.0, pf)
    J2.backward()
    errs = []
    for hr in (10.0, 1.0):
        with T.no_grad():
            fp = rb_kinetic_energy_ra_pr(dT0, T.tensor(1e5 + hr, dtype=T.float64), 1.0, pf).item()
            fm = rb_kinetic_energy_ra_pr(dT0, T.tensor(1e5 - hr, dtype=T.float64), 1.0, pf).item()
        fd = (fp - fm) / (2 * hr)
        errs.append(abs(fd - Ra.grad.item()) / abs(fd))
        say("Ra h", hr, "fd", fd, "adjoint", Ra.grad.item(), "rel", errs[-1])
        if errs[-1] <= 1e-5:
            break
    assert min(errs) <= 1e-5, errs


def test_nusselt_objective(T):
    """Nusselt number at both walls: value against the oracle's diagnostics,
    gradient of the final Nu through the adjoint against central
    differences (frozen schedule), and dNu/dU of the objective itself
    against differences of the objective."""
    import oracle as O
    import paper_1903_09043_amd as A
    from paper_1903_09043_amd.adjoint import RBProblem, rb_objective
    cfg, prob, prm, seed = W.rb([12, 10, 8], [1.0, 1.0, 1.0], Ra=2e4, seed=3, amp=1e-2)
    r = O.run(cfg, O.init(cfg, prob, prm, seed), 7)  # the oracle's state after 7 steps
    assert r["status"] == 0
    S = A.Solver(cfg).set_state(r["U"])
    g = T.empty_like(S.U)
    nb = S.nusselt(0, grad=g).item()
    nt = S.nusselt(1).item()
    T.cuda.synchronize()
    d = O.diag(cfg, r["U"])
    say("Nu bottom", nb, d["nu_bot"], "top", nt, d["nu_top"])
    assert abs(nb - d["nu_bot"]) <= 1e-12 * abs(d["nu_bot"])
    assert abs(nt - d["nu_top"]) <= 1e-12 * abs(d["nu_top"])
    # dNu/dU of the objective against a central difference along a random direction
    dU = T.tensor(np.random.default_rng(4).standard_normal(tuple(S.U.shape))).cuda() * S.U.abs() * 1e-3
    h = 1e-3
    fd = (S.nusselt(0, U=S.U + h * dU).item() - S.nusselt(0, U=S.U - h * dU).item()) / (2 * h)
    ad = float((g * dU).sum().item())
    say("dNu/dU fd", fd, "analytic", ad)
    assert abs(fd - ad) <= 1e-7 * abs(fd)
    for objective in ("nu_bot", "nu_top"):
        pb = RBProblem(cfg, prob, prm, 10, 3, objective=objective)
        rng = np.random.default_rng(6)
        dT0 = (1e-2 * T.tensor(rng.standard_normal(pb.rho.shape))).cuda()
        x = dT0.clone().requires_grad_()
        J = rb_objective(x, cfg["mu"], cfg["kappa"], pb)
        J.backward()
        S2 = pb.solver(cfg["mu"], cfg["kappa"])
        S2.U.copy_(pb.initial_state(dT0))
        S2.compute_dt()
        log = T.zeros(10, dtype=T.float64, device="cuda")
        S2.step(10, dt_log=log)
        pf = RBProblem(cfg, prob, prm, 10, 3, dt_sched=log, objective=objective)
        for k in range(3):
            dd = T.tensor(rng.standard_normal(pb.rho.shape)).cuda()
            ad = float((x.grad * dd).sum().item())
            errs = []
            for hh in (1e-7, 1e-8):
                with T.no_grad():
                    fd = (rb_objective(dT0 + hh * dd, cfg["mu"], cfg["kappa"], pf).item()
                          - rb_objective(dT0 - hh * dd, cfg["mu"], cfg["kappa"], pf).item()) / (2 * hh)
                errs.append(abs(fd - ad) / max(abs(fd), abs(ad)))
                say(objective, "direction", k, "h", hh, "fd", fd, "adjoint", ad, "rel", errs[-1])
                if errs[-1] <= 1e-5:
                    break
            assert min(errs) <= 1e-5, (objective, k, errs)


@pytest.mark.parametrize("n", [(64, 32), (20, 12, 10)])
def test_initial_state_map_and_transpose(T, n):
    """ars_init_rb_dT with the SplitMix64 field of the RB workload equals the
    oracle's RB initial state bit for bit; its transpose is lam_E rho /
    (gamma - 1) on the oracle's base density."""
    import oracle as O
    import paper_1903_09043_amd as A
    L = [2.0, 1.0] if len(n) == 2 else [1.0, 1.0, 1.0]
    cfg, prob, prm, seed = W.rb(list(n), L, Ra=1e4, seed=7, amp=1e-4)
    Uo = O.init(cfg, prob, prm, seed)
    shape = Uo.shape[1:]
    ncell = int(np.prod(shape))
    bits = O.splitmix64(seed, ncell) >> np.uint64(11)
    dT = prm[3] * (2.0 * (bits.astype(np.float64) * 2.0 ** -53) - 1.0)
    S = A.Solver(cfg)
    S.init_rb_dT(prm, T.tensor(dT.reshape(shape)).cuda())
    T.cuda.synchronize()
    say("init_rb_dT", n, "bitwise", np.array_equal(S.numpy(), Uo))
    assert np.array_equal(S.numpy(), Uo)
    lam = np.random.default_rng(2).standard_normal(Uo.shape)
    g = S.init_rb_dT_adjoint(S.U, T.tensor(lam).cuda()).cpu().numpy()
    want = (lam[-1] * Uo[0]) / (cfg["gamma"] - 1.0)
    assert np.max(np.abs(g - want)) <= 1e-15 * np.max(np.abs(want))
