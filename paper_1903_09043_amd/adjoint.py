"""Gradients of a convection run through the hand-written adjoint step.

``rb_kinetic_energy(dT0, mu, kappa, problem)`` is a ``torch.autograd.Function``:
its forward runs ``problem.nsteps`` explicit steps of the all-regime scheme
from the Rayleigh-Benard base state heated by the temperature perturbation
``dT0`` and returns the final kinetic energy (or, with
``RBProblem(objective="nu_bot" / "nu_top")`` and ``rb_objective``, the final
Nusselt number at the bottom / top wall); its backward returns
dJ/d(dT0), dJ/dmu and dJ/dkappa.  The time step of every step is the one the
forward run chose (the schedule is recorded and frozen: dt = CFL / max rate
is not differentiated).  Intermediate states are not all kept: the run
follows a binomial checkpointing plan (``ars_revolve_plan``) over
``problem.slots`` state snapshots.  The forward pass is the plan's forward
sweep (the snapshots written as the run goes), and the backward resumes the
plan at its first adjoint step, recomputing forward steps between
snapshots; no state is copied (out-of-place steps write each snapshot
directly, a restore only selects one).

Everything numerical runs in libars.so (forward steps, adjoint steps,
objective and its gradient); this module only sequences the calls.  Rayleigh
and Prandtl numbers enter through ``workloads.ra_pr_to_mu_kappa`` written in
torch operations, so autograd chains (Ra, Pr) -> (mu, kappa) -> J.
"""
import torch

from . import ArsError, Solver, revolve_plan, workloads

OP_ADVANCE, OP_STORE, OP_RESTORE, OP_ADJOINT = 0, 1, 2, 3


class RBProblem:
    """Base state and run length of the objective.

    cfg, prob, params, seed: a set-up from ``workloads`` (params[3], the
    seeded noise amplitude, is ignored: the perturbation is the argument
    ``dT0``).  ``u0`` (optional, state-layout velocity field tensor of shape
    (dim, ...)) adds a fixed initial flow.  ``dt_sched`` (optional device
    tensor) replaces the CFL time steps by a given schedule."""

    def __init__(self, cfg, prob, params, nsteps, slots, seed=0, u0=None, dt_sched=None, device="cuda",
                 objective="kinetic_energy"):
        if objective not in ("kinetic_energy", "nu_bot", "nu_top"):
            raise ValueError(f"unknown objective {objective!r}")
        self.objective = objective
        self.cfg = dict(cfg)
        self.nsteps = int(nsteps)
        self.slots = max(1, min(int(slots), self.nsteps))
        self.device = torch.device(device)
        self.params = list(params[:3])
        self._base = Solver(self.cfg, device=device)
        self.u0 = None
        if u0 is not None:
            self.u0 = torch.as_tensor(u0, dtype=torch.float64, device=self.device).contiguous()
        self.shape = tuple(self._base.U.shape[1:])
        self.dt_sched = dt_sched
        self._solvers = {}

    @property
    def rho(self):
        """Density field of the base state (any perturbation keeps it)."""
        return self.initial_state(torch.zeros(self.shape, dtype=torch.float64, device=self.device))[0]

    def solver(self, mu, kappa):
        key = (float(mu), float(kappa))
        if key not in self._solvers:
            self._solvers.clear()
            self._solvers[key] = Solver(dict(self.cfg, mu=key[0], kappa=key[1]), device=self.device)
        return self._solvers[key]

    def build(self, S, dT0):
        """U^0 into S.U (ars_init_rb_dT: base density and flow, p = rho (T + dT0))."""
        S.init_rb_dT(self.params, dT0.detach().to(self.device, torch.float64).contiguous(), self.u0)
        return S.U

    def initial_state(self, dT0):
        """A copy of U^0 for the perturbation dT0."""
        return self.build(self._base, dT0).clone()


def scratch_states(S):
    """Four scratch states for the executors below (the solver's state and
    scratch and two more): with the current state and an advance's output
    among them, two remain for its ping-pong."""
    return [S.U, S.tmp, torch.empty_like(S.U), torch.empty_like(S.U)]


def _advance(S, plan, i, cur, snaps, scratch, log, adaptive):
    """The advance plan[i] out of place from cur, its last step written
    straight into the snapshot a following store names (that store is then
    done: the returned index points at it); adaptive: CFL steps that log
    their dt into log, else the logged dts.  Returns (index, output)."""
    _, step, arg = plan[i]
    nxt = plan[i + 1] if i + 1 < len(plan) else None
    out = None
    if nxt is not None and nxt[0] == OP_STORE and (snaps[nxt[2]] is not cur or arg - step >= 2):
        out = snaps[nxt[2]]
        i += 1
    free = [b for b in scratch if b is not cur and b is not out]
    if out is None:
        out = free.pop()
    if adaptive:
        S.step_to(cur, out, free[0], free[1], arg - step, dt_log=log[step:arg])
    else:
        S.step_sched_to(cur, out, free[0], free[1], log[step:arg])
    return i, out


def run_to_first_adjoint(S, plan, snaps, log, scratch, adaptive):
    """The plan's forward sweep, every operation before its first adjoint
    step, without state copies (a restore selects its snapshot, a store is
    the preceding advance's last write).  Returns the index of that adjoint
    operation and the buffer holding its state (step n - 1)."""
    cur = snaps[0]
    i = 0
    while plan[i][0] != OP_ADJOINT:
        op, step, arg = plan[i]
        if op == OP_RESTORE:
            cur = snaps[arg]
        elif op == OP_ADVANCE and arg > step:
            i, cur = _advance(S, plan, i, cur, snaps, scratch, log, adaptive)
        elif op == OP_STORE and snaps[arg] is not cur:
            snaps[arg].copy_(cur)
            cur = snaps[arg]
        i += 1
    return i, cur


def run_plan(S, plan, snaps, log, lam, lam_next, pg, start=0, cur=None, scratch=None):
    """Execute a revolve plan from operation `start` (the state of that
    point in `cur`, default snapshot 0) without state copies: the current
    state is wherever it was last written (a snapshot or one of the scratch
    states); a restore only selects its snapshot, an advance runs out of
    place (ars_step_sched_to, the logged dts) with its last step written
    straight into the snapshot a following store names, and the adjoint
    step reads the current state in place.  lam and lam_next alternate;
    returns the one that holds the last adjoint."""
    scratch = scratch_states(S) if scratch is None else scratch
    cur = snaps[0] if cur is None else cur
    i = start
    while i < len(plan):
        op, step, arg = plan[i]
        if op == OP_RESTORE:
            cur = snaps[arg]
        elif op == OP_ADVANCE and arg > step:
            i, cur = _advance(S, plan, i, cur, snaps, scratch, log, False)
        elif op == OP_STORE:
            if snaps[arg] is not cur:
                snaps[arg].copy_(cur)
                cur = snaps[arg]
        elif op == OP_ADJOINT:
            S.step_adjoint(cur, lam, log[step:step + 1], lam_n=lam_next, param_grad=pg)
            lam, lam_next = lam_next, lam
        i += 1
    return lam


class _RBObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, dT0, mu, kappa, problem):
        S = problem.solver(mu.item(), kappa.item())
        U0 = problem.build(S, dT0).clone()
        n, s = problem.nsteps, problem.slots
        plan, _ = revolve_plan(n, s)
        snaps = [U0] + [torch.empty_like(U0) for _ in range(s - 1)]
        scratch = scratch_states(S)
        adaptive = problem.dt_sched is None
        if adaptive:
            log = torch.zeros(n, dtype=torch.float64, device=problem.device)
        else:
            log = problem.dt_sched.to(problem.device, torch.float64).contiguous()
        # the plan's forward sweep is the forward run itself (its CFL dts
        # logged), so the adjoint sweep starts at its first adjoint step
        start, cur = run_to_first_adjoint(S, plan, snaps, log, scratch, adaptive)
        free = [b for b in scratch if b is not cur]
        Un = free[0]
        if adaptive:
            S.step_to(cur, Un, free[1], free[2], 1, dt_log=log[n - 1:n])
        else:
            S.step_sched_to(cur, Un, free[1], free[2], log[n - 1:n])
        grad = torch.empty_like(U0)
        if problem.objective == "kinetic_energy":
            J = S.kinetic_energy(U=Un, grad=grad).clone()
        else:
            J = S.nusselt(0 if problem.objective == "nu_bot" else 1, U=Un, grad=grad).clone()
        rc, cell = S.fault()
        if rc != 0:
            raise ArsError(rc, f"forward run (fault at cell {cell})")
        ctx.problem = problem
        ctx.S = S
        ctx.run = (plan, snaps, scratch, start, cur)
        ctx.save_for_backward(U0, log, grad)
        return J.reshape(())

    @staticmethod
    def backward(ctx, gJ):
        problem, S = ctx.problem, ctx.S
        U0, log, gradN = ctx.saved_tensors
        plan, snaps, scratch, start, cur = ctx.run
        lam = gradN * gJ.to(gradN.dtype)
        lam_next = torch.empty_like(lam)
        pg = torch.zeros(2, dtype=torch.float64, device=problem.device)
        lam = run_plan(S, plan, snaps, log, lam, lam_next, pg, start=start, cur=cur, scratch=scratch)
        ctx.run = None
        g_dT = S.init_rb_dT_adjoint(U0, lam)
        return g_dT, pg[0].reshape(()), pg[1].reshape(()), None


def rb_objective(dT0, mu, kappa, problem):
    """J = problem.objective (final kinetic energy or Nusselt number) after
    problem.nsteps steps from the base state with temperature perturbation
    dT0 (differentiable in dT0, mu, kappa)."""
    mu = torch.as_tensor(mu, dtype=torch.float64)
    kappa = torch.as_tensor(kappa, dtype=torch.float64)
    return _RBObjective.apply(dT0, mu, kappa, problem)


def rb_kinetic_energy(dT0, mu, kappa, problem):
    """J = kinetic energy after problem.nsteps steps from the base state with
    temperature perturbation dT0 (differentiable in dT0, mu, kappa)."""
    if problem.objective != "kinetic_energy":
        raise ValueError("problem was built for another objective; use rb_objective")
    return rb_objective(dT0, mu, kappa, problem)


def rb_kinetic_energy_ra_pr(dT0, Ra, Pr, problem, **layer):
    """Same with the transport coefficients from (Ra, Pr) of the layer."""
    mu, kappa = workloads.ra_pr_to_mu_kappa(Ra, Pr, **layer)
    return rb_kinetic_energy(dT0, mu, kappa, problem)


def rb_objective_ra_pr(dT0, Ra, Pr, problem, **layer):
    """problem.objective with the transport coefficients from (Ra, Pr)."""
    mu, kappa = workloads.ra_pr_to_mu_kappa(Ra, Pr, **layer)
    return rb_objective(dT0, mu, kappa, problem)
