"""Binomial checkpointing plan (host code of the library; no GPU).

Pins: the minimal forward-step count equals Griewank's closed form
t(n, s) = r n - C(s + r, s + 1) with r the smallest integer such that
C(s + r, s) >= n (200 steps, 16 slots -> 429), and every plan, simulated on
integer 'states', runs each adjoint exactly once, in reverse order, on the
right state, within the slot budget, advancing exactly that many steps."""
from math import comb

import pytest

import paper_1903_09043_amd as A


def closed_form(n, s):
    r = 0
    while comb(s + r, s) < n:
        r += 1
    return r * n - comb(s + r, s + 1)


def test_closed_form_values():
    assert A.revolve_cost(200, 16) == 429
    for n in range(1, 160):
        for s in range(1, 12):
            assert A.revolve_cost(n, s) == closed_form(n, s), (n, s)


@pytest.mark.parametrize("n,s", [(1, 1), (2, 1), (7, 1), (10, 3), (33, 4), (200, 16), (64, 64), (129, 5)])
def test_plan_simulation(n, s):
    acts, fwd = A.revolve_plan(n, s)
    slots = {0: 0}
    work = None
    order = []
    advanced = 0
    for op, step, arg in acts:
        if op == 2:  # restore
            assert slots.get(arg) == step
            work = step
        elif op == 0:  # advance
            assert work == step and arg > step
            advanced += arg - step
            work = arg
        elif op == 1:  # store
            assert work == step and 0 <= arg < s
            slots[arg] = step
        elif op == 3:  # adjoint
            assert work == step
            order.append(step)
        else:
            raise AssertionError(op)
    assert order == list(range(n - 1, -1, -1))
    assert advanced == fwd == A.revolve_cost(n, s)
    assert max(slots) < s


class _LabelSolver:
    """Stand-in for the solver: a state buffer holds the index of the step
    whose state it is (NaN once clobbered as ping-pong scratch), and the
    calls check what ars_step_sched_to and the adjoint step require."""

    def __init__(self, torch):
        self.torch = torch
        self.U = torch.full((1,), float("nan"), dtype=torch.float64)
        self.tmp = torch.full((1,), float("nan"), dtype=torch.float64)
        self.seen = []
        self.copies = 0

    def step_sched_to(self, U_in, U_out, a, b, dt_sched):
        n = dt_sched.numel()
        assert n >= 1 and a is not b
        assert U_in is not a and U_in is not b and U_out is not a and U_out is not b
        assert not (n == 1 and U_out is U_in)
        start = U_in.item()
        assert start == start, "advance from a clobbered buffer"
        if n >= 2:
            a.fill_(float("nan"))
        if n >= 3:
            b.fill_(float("nan"))
        U_out.fill_(start + n)

    def step_to(self, U_in, U_out, a, b, n, dt_log=None):
        """CFL steps: the same rules, and each step logs its index as dt."""
        start = U_in.item()
        self.step_sched_to(U_in, U_out, a, b, self.torch.zeros(n, dtype=self.torch.float64))
        if dt_log is not None:
            dt_log.copy_(self.torch.arange(start, start + n, dtype=self.torch.float64))

    def step_adjoint(self, U_n, lam, dt, lam_n=None, param_grad=None):
        self.seen.append((int(dt[0].item()), U_n.item()))
        lam_n.copy_(lam + 1)


@pytest.mark.parametrize("n,s", [(200, 16), (50, 4), (10, 3), (7, 7), (30, 1), (5, 2), (1, 1)])
def test_copy_free_plan_executor(n, s):
    """The adjoint sweep's executor (no state copies) hands every adjoint
    step n-1, ..., 0 the state of its own step, never advances in place or
    from a clobbered buffer, and returns the last adjoint."""
    import torch
    from paper_1903_09043_amd.adjoint import run_plan
    plan, _ = A.revolve_plan(n, s)
    S = _LabelSolver(torch)
    U0 = torch.zeros(1, dtype=torch.float64)
    snaps = [U0] + [torch.full((1,), float("nan"), dtype=torch.float64) for _ in range(s - 1)]
    log = torch.arange(n, dtype=torch.float64)  # dt of step k = k: the adjoint step sees its index
    lam = torch.zeros(1, dtype=torch.float64)
    lam_next = torch.empty_like(lam)
    out = run_plan(S, plan, snaps, log, lam, lam_next, None)
    assert S.seen == [(k, float(k)) for k in range(n - 1, -1, -1)]
    assert out.item() == n
    assert U0.item() == 0.0


@pytest.mark.parametrize("n,s", [(200, 16), (50, 4), (10, 3), (7, 7), (30, 1), (5, 2), (1, 1)])
def test_forward_sweep_then_adjoint_sweep(n, s):
    """As the autograd objective runs it: the plan's forward sweep with CFL
    steps that log their dts (run_to_first_adjoint), state n from state
    n - 1 for the objective, then the adjoint sweep from the first adjoint
    step on the logged dts: every adjoint step sees its own state, and the
    log holds every step's dt."""
    import torch
    from paper_1903_09043_amd.adjoint import run_plan, run_to_first_adjoint, scratch_states
    plan, _ = A.revolve_plan(n, s)
    S = _LabelSolver(torch)
    U0 = torch.zeros(1, dtype=torch.float64)
    snaps = [U0] + [torch.full((1,), float("nan"), dtype=torch.float64) for _ in range(s - 1)]
    scratch = scratch_states(S)
    log = torch.full((n,), float("nan"), dtype=torch.float64)
    start, cur = run_to_first_adjoint(S, plan, snaps, log, scratch, True)
    assert plan[start][0] == 3 and plan[start][1] == n - 1 and cur.item() == n - 1
    free = [b for b in scratch if b is not cur]
    S.step_to(cur, free[0], free[1], free[2], 1, dt_log=log[n - 1:n])
    assert free[0].item() == n and cur.item() == n - 1
    assert torch.equal(log, torch.arange(n, dtype=torch.float64))
    lam = torch.zeros(1, dtype=torch.float64)
    out = run_plan(S, plan, snaps, log, lam, torch.empty_like(lam), None, start=start, cur=cur, scratch=scratch)
    assert S.seen == [(k, float(k)) for k in range(n - 1, -1, -1)]
    assert out.item() == n and U0.item() == 0.0
