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
