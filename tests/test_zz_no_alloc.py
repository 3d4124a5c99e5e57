"""ars_step_noalloc (static library scratch, no caller workspace) against
ars_step on the same inputs, through the C ABI (run on an MI355X).

Two calls in a row on one GPU, the second on a smaller state, each bit for
bit equal to ars_step (state, t, next dt, dt log); a state above the
scratch limit is refused before any launch; a numerical fault leaves dt NaN.
"""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1903_09043_amd import workloads as W

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


def _p(t):
    return C.c_void_p(t.data_ptr())


def _noalloc(A, S, U, t, dt, log, n):
    """ars_step_noalloc through the C ABI on copies of a solver's buffers."""
    import torch
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return A.lib().ars_step_noalloc(S.ctx.h, _p(U), int(n), _p(t), _p(dt), _p(log) if log is not None else None,
                                    stream)


def _compare(A, setup, n):
    import torch
    cfg, prob, prm, seed = setup
    S = A.Solver(cfg).init(prob, prm, seed)
    assert S.ctx.state_len <= A.NOALLOC_MAX_STATE
    U, t, dt = S.U.clone(), S.t.clone(), S.dt.clone()
    log_a = torch.zeros(n, dtype=torch.float64, device="cuda")
    log_b = torch.zeros(n, dtype=torch.float64, device="cuda")
    say("noalloc", cfg["n"], "steps", n)
    rc = _noalloc(A, S, U, t, dt, log_b, n)
    assert rc == A.OK, rc
    S.step(n, dt_log=log_a)
    torch.cuda.synchronize()
    assert torch.equal(U, S.U), cfg["n"]
    assert t.item() == S.t.item() and dt.item() == S.dt.item()
    assert torch.equal(log_a, log_b)
    assert np.isfinite(dt.item())


def test_noalloc_two_calls_second_smaller(A):
    # largest 2D grid that fits the scratch (4 x 256 x 128 doubles), odd
    # count: the result is copied back from the scratch
    _compare(A, W.rb([256, 128], [2.0, 1.0], Ra=2e3, seed=3, amp=1e-2), 7)
    # then a smaller state on the same scratch, even count
    _compare(A, W.rb2d_64x32(), 10)
    # and a 3D one
    _compare(A, W.rb([20, 12, 10], [1.0, 1.0, 1.0], Ra=1e5, seed=2, amp=1e-2), 5)


def test_noalloc_refuses_state_above_limit(A):
    import torch
    cfg, prob, prm, seed = W.rb([257, 128], [2.0, 1.0], Ra=2e3, seed=3, amp=1e-2)
    S = A.Solver(cfg).init(prob, prm, seed)
    assert S.ctx.state_len > A.NOALLOC_MAX_STATE
    U0 = S.U.clone()
    dt0 = S.dt.item()
    rc = _noalloc(A, S, S.U, S.t, S.dt, None, 3)
    torch.cuda.synchronize()
    assert rc == A.ESCRATCH
    assert torch.equal(S.U, U0) and S.dt.item() == dt0


def test_noalloc_fault_gives_nan_dt(A):
    import torch
    cfg = dict(dim=2, n=[16, 12], L=[1.0, 1.0], gamma=5.0 / 3.0, bc=[[0, 0], [0, 0]])
    S = A.Solver(cfg).init(W.PROB_UNIFORM, [1.0, 0.0, 0.0, 0.0, 1.0])
    U = S.U.clone()
    U[0, 5, 9] = -1.0
    dt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    rc = _noalloc(A, S, U, S.t, dt, None, 1)
    torch.cuda.synchronize()
    assert rc == A.OK
    assert np.isnan(dt.item())
    # the next call starts from a cleared latch
    _compare(A, W.rb2d_64x32(), 3)
