"""Batched persistent launch (ars_batch_*) on an MI355X.

Every instance of a batch must equal the single-problem path (ars_step on
that instance alone, the same kernel code) bit for bit: same states, same
accumulated time, same next dt.  One instance is also checked against the
oracle directly, to the 1e-12 scale-aware tolerance of tests/parity.py
(the oracle evaluates the paper's quotients, the kernels reciprocal
products).  Also: independence of the tiling (row
segments per workgroup, vertical chunks), continuation (a + b steps equal
a then b), graph capture and replay, and the largest instance size of the
batched workload.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1903_09043_amd import workloads as W
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


def mixed_setups():
    """Uneven sizes (including ragged widths and heights that are not
    multiples of a segment or a power of two), theta on and off, with and
    without dissipation, periodic / outflow sides."""
    out = []
    sizes = [(64, 32), (128, 64), (20, 12), (61, 7), (256, 128), (121, 40), (64, 32), (7, 5)]
    for k, (nx, nz) in enumerate(sizes):
        cfg, prob, prm, seed = W.rb([nx, nz], [2.0, 1.0], Ra=10 ** (2.7 + 0.2 * k), seed=100 + k, amp=1e-2,
                                    low_mach=k % 2)
        if k == 3:
            cfg = dict(cfg, mu=0.0, kappa=0.0)
        if k == 5:
            cfg = dict(cfg, bc=[[2, 2], [1, 1]])
        out.append((cfg, prob, prm, seed))
    cfg, prob, prm, seed = W.gresho(n=48, Ma=0.05)
    out.append((cfg, prob, prm, seed))
    return out


def init_batch(A, setups):
    import torch
    B = A.Batch([s[0] for s in setups])
    for k, (cfg, prob, prm, seed) in enumerate(setups):
        U = A.Context(cfg).init_host(prob, prm, seed)
        B.view(k).copy_(torch.from_numpy(U))
    return B


def single(A, cfg, prob, prm, seed, n):
    import torch
    S = A.Solver(cfg).init(prob, prm, seed)
    S.step(n)
    torch.cuda.synchronize()
    rc, fc = S.fault()
    assert rc == 0, (cfg["n"], fc)
    return S.numpy(), S.t.item(), S.dt.item()


def check_against_single(A, B, setups, n, what):
    import torch
    torch.cuda.synchronize()
    t, dt, fc, rc = B.read()
    assert rc == 0 and np.all(fc == -1), fc
    for k, s in enumerate(setups):
        U, ts, dts = single(A, *s, n)
        Ub = B.view(k).cpu().numpy()
        ok = np.array_equal(Ub, U) and t[k] == ts and dt[k] == dts
        if not ok:
            say(what, "instance", k, s[0]["n"], "max diff", float(np.max(np.abs(Ub - U))), t[k], ts, dt[k], dts)
        assert ok, (what, k)


def test_batch_equals_single_path(A):
    setups = mixed_setups()
    n = 40
    for rows in (4, 8):
        say("batch rows", rows, "instances", len(setups), "steps", n)
        B = init_batch(A, setups)
        B.set_tiling(rows).bind()
        B.step(n)
        check_against_single(A, B, setups, n, f"rows={rows}")


def test_batch_tiling_independence(A):
    import torch
    setups = mixed_setups()
    n = 25
    ref = None
    for rows, zmode in ((4, "default"), (8, "default"), (4, "one"), (8, "max"), (4, "max")):
        B = init_batch(A, setups)
        zc = None
        if zmode == "one":
            zc = [1] * len(setups)
        elif zmode == "max":
            zc = [max(z for z in (1, 2, 4, 8, 16) if c["n"][1] % z == 0) for c, *_ in setups]
        B.set_tiling(rows, zc).bind()
        say("tiling", rows, zmode, B.tiling()[1])
        B.step(n)
        torch.cuda.synchronize()
        got = (B.states.cpu().numpy(), B.read()[:2])
        if ref is None:
            ref = got
        else:
            assert np.array_equal(got[0], ref[0])
            assert np.array_equal(got[1][0], ref[1][0]) and np.array_equal(got[1][1], ref[1][1])


def test_batch_continuation_and_graph(A):
    import torch
    setups = mixed_setups()
    B1 = init_batch(A, setups)
    B1.step(30)
    torch.cuda.synchronize()
    B2 = init_batch(A, setups)
    B2.step(12).step(18)
    torch.cuda.synchronize()
    assert np.array_equal(B1.states.cpu().numpy(), B2.states.cpu().numpy())
    assert np.array_equal(B1.read()[0], B2.read()[0])
    # graph: capture 10 steps, replay 3 times; after every replay compare
    # with the eager batch advanced by the same number of steps
    G = init_batch(A, setups)
    E = init_batch(A, setups)
    s = torch.cuda.Stream()
    G.bind()
    with torch.cuda.stream(s):
        G.capture(10, s)
    for r in range(3):
        with torch.cuda.stream(s):
            G.replay(s)
        s.synchronize()
        E.step(10)
        torch.cuda.synchronize()
        say("replay", r)
        assert np.array_equal(G.states.cpu().numpy(), E.states.cpu().numpy())
        assert np.array_equal(G.read()[0], E.read()[0])


def test_batch_instance_vs_oracle(A):
    """One batched instance (2D RB 64x32, Ra = 1e4, theta on) against the
    oracle directly, 300 steps, beside two other instances."""
    import torch
    setups = [W.rb2d_64x32(), W.rb([128, 64], [2.0, 1.0], Ra=2e3, seed=9), W.rb([30, 20], [2.0, 1.0], Ra=800, seed=4)]
    B = init_batch(A, setups)
    B.step(300)
    torch.cuda.synchronize()
    cfg, prob, prm, seed = setups[0]
    Uo = O.init(cfg, prob, prm, seed)
    r = O.run(cfg, Uo, 300)
    assert r["status"] == 0
    U = B.view(0).cpu().numpy()
    o = r["U"]
    err = P.rel_err(cfg, U, o)
    say("batch instance vs oracle, 300 steps: parity %.3e (each variable on its own max: %.3e)"
        % (err, P.strict_err(U, o)), "bitwise", np.array_equal(U, o))
    assert err <= 1e-12
    assert abs(B.read()[0][0] - r["t"]) <= 1e-13 * r["t"]


def test_batch_workload_sizes_500_steps(A):
    """The first 24 instances of the 512-instance batched workload (sizes
    from {64x32, 128x64, 256x128}, Ra log-uniform in [5e2, 5e3]), 500 steps,
    against the single-problem path."""
    setups = W.rb2d_batch()[:24]
    B = init_batch(A, setups)
    B.step(500)
    check_against_single(A, B, setups, 500, "rb2d_batch[:24]")


def test_autotune_and_cache(A, tmp_path):
    """The batch and step autotuners pick a shape, store it in the cache,
    find it there the second time, and leave results unchanged."""
    import torch
    setups = mixed_setups()
    cache = str(tmp_path / "tune.txt")
    B = init_batch(A, setups)
    r1 = B.autotune(trial_steps=3, cache_path=cache)
    say("batch tune", r1, B.tiling()[0])
    assert r1["from_cache"] == 0 and r1["n_candidates"] >= 2 and r1["rows"] in (4, 8)
    B.step(20)
    check_against_single(A, B, setups, 20, "tuned")
    B2 = init_batch(A, setups)
    r2 = B2.autotune(trial_steps=3, cache_path=cache)
    assert r2["from_cache"] == 1 and r2["rows"] == r1["rows"] and r2["zc_policy"] == r1["zc_policy"]
    cfg, prob, prm, seed = W.rb([40, 24, 16], [1.0, 1.0, 1.0], Ra=1e5, seed=2)
    S = A.Solver(cfg).init(prob, prm, seed)
    U0 = S.U.clone()
    r3 = S.autotune(trial_steps=2, cache_path=cache)
    say("step tune", r3)
    assert r3["from_cache"] == 0 and r3["n_candidates"] >= 2
    assert torch.equal(S.U, U0)
    assert S.ctx.tiling() == (r3["zchunk"], r3["wg_per_cu"]) and S.ctx.tile3 == r3["tile3"]
    S.compute_dt()
    S.step(5)
    ref = A.Solver(cfg).init(prob, prm, seed).step(5)
    torch.cuda.synchronize()
    assert torch.equal(S.U, ref.U) and S.t.item() == ref.t.item()
    assert S.fault()[0] == 0
    # the tuned run against the oracle directly
    r = O.run(cfg, O.init(cfg, prob, prm, seed), 5)
    err = P.rel_err(cfg, S.numpy(), r["U"])
    say("tuned step vs oracle", err)
    assert err <= 1e-12
    S2 = A.Solver(cfg)
    S2.U.copy_(U0)
    assert S2.autotune(trial_steps=2, cache_path=cache)["from_cache"] == 1
    lines = open(cache).read().splitlines()
    assert len(lines) == 2 and lines[0].startswith("batch:") and lines[1].startswith("step:")


def test_batch_degenerate_instances(A):
    """Instances one cell wide or tall, narrower than a row segment, or with
    outflow sides, mixed with a regular one: bitwise equal to the
    single-problem path after 30 steps, for both row counts."""
    import torch
    from tests import inputs as I

    def cfg(n, L, bc, g=0.0, thermal=(0, 0), T_wall=(1.0, 1.0), lm=1):
        return dict(dim=2, n=list(n), L=list(L), gamma=5.0 / 3.0, g=g, mu=2e-3, kappa=3e-3, K=1.1, cfl=0.4,
                    low_mach=lm, dt_mode=0, bc=bc, wall_noslip=1, thermal=list(thermal), T_wall=list(T_wall))

    cfgs = [cfg([1, 7], [0.2, 1.0], [[0, 0], [1, 1]], g=1.0, thermal=(1, 1), T_wall=(1.0, 0.5)),
            cfg([5, 1], [1.0, 0.2], [[0, 0], [0, 0]]),
            cfg([3, 2], [1.0, 1.0], [[2, 2], [2, 2]], lm=0),
            cfg([61, 4], [2.0, 1.0], [[2, 2], [1, 1]], g=1.0, thermal=(1, 0), T_wall=(1.0, 0.5)),
            W.rb([64, 32], [2.0, 1.0], Ra=1e4)[0]]
    states = []
    for k, c in enumerate(cfgs):
        if c["g"] != 0.0:
            U = O.init(c, W.PROB_RB, [c["T_wall"][0], c["T_wall"][1], -1.0, 1e-2], k)
        else:
            U = I.white_random(c, seed=k)
        states.append(U)
    for rows in (4, 8):
        B = A.Batch(cfgs)
        for k, U in enumerate(states):
            B.view(k).copy_(torch.from_numpy(U))
        B.set_tiling(rows).bind()
        B.step(30)
        torch.cuda.synchronize()
        t, dt, fc, rc = B.read()
        assert rc == 0
        for k, (c, U) in enumerate(zip(cfgs, states)):
            S = A.Solver(c)
            S.set_state(U)
            S.step(30)
            torch.cuda.synchronize()
            assert np.array_equal(B.view(k).cpu().numpy(), S.numpy()), (rows, k, c["n"])
            assert t[k] == S.t.item() and dt[k] == S.dt.item()


def test_batch_nonconservative_instances(A):
    """Instances with the App. B energy form beside conservative ones (two
    variants of the batched kernel in one step call): each equals its
    single-problem run bit for bit."""
    import torch
    setups = [W.rb([64, 32], [2.0, 1.0], Ra=2e3, seed=3, amp=1e-2), W.rb([30, 20], [2.0, 1.0], Ra=900, seed=4, amp=1e-2),
              W.rb([128, 64], [2.0, 1.0], Ra=3e3, seed=5, amp=1e-2)]
    setups = [(dict(c, energy_form=k % 2), p, q, s) for k, (c, p, q, s) in enumerate(setups)]
    B = init_batch(A, setups)
    B.step(40)
    check_against_single(A, B, setups, 40, "energy forms")
