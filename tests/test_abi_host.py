"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point include/ars.h declares, validates configurations like the
oracle, and builds initial states bit-identical to the oracle's."""
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1903_09043_amd as A
from paper_1903_09043_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "ars.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ars_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = A.lib()
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(L, s), s
    bound = {name for name, _, _ in A.SIGNATURES}
    assert set(syms) <= bound, set(syms) - bound


def test_strerror():
    for s in (0, -1, -2, -3, -4, -5):
        assert A.lib().ars_strerror(s)


CFGS = [
    W.rb2d_64x32()[0],
    W.gresho(n=64)[0],
    W.rb([12, 10, 8], [1.0, 1.0, 1.0], Ra=1e5)[0],
]


def test_validate_agrees_with_oracle():
    good = dict(CFGS[0])
    cases = [{}, dict(dim=4), dict(n=[0, 8]), dict(gamma=1.0), dict(mu=-1.0), dict(K=0.9), dict(cfl=0.0),
             dict(bc=[[0, 0], [0, 0]]), dict(bc=[[1, 1], [1, 1]]), dict(bc=[[0, 2], [1, 1]]), dict(dt_mode=3),
             dict(g=0.0, bc=[[2, 2], [0, 0]]), dict(g=0.0, bc=[[0, 0], [2, 2]])]
    for c in cases:
        cfg = dict(good)
        cfg.update(c)
        assert (A.validate(cfg) == 0) == (O.validate(cfg) == 0), c


def test_create_rejects_1d():
    cfg = dict(dim=1, n=[16], L=[1.0], bc=[[0, 0]])
    assert A.validate(cfg) == 0
    with pytest.raises(A.ArsError) as e:
        A.Context(cfg)
    assert e.value.status == A.EUNSUPPORTED


@pytest.mark.parametrize("which", ["rb2d", "rb3d", "gresho", "gresho_odd", "sod", "iso", "uniform", "rb2d_seed"])
def test_host_init_bitwise_equals_oracle(which):
    if which == "rb2d":
        cfg, prob, prm, seed = W.rb2d_64x32()
    elif which == "rb2d_seed":
        cfg, prob, prm, seed = W.rb([30, 17], [2.0, 1.0], Ra=3e3, seed=987654321, amp=1e-3)
    elif which == "rb3d":
        cfg, prob, prm, seed = W.rb([12, 10, 9], [1.0, 1.0, 1.0], Ra=1e5, seed=5)
    elif which == "gresho":
        cfg, prob, prm, seed = W.gresho(n=96, Ma=1e-2)
    elif which == "gresho_odd":  # a cell centre on the vortex centre
        cfg, prob, prm, seed = W.gresho(n=33, Ma=1e-2)
    elif which == "sod":
        cfg = dict(dim=2, n=[100, 3], L=[1.0, 1.0], gamma=1.4, bc=[[2, 2], [0, 0]])
        prob, prm, seed = W.PROB_SOD, [], 0
    elif which == "iso":
        cfg = dict(dim=2, n=[4, 128], L=[1.0, 3.0], g=1.0, bc=[[0, 0], [1, 1]])
        prob, prm, seed = W.PROB_ISOTHERMAL, [], 0
    else:
        cfg = dict(dim=3, n=[5, 4, 3], L=[1.0, 1.0, 1.0], bc=[[0, 0]] * 3)
        prob, prm, seed = W.PROB_UNIFORM, [1.2, 0.1, -0.2, 0.3, 2.5], 0
    a = A.Context(cfg).init_host(prob, prm, seed)
    b = O.init(cfg, prob, prm, seed)
    assert a.shape == b.shape
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))


def test_workloads_transport_coefficients():
    """Ra/Pr -> (mu, kappa) reading for the linear-T layer: mu * kappa ~ 1/Ra
    and the values quoted for Ra = 1e4, Pr = 1."""
    mu, k = W.ra_pr_to_mu_kappa(1e4, 1.0)
    assert abs(mu - 2.7386e-3) < 1e-7 and abs(k - 6.8465e-3) < 1e-7
    mu2, k2 = W.ra_pr_to_mu_kappa(4e4, 1.0)
    assert abs(mu2 * k2 * 4 - mu * k) < 1e-15
    insts = W.rb2d_batch()
    assert len(insts) == 512
    sizes = {tuple(c["n"]) for c, *_ in insts}
    assert sizes == {(64, 32), (128, 64), (256, 128)}
    ras = [W.ra_pr_to_mu_kappa(1.0, 1.0)[0] / c["mu"] for c, *_ in insts]
    ras = np.array(ras) ** 2
    assert ras.min() >= 5e2 * (1 - 1e-9) and ras.max() <= 5e3 * (1 + 1e-9)


def test_batch_host_side():
    """ars_batch_create / tiling / layout need no GPU: sizes, offsets,
    rejection of 3D and invalid instances, tiling checks."""
    import ctypes as C
    L = A.lib()
    cfgs = [W.rb([64, 32], [2.0, 1.0])[0], W.rb([20, 12], [2.0, 1.0])[0], W.gresho(n=48)[0]]

    def create(cs):
        arr = (A.ArsConfig * len(cs))(*[A.make_config(c) for c in cs])
        h = C.c_void_p()
        return L.ars_batch_create(len(cs), arr, C.byref(h)), h

    rc, h = create(cfgs)
    assert rc == 0
    try:
        cells = [64 * 32, 20 * 12, 48 * 48]
        assert L.ars_batch_state_len(h) == 4 * sum(cells)
        assert [L.ars_batch_state_offset(h, k) for k in range(3)] == [0, 4 * cells[0], 4 * (cells[0] + cells[1])]
        assert L.ars_batch_table_bytes(h) > 0
        r = C.c_int()
        z = (C.c_int * 3)()
        assert L.ars_batch_get_tiling(h, C.byref(r), z) == 0 and r.value == 4
        assert all(cfg["n"][1] % v == 0 for cfg, v in zip(cfgs, z))
        assert L.ars_batch_set_tiling(h, 6, None) == A.EINVAL
        assert L.ars_batch_set_tiling(h, 8, (C.c_int * 3)(2, 5, 1)) == A.EINVAL  # 5 does not divide 12
        assert L.ars_batch_set_tiling(h, 8, (C.c_int * 3)(2, 4, 16)) == 0
        assert L.ars_batch_get_tiling(h, C.byref(r), z) == 0 and r.value == 8 and list(z) == [2, 4, 16]
        assert L.ars_batch_replay(h, None) == A.EINVAL  # nothing captured
    finally:
        L.ars_batch_destroy(h)
    assert create(cfgs + [W.rb([8, 8, 8], [1.0, 1.0, 1.0])[0]])[0] == A.EUNSUPPORTED
    assert create([dict(cfgs[0], cfl=0.0)])[0] == A.EINVAL
    assert L.ars_batch_create(0, None, C.byref(C.c_void_p())) == A.EINVAL


def test_energy_form_validation():
    """Both energy forms (the relaxed total energy and App. B) are valid
    configurations for every entry point, the adjoint included; any other
    value is rejected by the library and by the oracle, and the adjoint
    entry point checks its pointers before touching any device buffer."""
    import ctypes as C
    cfg, prob, prm, seed = W.rb([8, 6], [2.0, 1.0])
    assert A.validate(dict(cfg, energy_form=1)) == A.OK
    assert A.validate(dict(cfg, energy_form=2)) == A.EINVAL
    assert O.validate(dict(cfg, energy_form=2)) != 0
    ctx = A.Context(dict(cfg, energy_form=1))
    dummy = C.c_void_p(1)
    rc = A.lib().ars_step_adjoint(ctx.h, dummy, dummy, dummy, dummy, None, dummy, None)
    assert rc == A.EINVAL  # d_lam_n aliases d_lam_np1
    rc = A.lib().ars_step_adjoint(ctx.h, dummy, None, C.c_void_p(2), dummy, None, dummy, None)
    assert rc == A.EINVAL


def test_step_sched_to_rejects_aliasing():
    """ars_step_sched_to checks its buffers before any launch: distinct
    scratch states, an input and an output that are not scratch, no
    single step in place, at least one step."""
    import ctypes as C
    cfg, prob, prm, seed = W.rb([8, 6], [2.0, 1.0])
    ctx = A.Context(cfg)
    f = A.lib().ars_step_sched_to
    i, a, b, o, w, d = (C.c_void_p(k) for k in (1, 2, 3, 4, 5, 6))
    assert f(ctx.h, i, a, a, o, w, 2, d, None, None) == A.EINVAL   # a == b
    assert f(ctx.h, a, a, b, o, w, 2, d, None, None) == A.EINVAL   # in == a
    assert f(ctx.h, i, a, b, b, w, 2, d, None, None) == A.EINVAL   # out == b
    assert f(ctx.h, i, a, b, i, w, 1, d, None, None) == A.EINVAL   # one step in place
    assert f(ctx.h, i, a, b, o, w, 0, d, None, None) == A.EINVAL   # no step
    assert f(ctx.h, i, a, b, o, None, 2, d, None, None) == A.EINVAL  # no workspace
    assert f(ctx.h, i, a, b, o, w, 2, None, None, None) == A.EINVAL  # no schedule
    g = A.lib().ars_step_to  # the same rules for the CFL-step form, which also needs d_dt
    assert g(ctx.h, i, a, a, o, w, 2, None, d, None, None) == A.EINVAL   # a == b
    assert g(ctx.h, i, a, b, i, w, 1, None, d, None, None) == A.EINVAL   # one step in place
    assert g(ctx.h, i, a, b, a, w, 2, None, d, None, None) == A.EINVAL   # out == a
    assert g(ctx.h, i, a, b, o, w, 2, None, None, None, None) == A.EINVAL  # no dt


def test_spectrum_host_side():
    """Shell counts and scratch size of the plane spectrum, and its argument
    checks, which return before any device use."""
    import ctypes as C
    L = A.lib()
    base = dict(CFGS[2])
    for n, shells in (([20, 12, 3], 13), ([32, 24, 4], 21), ([4, 4, 2], 4), ([1, 40, 3], 21), ([1, 1, 2], 1)):
        ctx = A.Context(dict(base, n=n))
        assert L.ars_spectrum_len(ctx.h) == shells
        ref = len(O.spectrum(dict(base, n=n), np.ones((5, n[2], n[1], n[0])), 0))
        assert ref == shells
        assert L.ars_workspace_bytes_spectrum(ctx.h) == 12 * n[0] * n[1] * 8
    ctx2 = A.Context(W.rb2d_64x32()[0])
    assert L.ars_spectrum_len(ctx2.h) == 33
    assert L.ars_workspace_bytes_spectrum(ctx2.h) == 8 * 64 * 8
    d = C.c_void_p(1)
    ctx = A.Context(dict(base, n=[16, 16, 8]))
    assert L.ars_spectrum(ctx.h, d, 8, d, d, None) == A.EINVAL
    assert L.ars_spectrum(ctx.h, d, -1, d, d, None) == A.EINVAL
    assert L.ars_spectrum(ctx.h, None, 0, d, d, None) == A.EINVAL
    assert L.ars_spectrum(ctx.h, d, 0, d, None, None) == A.EINVAL
    big = A.Context(dict(base, n=[2049, 4, 2]))
    assert L.ars_spectrum(big.h, d, 0, d, d, None) == A.EUNSUPPORTED


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built HIP library the binding raises instead of falling
    back to anything else, and a solver refuses to run without a GPU."""
    import paper_1903_09043_amd as P
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "libars.so"))
    with pytest.raises(ImportError):
        P.lib()
    with pytest.raises(ImportError):
        P.validate(W.rb2d_64x32()[0])
    monkeypatch.undo()
    import torch
    if not torch.cuda.is_available():
        with pytest.raises(RuntimeError):
            P.Solver(W.rb2d_64x32()[0])


def test_default_vertical_chunk():
    """The default launch shape chosen at ars_create (results never depend
    on it): in 2D a share of about sqrt(segments x planes) / 13 planes, one
    plane for small grids; the 3D bench grid keeps its 37-plane chunks."""
    def zc(cfg):
        return A.Context(cfg).zchunk()
    assert zc(W.rb2d_64x32()[0]) == 1
    assert zc(W.rb([256, 128], [2.0, 1.0])[0]) == 2
    assert zc(W.gresho_1024()[0]) == 10
    assert zc(W.rb3d_ra1e6()[0]) == 37
