"""GPU parity of the plane kinetic-energy spectrum (ars_spectrum) against the
oracle's FFT spectrum, on seeded synthetic states.

Acceptance: |E_gpu(s) - E_oracle(s)| <= 1e-12 * sum_s E_oracle + 1e-10 |E_oracle(s)|
per shell.  The GPU path is a radix-2 FFT when both sides are powers of two
and a direct DFT otherwise, the oracle an FFT, so the two differ only by
rounding: a sum of n products carries an error of a few n eps relative to
the field's energy (log2 n eps for the FFT), below 1e-12 for n <= 2048.
The sizes below take both paths.
"""
import sys

import numpy as np
import pytest

import oracle as O
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


def cfg_of(dim, n):
    return dict(dim=dim, n=list(n), L=[1.0] * dim, gamma=5.0 / 3.0, g=0.0, mu=0.0, kappa=0.0, K=1.1, cfl=0.4,
                low_mach=1, dt_mode=0, bc=[[0, 0]] * dim, wall_noslip=1, thermal=[0, 0], T_wall=[1.0, 1.0])


def gpu_spectrum(A, cfg, U, kz):
    import torch
    S = A.Solver(cfg)
    S.set_state(U)
    e1 = S.spectrum(kz)
    e2 = S.spectrum(kz)
    torch.cuda.synchronize()
    e1, e2 = e1.cpu().numpy(), e2.cpu().numpy()
    assert np.array_equal(e1, e2), "spectrum not deterministic"
    return e1


def check(g, o):
    assert g.shape == o.shape, (g.shape, o.shape)
    tol = 1e-12 * o.sum() + 1e-10 * np.abs(o)
    err = np.abs(g - o)
    assert np.all(err <= tol), f"worst shell {int(np.argmax(err - tol))}: {err.max():.3e}"


@pytest.mark.parametrize("dim,n,kz,kind", [
    (3, [64, 48, 8], 4, "white"),
    (3, [37, 29, 5], 2, "white"),        # odd sides: ragged rows of the 256-thread blocks
    (3, [96, 80, 6], 3, "smooth"),
    (3, [300, 2, 3], 1, "white"),        # two-cell side
    (3, [1, 40, 3], 0, "white"),         # one-cell side
    (3, [1000, 750, 3], 1, "smooth"),    # ragged 16 x 16 matrix tiles in both directions, large
    (2, [257, 9], 4, "white"),           # 2D: a line
    (2, [2048, 5], 2, "white"),          # 2D: the longest line
    (2, [1, 4], 3, "white"),             # a single cell
    (3, [64, 32, 4], 2, "white"),        # powers of two: the FFT path (4-column tiles)
    (3, [2, 4, 3], 1, "white"),          # the FFT path at its smallest transforms
    (3, [16, 1, 3], 1, "white"),         # the FFT path with a one-cell side
    (2, [256, 5], 1, "smooth"),          # 2D line on the FFT path
])
def test_spectrum_vs_oracle(A, dim, n, kz, kind):
    say("spectrum", dim, n, kz, kind)
    cfg = cfg_of(dim, n)
    U = I.white_random(cfg, 21, amp=0.3) if kind == "white" else I.smooth_random(cfg, 22, amp_u=0.4, modes=9)
    check(gpu_spectrum(A, cfg, U, kz), O.spectrum(cfg, U, kz))


def test_spectrum_single_mode(A):
    """u_x = A cos(2 pi (3 x + 4 y)) at uniform density: all energy rho A^2 / 4
    in shell 5."""
    say("spectrum single mode")
    cfg = cfg_of(3, [32, 24, 4])
    U = np.zeros((5, 4, 24, 32))
    U[0] = 1.3
    U[4] = 2.0
    y = (np.arange(24) / 24)[:, None]
    x = (np.arange(32) / 32)[None, :]
    U[1, 2] = 1.3 * 0.7 * np.cos(2 * np.pi * (3 * x + 4 * y))
    E = gpu_spectrum(A, cfg, U, 2)
    assert E.shape == (21,)
    assert abs(E[5] - 1.3 * 0.49 / 4) <= 1e-14
    assert np.all(np.abs(np.delete(E, 5)) <= 1e-14)


def test_spectrum_full_plane_512(A):
    """The 512^2 middle plane of the largest 3D Rayleigh-Benard grid (the
    spectrum's own workload), with a white velocity field; the shells also
    sum to the plane's mean kinetic energy."""
    say("spectrum 512^2 plane")
    cfg = cfg_of(3, [512, 512, 4])
    U = I.white_random(cfg, 23, amp=0.3)
    g = gpu_spectrum(A, cfg, U, 2)
    check(g, O.spectrum(cfg, U, 2))
    ke = np.mean(sum(U[1 + c][2] ** 2 for c in range(3)) / U[0][2]) / 2
    assert abs(g.sum() - ke) <= 1e-12 * ke


def test_spectrum_max_plane(A):
    """The largest plane the kernels take, 2048 x 2048 (LDS holds a column
    of 2048 complex values and its twiddles)."""
    say("spectrum 2048^2 plane")
    cfg = cfg_of(3, [2048, 2048, 2])
    U = I.white_random(cfg, 24, amp=0.3)
    check(gpu_spectrum(A, cfg, U, 1), O.spectrum(cfg, U, 1))


def test_binding_rejects_bad_tensors(A):
    """The binding checks caller tensors before passing their pointers to
    the C ABI (the kernels would read past a short or mistyped buffer): no
    kernel runs for any of these calls."""
    import torch
    cfg = cfg_of(3, [16, 12, 8])
    S = A.Solver(cfg)
    S.set_state(I.white_random(cfg, 1))
    good = S.U.clone()
    bad = [good.float(), good.transpose(1, 2), good.reshape(-1)[:-1], good.cpu()]
    for U in bad:
        with pytest.raises(ValueError):
            S.spectrum(U=U)
        with pytest.raises(ValueError):
            S.kinetic_energy(U=U)
    with pytest.raises(ValueError):
        S.spectrum(out=torch.empty(3, dtype=torch.float64, device="cuda"))
    lam = torch.zeros_like(good)
    with pytest.raises(ValueError):
        S.step_adjoint(good, lam.reshape(-1)[:-1], torch.tensor([1e-3], dtype=torch.float64))
    with pytest.raises(ValueError):
        S.step_adjoint(good, lam, torch.tensor([1e-3], dtype=torch.float64),
                       param_grad=torch.zeros(1, dtype=torch.float64, device="cuda"))
    # and the good tensors pass
    E = S.spectrum(U=good)
    torch.cuda.synchronize()
    assert torch.isfinite(E).all()
