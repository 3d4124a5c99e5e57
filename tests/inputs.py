"""Seeded synthetic inputs shared by the oracle tests and the GPU parity
tests.  Holds no arithmetic of the method: only random primitive fields and
their conversion to the state variables (rho, rho u, rho e + rho |u|^2 / 2),
which is the definition of those variables.
"""
import numpy as np


def grid_shape(cfg):
    return tuple(int(cfg["n"][a]) for a in reversed(range(cfg["dim"])))


def prim_to_state(cfg, rho, u, p):
    """rho, p: arrays of grid_shape; u: list of D arrays.  Returns (D+2, ...)"""
    D = cfg["dim"]
    gamma = cfg.get("gamma", 5.0 / 3.0)
    U = np.empty((D + 2,) + rho.shape, dtype=np.float64)
    U[0] = rho
    kin = np.zeros_like(rho)
    for k in range(D):
        U[1 + k] = rho * u[k]
        kin += u[k] * u[k]
    U[1 + D] = p / (gamma - 1.0) + 0.5 * rho * kin
    return U


def smooth_random(cfg, seed, rho0=1.0, p0=1.0, amp_rho=0.2, amp_u=0.3, amp_p=0.2, modes=3):
    """Smooth periodic random field: sums of a few random Fourier modes."""
    rng = np.random.default_rng(seed)
    shape = grid_shape(cfg)
    D = cfg["dim"]
    axes = [np.arange(n) / n for n in shape]  # reversed order (z.., y, x)
    mesh = np.meshgrid(*axes, indexing="ij")

    def field(amp):
        f = np.zeros(shape)
        for _ in range(modes):
            k = rng.integers(-2, 3, size=len(shape))
            ph = rng.uniform(0, 2 * np.pi)
            arg = sum(2 * np.pi * k[i] * mesh[i] for i in range(len(shape))) + ph
            f += rng.uniform(-1, 1) * np.cos(arg)
        return amp * f / modes

    rho = rho0 * (1.0 + field(amp_rho))
    p = p0 * (1.0 + field(amp_p))
    u = [field(amp_u) for _ in range(D)]
    return prim_to_state(cfg, rho, u, p)


def white_random(cfg, seed, rho0=1.0, p0=1.0, amp=0.1):
    rng = np.random.default_rng(seed)
    shape = grid_shape(cfg)
    D = cfg["dim"]
    rho = rho0 * (1.0 + amp * rng.uniform(-1, 1, shape))
    p = p0 * (1.0 + amp * rng.uniform(-1, 1, shape))
    u = [amp * rng.uniform(-1, 1, shape) for _ in range(D)]
    return prim_to_state(cfg, rho, u, p)
