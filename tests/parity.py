"""Acceptance measure for comparing a GPU state with the oracle's state.

Cell-wise, per conserved variable v:

    |g - o| <= tol * max(|o|, s_v)

with s_v the magnitude scale of that variable over the whole grid:

* density and total energy: s_v = max |o_v|;
* every momentum component: s_m = max(max |o_m|, max rho c), the momentum of
  a flow at unit Mach number.

Why the momentum takes the acoustic scale: its update in eq.
(all_regime_scheme) is the difference of the interface pressures Pi* of
Sec. 2.1.2 (magnitude p = rho c^2 / gamma) minus the gravity source S-bar,
and at hydrostatic equilibrium the two cancel exactly (the well-balanced
property, Sec. 2.1.5); for low-Mach flows they nearly cancel (Sec. 2.1.6).
The momentum of a near-rest or low-Mach state is therefore a small residual
of O(p) terms, and two evaluations of the same formulas that round
differently (quotients in the oracle, reciprocal products in the kernels)
differ by about eps * lambda * p per step in the momentum, however small the
flow is.  Measured against the flow's own largest momentum (1e-6 in the
Rayleigh-Benard runs that start at rest with a 1e-4 temperature
perturbation) that difference reads 1e-10; measured against rho c it is the
1e-16 that FP64 can carry.  ``strict_err`` reports the first figure too.
"""
import numpy as np


def _pressure_and_rhoc(cfg, o):
    D = cfg["dim"]
    rho = o[0]
    kin = 0.5 * sum(o[1 + k] * o[1 + k] for k in range(D)) / rho
    p = (cfg["gamma"] - 1.0) * (o[D + 1] - kin)
    return p, np.sqrt(cfg["gamma"] * np.abs(p) * rho)


def scales(cfg, o):
    """s_v for every variable of the oracle state ``o`` (shape (NV, ...))."""
    o = np.asarray(o)
    D = cfg["dim"]
    s = np.max(np.abs(o.reshape(o.shape[0], -1)), axis=1)
    _, rc = _pressure_and_rhoc(cfg, o)
    rcmax = float(np.max(rc))
    for k in range(D):
        s[1 + k] = max(s[1 + k], rcmax)
    return np.maximum(s, np.finfo(np.float64).tiny)


def rel_err(cfg, g, o):
    """Largest cell-wise |g - o| / max(|o|, s_v) over the state."""
    g = np.asarray(g)
    o = np.asarray(o)
    assert g.shape == o.shape
    s = scales(cfg, o).reshape((-1,) + (1,) * (o.ndim - 1))
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), s)))


def strict_err(g, o):
    """The same with s_v = max |o_v| for every variable (reported only)."""
    g = np.asarray(g)
    o = np.asarray(o)
    s = np.max(np.abs(o.reshape(o.shape[0], -1)), axis=1)
    s = np.maximum(s, np.finfo(np.float64).tiny).reshape((-1,) + (1,) * (o.ndim - 1))
    return float(np.max(np.abs(g - o) / np.maximum(np.abs(o), s)))
