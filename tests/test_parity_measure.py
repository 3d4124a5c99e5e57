"""The acceptance measure of tests/parity.py on constructed states (CPU)."""
import numpy as np

from tests import parity as P


def _cfg():
    return dict(dim=2, gamma=5.0 / 3.0)


def _state(m_amp):
    rng = np.random.default_rng(0)
    rho = 1.0 + 0.1 * rng.random((6, 5))
    m = m_amp * rng.standard_normal((2, 6, 5))
    p = np.ones((6, 5))
    E = p / (2.0 / 3.0) + 0.5 * (m[0] ** 2 + m[1] ** 2) / rho
    return np.stack([rho, m[0], m[1], E])


def test_momentum_on_acoustic_scale():
    """A near-rest state: a 1e-15 momentum difference is 1e-15 of rho c on
    the parity measure but 1e-9 of the flow's own largest momentum."""
    o = _state(1e-6)
    g = o.copy()
    g[1, 2, 3] += 1e-15
    rc = np.sqrt(5.0 / 3.0 * 1.0 * o[0])
    assert abs(P.rel_err(_cfg(), g, o) - 1e-15 / rc.max()) < 1e-18
    assert P.strict_err(g, o) > 1e-10


def test_fast_flow_uses_own_scale():
    """Where the flow's momentum exceeds rho c its own maximum is the scale."""
    o = _state(10.0)
    g = o.copy()
    g[2, 1, 1] += 1e-12
    s = np.max(np.abs(o[2]))
    assert s > np.max(np.sqrt(5.0 / 3.0 * o[0]))
    want = 1e-12 / max(abs(o[2, 1, 1]), s)
    assert abs(P.rel_err(_cfg(), g, o) - want) < 1e-3 * want


def test_density_and_energy_errors_detected():
    o = _state(1e-6)
    for v in (0, 3):
        g = o.copy()
        g[v, 0, 0] *= 1.0 + 1e-11
        assert P.rel_err(_cfg(), g, o) > 5e-12
