"""Problem set-ups of the paper's convection and low-Mach tests, as plain
configuration dicts (the same keys as the public ``ars_config`` struct).

Nothing here is the method's arithmetic: these are the inputs (grid, gas,
boundary conditions, transport coefficients, initial-state parameters) of
Sec. 4 of arXiv 1903.09043 at the sizes this library is measured on.

Rayleigh and Prandtl numbers are turned into constant dynamic viscosity and
conductivity with the Boussinesq-type reading used throughout: the
super-adiabatic temperature drop over the layer, expansion coefficient
1/T and density taken at mid-depth (the paper never defines Ra; Sec. 4.5).
"""
import math

BC_PERIODIC, BC_WALL, BC_OUTFLOW = 0, 1, 2
TH_ADIABATIC, TH_FIXED = 0, 1
PROB_UNIFORM, PROB_RB, PROB_GRESHO, PROB_SOD, PROB_ISOTHERMAL = 0, 1, 2, 3, 4

GAMMA = 5.0 / 3.0


def ra_pr_to_mu_kappa(Ra, Pr, T_bottom=1.0, T_top=0.5, g=1.0, depth=1.0, gamma=GAMMA):
    """(mu, kappa) for a layer of ideal gas (R = 1) heated from below.

    chi = sqrt(g alpha dT_sa depth^3 / (Ra Pr)), nu = Pr chi,
    mu = rho_mid nu, kappa = rho_mid c_p chi, with c_p = gamma / (gamma - 1),
    dT_sa = (T_bottom - T_top) - g depth / c_p, alpha = 1 / T_mid and rho_mid
    the polytropic density at mid-depth (bottom density 1).
    Works with python floats or torch scalars (for gradients)."""
    cp = gamma / (gamma - 1.0)
    dT = T_bottom - T_top
    dT_sa = dT - g * depth / cp
    T_mid = 0.5 * (T_bottom + T_top)
    m = g * depth / dT - 1.0
    rho_mid = (T_mid / T_bottom) ** m
    alpha = 1.0 / T_mid
    chi = (g * alpha * dT_sa * depth ** 3 / (Ra * Pr)) ** 0.5
    return rho_mid * Pr * chi, rho_mid * cp * chi


def rb(n, L, Ra=1e4, Pr=1.0, low_mach=1, seed=0, amp=1e-4, T_bottom=1.0, T_top=0.5, g=1.0,
       cfl=0.4, K=1.1, dt_mode=0):
    """Rayleigh-Benard layer: periodic horizontally, no-slip fixed-T walls at
    the bottom/top of the last axis, linear-T hydrostatic base (the m = 1
    polytrope for the default temperatures), seeded temperature noise."""
    dim = len(n)
    mu, kappa = ra_pr_to_mu_kappa(Ra, Pr, T_bottom, T_top, g, L[-1])
    bc = [[BC_PERIODIC, BC_PERIODIC] for _ in range(dim - 1)] + [[BC_WALL, BC_WALL]]
    cfg = dict(dim=dim, n=list(n), L=list(L), gamma=GAMMA, g=g, mu=mu, kappa=kappa, K=K, cfl=cfl,
               low_mach=int(low_mach), dt_mode=dt_mode, bc=bc, wall_noslip=1,
               thermal=[TH_FIXED, TH_FIXED], T_wall=[T_bottom, T_top])
    return cfg, PROB_RB, [T_bottom, T_top, -1.0, amp], seed


def gresho(n=1024, Ma=1e-3, low_mach=1, cfl=0.4, K=1.1):
    cfg = dict(dim=2, n=[n, n], L=[1.0, 1.0], gamma=GAMMA, g=0.0, mu=0.0, kappa=0.0, K=K, cfl=cfl,
               low_mach=int(low_mach), dt_mode=0, bc=[[BC_PERIODIC, BC_PERIODIC]] * 2, wall_noslip=1,
               thermal=[TH_ADIABATIC, TH_ADIABATIC], T_wall=[1.0, 1.0])
    return cfg, PROB_GRESHO, [Ma], 0


def rb2d_64x32(low_mach=1):
    """2D RB 64x32 on [0,2]x[0,1], Ra = 1e4, Pr = 1, 1000 steps."""
    return rb([64, 32], [2.0, 1.0], Ra=1e4, low_mach=low_mach)


def rb3d_ra1e6(n=256):
    """3D RB 256^3 on the unit cube, Ra = 1e6, Pr = 1, 2000 steps, forward only."""
    return rb([n, n, n], [1.0, 1.0, 1.0], Ra=1e6)


def gresho_1024(low_mach=1, n=1024):
    """2D Gresho vortex 1024^2, Ma = 1e-3, 5000 steps, theta on and off."""
    return gresho(n=n, Ma=1e-3, low_mach=low_mach)


def rb3d_ra1e5(n=128):
    """3D RB 128^3, Ra = 1e5, Pr = 1: adjoint over 200 steps, 16 snapshots."""
    return rb([n, n, n], [1.0, 1.0, 1.0], Ra=1e5)


def rb2d_weak(n=32, Ra=2000.0, low_mach=1, chi=1.1, m=1.3, Pr=1.0, amp=1e-4, seed=1):
    """The 2D onset runs of Sec. 4.5: weak stratification chi = 1.1 and
    m = 1.3 (close to the adiabatic gradient), so the convective flows are
    slow.  Box [0, 2] x [0, 1] with 2n x n cells (the paper gives 128^2 and
    no box), fixed-T walls (the paper imposes the heat flux at the bottom, a
    wall kind this library does not have), seeded temperature noise (the
    paper starts near the fundamental velocity mode).  T_top / T_bottom =
    chi^(-1/m), g = (m + 1)(T_bottom - T_top)."""
    T_top = chi ** (-1.0 / m)
    g = (m + 1.0) * (1.0 - T_top)
    return rb([2 * n, n], [2.0, 1.0], Ra=Ra, Pr=Pr, low_mach=low_mach, seed=seed, amp=amp, T_bottom=1.0,
              T_top=T_top, g=g)


def rb3d_weak(n=64, low_mach=1, chi=1.1, m=0.1, Ra=6.5e5, Pr=1.0, amp=1e-3, seed=0):
    """The 3D convection run of Sec. 4.5 whose middle-plane kinetic-energy
    spectrum the paper shows: polytropic index m = 0.1, Ra = 6.5e5, fixed-T
    walls, unit cube, periodic x/y.  The paper calls the stratification
    weak but gives no density ratio for 3D; the 2D weak case's chi = 1.1 is
    taken: T_top / T_bottom = chi^(-1/m) and g = (m + 1)(T_bottom - T_top)
    (R = 1, unit depth), so that the linear-T base is the m polytrope with
    that density ratio.  Pr (not given) = 1."""
    T_top = chi ** (-1.0 / m)
    g = (m + 1.0) * (1.0 - T_top)
    return rb([n, n, n], [1.0, 1.0, 1.0], Ra=Ra, Pr=Pr, low_mach=low_mach, seed=seed, amp=amp, T_bottom=1.0,
              T_top=T_top, g=g)


def splitmix64(state):
    """One SplitMix64 step (published definition); returns (new_state, out)."""
    M = (1 << 64) - 1
    state = (state + 0x9E3779B97F4A7C15) & M
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return state, z ^ (z >> 31)


def rb2d_batch(n_inst=512, seed=1000):
    """Batched 2D RB: sizes uniform over {64x32, 128x64, 256x128} on
    [0,2]x[0,1], Ra log-uniform in [5e2, 5e3], Pr = 1, per-instance seeds
    SplitMix64(seed + k).  Returns a list of (cfg, problem, params, seed)."""
    sizes = [(64, 32), (128, 64), (256, 128)]
    out = []
    for k in range(n_inst):
        s, a = splitmix64(seed + k)
        s, b = splitmix64(s)
        u0 = (a >> 11) * 2.0 ** -53
        u1 = (b >> 11) * 2.0 ** -53
        nx, ny = sizes[min(int(3 * u0), 2)]
        Ra = math.exp(math.log(5e2) + u1 * math.log(10.0))
        out.append(rb([nx, ny], [2.0, 1.0], Ra=Ra, seed=a))
    return out
