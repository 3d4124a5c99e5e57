// ars_dev.h -- device-side building blocks of the all-regime, well-balanced
// step (arXiv 1903.09043, Sec. 2) for gfx950, shared by the fused kernels,
// the phase-by-phase reference kernels, the batched kernel and the adjoint.
//
// Every function fixes one expression tree (operation order; the library is
// built with -ffp-contract=on, which fuses a multiply and an add only inside
// one expression) so that all GPU paths produce the same bits.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ars {

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_OUTFLOW = 2 };
enum { TH_ADIABATIC = 0, TH_FIXED = 1 };

// Scalar problem constants, derived once on the host.
struct Params {
  int dim;              // 2 or 3
  int nx, ny, nz;       // lateral x, lateral y (1 in 2D), vertical (gravity axis)
  int bcx[2], bcy[2], bcz[2];
  long long ncell;
  double dx[3], idx[3], qidx[3];  // per physical axis (x, y, z); 2D uses [0],[2]
  double gamma, gm1, g, K, hK, cfl, mu, kappa, eta, dmax, sumidx2;  // hK = 0.5 / K
  double Tw2[2];        // 2 T_wall (bottom, top)
  int thermal[2];
  int noslip;
  int dt_mode;
  int low_mach;
  int diss;             // mu > 0 || kappa > 0
  int nc;               // 1: non-conservative energy scheme (App. B)
};

// Workspace control block (first 256 bytes of the workspace).
struct Control {
  unsigned long long lammax[4];   // max rate slots (FP64 bits; rates are >= 0)
  unsigned long long fault_cell;  // min faulting cell (ULLONG_MAX = none)
  unsigned int fault;             // latched flag
  unsigned int pad0;
  double t_scratch;
  unsigned long long pad1[25];
};

#ifndef ARS_FASTMATH
#define ARS_FASTMATH 1
#endif

// Reciprocal and reciprocal square root to about one ulp: the hardware
// estimates (v_rcp_f64 / v_rsq_f64, good to about 2^-23) refined by two
// Newton-Raphson steps each (quadratic convergence), a third of the
// instructions of the correctly rounded division and square root the
// compiler expands.  Every GPU path calls these same functions, so all of
// them round alike.
__device__ __forceinline__ double rcp_nr(double x) {
#if ARS_FASTMATH
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
#else
  return 1.0 / x;
#endif
}
__device__ __forceinline__ double rsq_nr(double x) {
#if ARS_FASTMATH
  double y = __builtin_amdgcn_rsq(x);
  double t = x * y;
  double e = __builtin_fma(-t, y, 1.0);  // 1 - x y^2
  y = __builtin_fma(0.5 * y, e, y);
  t = x * y;
  e = __builtin_fma(-t, y, 1.0);
  return __builtin_fma(0.5 * y, e, y);
#else
  return 1.0 / sqrt(x);
#endif
}

__device__ __forceinline__ double dmax2(double a, double b) { return a >= b ? a : b; }
__device__ __forceinline__ double dmin2(double a, double b) { return a <= b ? a : b; }

// Gravitational potential at the centre of the cell with vertical index kz
// (Phi = g z, z = (kz + 1/2) dz); every Delta Phi is a difference of two such
// values.
__device__ __forceinline__ double phi_at(const Params& P, int kz) {
  return P.g * (((double)kz + 0.5) * P.dx[2]);
}

// Primitive values of one cell (Sec. 4 ideal gas; R = 1 so T = p / rho).
template <int DIM>
struct Prim {
  double rho, r, u[DIM], p, c, rc, T;
  double ic, irc;  // 1/c, 1/(rho c)
};

// Conservative -> primitive (b = rho, m_0..m_{DIM-1}, E).
template <int DIM>
__device__ __forceinline__ Prim<DIM> cons_to_prim(const Params& P, const double* b) {
  Prim<DIM> q;
  q.rho = b[0];
  q.r = rcp_nr(q.rho);
#pragma unroll
  for (int k = 0; k < DIM; ++k) q.u[k] = b[1 + k] * q.r;
  double kin = b[1] * q.u[0];
#pragma unroll
  for (int k = 1; k < DIM; ++k) kin = kin + b[1 + k] * q.u[k];
  kin = 0.5 * kin;
  q.p = P.gm1 * (b[DIM + 1] - kin);
  const double c2 = (P.gamma * q.p) * q.r;  // c^2 = gamma p / rho
  q.ic = rsq_nr(c2);
  q.c = c2 * q.ic;
  q.rc = q.rho * q.c;
  q.T = q.p * q.r;
  q.irc = q.r * q.ic;
  return q;
}

// Wall ghost from the adjacent interior cell (Sec. 4.3 hydrostatic
// extrapolation through eq. well_balanced_formula solved for the ghost
// density; reflexive velocity; ghost temperature 2 T_wall - T for a fixed-T
// wall, T for an adiabatic one).  delta = Phi_ghost - Phi_interior.
template <int DIM>
__device__ __forceinline__ Prim<DIM> wall_ghost(const Params& P, const Prim<DIM>& in, int side, double delta) {
  Prim<DIM> g;
  const double Ti = in.T;
  const double Tg = (P.thermal[side] == TH_FIXED) ? P.Tw2[side] - Ti : Ti;
  const double hd = 0.5 * delta;
  g.rho = (in.rho * (Ti - hd)) / (Tg + hd);
  g.r = rcp_nr(g.rho);
  g.p = g.rho * Tg;
  g.T = Tg;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const bool flip = P.noslip ? true : (k == DIM - 1);
    g.u[k] = flip ? -in.u[k] : in.u[k];
  }
  const double c2 = (P.gamma * g.p) * g.r;
  g.ic = rsq_nr(c2);
  g.c = c2 * g.ic;
  g.rc = g.rho * g.c;
  g.irc = g.r * g.ic;
  return g;
}

// Acoustic interface solver (Sec. 2.1.2 + eq. low_mach_correction) between L
// and R along a LATERAL axis (no gravity source).  a = K max(rho c);
// 1/(2a) = (0.5/K) min(1/(rho c)) and 1/max(c) = min(1/c), so the face needs
// no division.  Outputs u*, Pi*, P = Pi* u*.
template <bool LM>
__device__ __forceinline__ void face_lat(const Params& P, double rcL, double ircL, double icL, double pL, double uL,
                                         double rcR, double ircR, double icR, double pR, double uR, double& ustar,
                                         double& pistar, double& Pf) {
  const double a = P.K * dmax2(rcL, rcR);
  ustar = 0.5 * (uL + uR) - (pR - pL) * (P.hK * dmin2(ircL, ircR));
  double theta = 1.0;
  if (LM) {
    const double Ma = fabs(ustar) * dmin2(icL, icR);
    theta = dmin2(Ma, 1.0);
  }
  pistar = 0.5 * (pL + pR) - ((0.5 * a) * theta) * (uR - uL);
  Pf = pistar * ustar;
}

// Same along the vertical (gravity) axis, with the interface source
// S_{i+1/2} = -(rho_L + rho_R)/2 (Phi_R - Phi_L); at a wall face u* = 0.
template <bool LM, int DIM>
__device__ __forceinline__ void face_vert(const Params& P, const Prim<DIM>& L, const Prim<DIM>& R, double dphi,
                                          bool wall, double& ustar, double& pistar, double& Pf, double& S) {
  constexpr int Z = DIM - 1;
  const double a = P.K * dmax2(L.rc, R.rc);
  S = (-0.5 * (L.rho + R.rho)) * dphi;
  ustar = wall ? 0.0 : 0.5 * (L.u[Z] + R.u[Z]) - ((R.p - L.p) - S) * (P.hK * dmin2(L.irc, R.irc));
  double theta = 1.0;
  if (LM) {
    const double Ma = fabs(ustar) * dmin2(L.ic, R.ic);
    theta = dmin2(Ma, 1.0);
  }
  pistar = 0.5 * (L.p + R.p) - ((0.5 * a) * theta) * (R.u[Z] - L.u[Z]);
  Pf = pistar * ustar;
}

// Largest local rate of a cell for the CFL reduction (time-step kernel):
// sum_d (|u_d| + c)/dx_d, plus 2 D sum_d dx_d^-2 with D = dmax / rho when
// dt_mode == 0; dt_mode 1 drops the diffusive part, dt_mode 2 (for the
// IMEX step, whose acoustic part is implicit) the sound speed.  Non-finite
// rates count as +inf.
template <int DIM>
__device__ __forceinline__ double cell_rate(const Params& P, const Prim<DIM>& q) {
  const double cs = (P.dt_mode == 2) ? 0.0 : q.c;  // dt_mode 2 (IMEX step): no sound speed
  double h = (fabs(q.u[0]) + cs) * P.idx[0];
  if (DIM == 3) h = h + (fabs(q.u[1]) + cs) * P.idx[1];
  h = h + (fabs(q.u[DIM - 1]) + cs) * P.idx[2];
  double l = h;
  if (P.dt_mode != 1) l = h + (2.0 * (P.dmax * q.r)) * P.sumidx2;
  if (!(l < __builtin_huge_val())) l = __builtin_huge_val();
  return l;
}

// Periodic wrap / outflow clamp of a lateral index r along an axis of n cells.
__device__ __forceinline__ int resolve_lat(int r, int n, const int* bc) {
  if (r >= 0 && r < n) return r;
  if (bc[0] == BC_PERIODIC) {
    int m = r % n;
    return m < 0 ? m + n : m;
  }
  return r < 0 ? 0 : n - 1;
}

__device__ __forceinline__ void atomic_max_rate(unsigned long long* slot, double v) {
  atomicMax(slot, (unsigned long long)__double_as_longlong(v));
}

}  // namespace ars
