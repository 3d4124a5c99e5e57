// ars_imex.hip -- implicit acoustic (IMEX) step of the all-regime scheme:
// the further work the paper names in its Conclusion (solve the acoustic
// part implicitly to lift the acoustic CFL condition, keeping the
// well-balanced gravity source).  The paper prints no scheme; the reading:
// Sec. 2.1.2's acoustic step with its interface values taken at the END of
// the step (backward Euler on the linear relaxation system at frozen
// a, S, theta of t^n).  Unknowns per interior cell i: Pi_i and the normal
// velocities u_{d,i}; with lambda_d = dt / dx_d,
//   u*_j  = (u_L + u_R)/2 - (Pi_R - Pi_L - S_j) / (2 a_j)       (0 at walls)
//   Pi*_j = (Pi_L + Pi_R)/2 - (a_j theta_j / 2)(u^n_R - u^n_L)
//   u_{d,i} = u^n_{d,i} - lambda_d tau_i ([Pi*]_{d,i} - S-bar_{d,i})
//   Pi_i    = p_i - rho_i c_i^2 sum_d lambda_d [u*]_{d,i}
// (the pressure row is the Lagrangian update linearised through the
// equation of state; the acoustic dissipation of Pi* acts on u^n, so the
// velocity rows are explicit in Pi and u is eliminated: the system is for
// Pi alone, its rows scaled by 1 / (rho c^2)).  Ghost cells take the boundary rules of the explicit
// step applied to the unknowns (periodic images, outflow copies; at walls
// Pi_g = Pi_i + (p_g - p_i)^n and the reflected velocity).  The implicit
// (u*, Pi*) then replace the explicit ones in the acoustic cell values,
// the transport, the update and the relaxation, which are the explicit
// step's (the dissipative fluxes stay explicit).
//
// GPU layout: the reference step's padded workspace (primitives, explicit
// faces for a, S, theta, then the implicit faces, L, b~, fluxes), padded
// extensions of Pi and of the velocities it gives, and the vectors of an
// unpreconditioned Krylov solver on the N unknowns Pi: conjugate gradients
// when every axis is periodic or walled at both ends (the operator is then
// symmetric positive definite), BiCGSTAB otherwise (outflow).  The operator is applied
// matrix-free: one kernel extends Pi to the ghost cells, one forms the
// velocities of every padded cell from the Pi* of its two faces per axis
// (ghosts by the boundary rules), one forms every row from the u* of the
// two faces of each axis.  Dot products are two-level reductions in a
// fixed order (deterministic); the iteration's scalars stay on the device
// and the host reads the residual norm every few iterations.
#include <hip/hip_runtime.h>

#include <cmath>
#include <vector>

#include "../../include/ars.h"
#include "ars_dev.h"
#include "ars_internal.h"
#include "ars_ref.h"

namespace ars {

namespace {

constexpr int DOT_BLOCKS = 1024;
constexpr int CG_BLOCKS = 1024;  // blocks of the CG kernels (<= the partial-sum slots)
constexpr int BS = 256;
constexpr int CG_CHECK = 16;  // CG iterations between host reads of the residual
// scalar slots of the iteration
enum { SC_RHO_OLD = 0, SC_ALPHA, SC_OMEGA, SC_RHO_NEW, SC_RV, SC_TS, SC_TT, SC_RR, SC_BB,
       SC_CG_RR,      // (r, r) of CG iterations 0, 2, 4, ... (SC_CG_RR + 1: 1, 3, 5, ...)
       SC_CG_CHK = 11, SC_N = 16 };

struct ImexLayout {
  RefGrid G;
  long long n;      // unknowns: Pi of every interior cell
  double* W;        // reference workspace
  double* ext;      // (D + 1) padded fields: Pi, u_0..u_{D-1}
  double* x;        // solution
  double* r;
  double* rh;       // shadow residual
  double* p;
  double* v;
  double* sv;
  double* t;
  double* b;
  double* r2;       // CG, 2D: the second residual and product of the ping-pong
  double* q2;
  double* part;     // partial sums (one per block of a reduction; CG: up to two sets of four)
  double* sc;       // scalars
};

ImexLayout layout_of(const Params& P, void* work) {
  ImexLayout L;
  L.G = make_grid(P);
  const int D = P.dim;
  L.n = P.ncell;
  char* w = (char*)work;
  size_t off = 0;
  auto take = [&](size_t count) {
    double* q = (double*)(w + off);
    off += ((count * sizeof(double) + 255) / 256) * 256;
    return q;
  };
  L.W = take((size_t)R_NFIELD * L.G.npad);
  L.ext = take((size_t)(D + 1) * L.G.npad);
  L.x = take(L.n);
  L.r = take(L.n);
  L.rh = take(L.n);
  L.p = take(L.n);
  L.v = take(L.n);
  L.sv = take(L.n);
  L.t = take(L.n);
  L.b = take(L.n);
  L.r2 = take(L.n);
  L.q2 = take(L.n);
  L.part = take(8 * (CG_BLOCKS > DOT_BLOCKS ? CG_BLOCKS : DOT_BLOCKS));
  L.sc = take(SC_N);
  return L;
}

__device__ __forceinline__ int comp_axis(int DIM, int a) { return a == 2 ? DIM - 1 : a; }

// Interior source cell of a padded cell (periodic image, outflow copy, or
// the interior neighbour of a wall ghost: wall = 0 bottom, 1 top, -1 none).
template <int DIM>
__device__ __forceinline__ void source_cell(const Params& P, int qx, int qy, int qz, int& cx, int& cy, int& kz,
                                            int& wall) {
  cx = resolve_lat(qx - 2, P.nx, P.bcx);
  cy = (DIM == 3) ? resolve_lat(qy - 2, P.ny, P.bcy) : 0;
  kz = qz - 2;
  wall = -1;
  if (kz < 0 || kz >= P.nz) {
    const int side = kz < 0 ? 0 : 1;
    if (P.bcz[side] == BC_WALL) {
      wall = side;
      kz = side == 0 ? 0 : P.nz - 1;
    } else {
      kz = resolve_lat(kz, P.nz, P.bcz);
    }
  }
}

// Padded extension of Pi (cst: with the wall ghosts' hydrostatic offset).
template <int DIM>
__global__ void k_schur_extP(Params P, RefGrid G, const double* __restrict__ W, const double* __restrict__ x, int cst,
                             double* __restrict__ ext) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.npad) return;
  int qx, qy, qz, cx, cy, kz, wall;
  decode(G, i, qx, qy, qz);
  source_cell<DIM>(P, qx, qy, qz, cx, cy, kz, wall);
  const long long n = G.npad;
  double Pi = x[cx + (long long)P.nx * (cy + (long long)P.ny * kz)];
  if (wall >= 0 && cst) {
    const long long qi = G.pad(qx, qy, wall == 0 ? 2 : P.nz + 1);
    Pi = Pi + (W[R_P * n + i] - W[R_P * n + qi]);
  }
  ext[i] = Pi;
}

// Acoustic dissipation term of Pi* on face (a, l | l + e_a), on the
// velocities of t^n: (a_j theta_j / 2)(u^n_R - u^n_L).
template <int DIM, bool LM>
__device__ __forceinline__ double dissip_n(const Params& P, const RefGrid& G, const double* __restrict__ W,
                                           long long l, int a) {
  const long long n = G.npad;
  const long long r = l + astride(G, a);
  const double am = P.K * dmax2(W[R_RC * n + l], W[R_RC * n + r]);
  double theta = 1.0;
  if (LM) {
    const double use = W[(R_FACE + 4 * a) * n + l];  // explicit u* of t^n
    theta = dmin2(fabs(use) * dmin2(W[R_IC * n + l], W[R_IC * n + r]), 1.0);
  }
  const int uf = ufield(DIM, a == 2 ? DIM - 1 : a);
  return ((0.5 * am) * theta) * (W[uf * n + r] - W[uf * n + l]);
}

// Velocities of every padded cell from Pi (its source cell's velocity
// rows, then the ghost rule): u = cst u^n - lambda tau ([Pi*] - cst S-bar).
template <int DIM, bool LM>
__global__ void k_schur_u(Params P, RefGrid G, const double* __restrict__ W, const double* __restrict__ d_dt, int cst,
                          double* __restrict__ ext) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.npad) return;
  int qx, qy, qz, cx, cy, kz, wall;
  decode(G, i, qx, qy, qz);
  source_cell<DIM>(P, qx, qy, qz, cx, cy, kz, wall);
  const long long n = G.npad;
  const long long q = G.pad(cx + 2, DIM == 3 ? cy + 2 : 0, kz + 2);  // padded index of the source cell
  const double dt = *d_dt;
  const int axes[3] = {0, DIM == 3 ? 1 : 2, 2};
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    const int a = axes[t];
    const long long e = astride(G, a);
    double pp = 0.5 * (ext[q] + ext[q + e]);
    double pm = 0.5 * (ext[q - e] + ext[q]);
    double dpi;
    if (cst) {
      pp = pp - dissip_n<DIM, LM>(P, G, W, q, a);
      pm = pm - dissip_n<DIM, LM>(P, G, W, q - e, a);
      dpi = pp - pm;
      if (a == 2) dpi = dpi - 0.5 * (W[(R_FACE + 4 * a + 3) * n + q] + W[(R_FACE + 4 * a + 3) * n + q - e]);
    } else {
      dpi = pp - pm;
    }
    const int k = comp_axis(DIM, a);
    double u = (cst ? W[ufield(DIM, k) * n + q] : 0.0) - ((dt / P.dx[a]) * W[R_R * n + q]) * dpi;
    if (wall >= 0 && (P.noslip || k == DIM - 1)) u = -u;
    ext[(1 + k) * n + i] = u;
  }
}

// Implicit u* of face (a, l | l + e_a) from the extensions.
template <int DIM>
__device__ __forceinline__ double ustar_imp(const Params& P, const RefGrid& G, const double* __restrict__ W,
                                            const double* __restrict__ ext, long long l, int lz, int a, int cst) {
  if (ref_wall(P, a, lz)) return 0.0;
  const long long n = G.npad;
  const long long r = l + astride(G, a);
  const int k = comp_axis(DIM, a);
  const double h2a = P.hK * dmin2(W[R_IRC * n + l], W[R_IRC * n + r]);  // 1 / (2a)
  const double S = (a == 2 && cst) ? W[(R_FACE + 4 * a + 3) * n + l] : 0.0;
  return 0.5 * (ext[(1 + k) * n + l] + ext[(1 + k) * n + r]) - ((ext[r] - ext[l]) - S) * h2a;
}

// Rows of the system for Pi at every interior cell, scaled by 1/(rho c^2):
// y = (Pi - cst p) / (rho c^2) + sum_d lambda_d [u*]_d.
template <int DIM>
__global__ void k_schur_rows(Params P, RefGrid G, const double* __restrict__ W, const double* __restrict__ ext,
                             const double* __restrict__ d_dt, const double* __restrict__ x, int cst,
                             double* __restrict__ y) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  const int cxx = (int)(c % P.nx);
  const long long rr = c / P.nx;
  const int cyy = (int)(rr % P.ny);
  const int czz = (int)(rr / P.ny);
  const long long q = G.pad(cxx + 2, DIM == 3 ? cyy + 2 : 0, czz + 2);
  const long long n = G.npad;
  const double dt = *d_dt;
  const int axes[3] = {0, DIM == 3 ? 1 : 2, 2};
  double div = 0.0;
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    const int a = axes[t];
    const double usp = ustar_imp<DIM>(P, G, W, ext, q, czz + 2, a, cst);
    const double usm = ustar_imp<DIM>(P, G, W, ext, q - astride(G, a), czz + 2 - (a == 2), a, cst);
    div = div + (dt / P.dx[a]) * (usp - usm);
  }
  const double rc2 = W[R_RC * n + q] * W[R_C * n + q];  // rho c^2
  y[c] = (x[c] - (cst ? W[R_P * n + q] : 0.0)) / rc2 + div;
}

// Implicit faces of every padded face into the workspace (u*, Pi*, Pi* u*;
// S untouched); every thread reads only its own faces' explicit u* (for
// theta) before overwriting them.
template <int DIM, bool LM>
__global__ void k_imex_faces(Params P, RefGrid G, double* __restrict__ W, const double* __restrict__ ext) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.npad) return;
  int qx, qy, qz;
  decode(G, i, qx, qy, qz);
  const long long n = G.npad;
  const int axes[3] = {0, DIM == 3 ? 1 : 2, 2};
  double us[3], pi[3];
  bool has[3];
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    const int a = axes[t];
    const int qa = a == 0 ? qx : (a == 1 ? qy : qz);
    const int Pa = a == 0 ? G.Px : (a == 1 ? G.Py : G.Pz);
    has[t] = qa + 1 < Pa;
    us[t] = pi[t] = 0.0;
    if (has[t]) {
      us[t] = ustar_imp<DIM>(P, G, W, ext, i, qz, a, 1);
      pi[t] = 0.5 * (ext[i] + ext[i + astride(G, a)]) - dissip_n<DIM, LM>(P, G, W, i, a);
    }
  }
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    if (!has[t]) continue;
    const int f = R_FACE + 4 * axes[t];
    W[(f + 0) * n + i] = us[t];
    W[(f + 1) * n + i] = pi[t];
    W[(f + 2) * n + i] = pi[t] * us[t];
  }
}

// Acoustic cell values L, S-bar, b~ (Sec. 2.1.2) from the stored faces.
template <int DIM>
__global__ void k_imex_cell(Params P, RefGrid G, const double* __restrict__ d_dt, double* __restrict__ W) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.npad) return;
  constexpr int NV = DIM + 2;
  int qx, qy, qz;
  decode(G, i, qx, qy, qz);
  const bool cell = qx >= 1 && qx < G.Px - 1 && qz >= 1 && qz < G.Pz - 1 && (DIM == 2 || (qy >= 1 && qy < G.Py - 1));
  if (!cell) return;
  const long long n = G.npad;
  const double dt = *d_dt;
  const int axes[3] = {0, DIM == 3 ? 1 : 2, 2};
  double Lc = 1.0, Am[3], AE = 0.0;
  const long long sz = astride(G, 2);
  const double sb = 0.5 * (W[(R_FACE + 4 * 2 + 3) * n + i] + W[(R_FACE + 4 * 2 + 3) * n + i - sz]);
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    const int a = axes[t];
    const int f = R_FACE + 4 * a;
    const long long m = i - astride(G, a);
    const double lam = dt / P.dx[a];
    Lc = Lc + lam * (W[f * n + i] - W[f * n + m]);
    double dpi = W[(f + 1) * n + i] - W[(f + 1) * n + m];
    if (a == 2) dpi = dpi - sb;
    Am[t] = lam * dpi;
    const double term = lam * (W[(f + 2) * n + i] - W[(f + 2) * n + m]);
    AE = (t == 0) ? term : AE + term;
  }
  const double rho = W[R_CONS * n + i];
  const double calE = W[(R_CONS + NV - 1) * n + i] + rho * phi_at(P, qz - 2);
  const double iL = rcp_nr(Lc);
  W[R_L * n + i] = Lc;
  W[R_SB * n + i] = sb;
  W[R_BT * n + i] = rho * iL;
#pragma unroll
  for (int k = 0; k < DIM; ++k) W[(R_BT + 1 + k) * n + i] = (W[(R_CONS + 1 + k) * n + i] - Am[k]) * iL;
  W[(R_BT + NV - 1) * n + i] = (calE - AE) * iL;
}

// ------------------------------------------------------------ BiCGSTAB ----
__global__ void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b, long long n,
                              double* __restrict__ part) {
  __shared__ double sh[BS];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < n; i += (long long)gridDim.x * BS)
    s = s + a[i] * b[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_dot_final(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[BS];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += BS) s = s + part[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = BS / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = sh[threadIdx.x] + sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// r = b - r (r holds A x on entry); rh = r; p = v = 0; scalars start.
__global__ void k_bicg_start(long long n, const double* __restrict__ b, double* __restrict__ r, double* __restrict__ rh,
                             double* __restrict__ p, double* __restrict__ v, double* __restrict__ sc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    sc[SC_RHO_OLD] = 1.0;
    sc[SC_ALPHA] = 1.0;
    sc[SC_OMEGA] = 1.0;
  }
  if (i >= n) return;
  const double ri = b[i] - r[i];
  r[i] = ri;
  rh[i] = ri;
  p[i] = 0.0;
  v[i] = 0.0;
}

// p = r + beta (p - omega v),  beta = (rho_new / rho_old) (alpha / omega)
__global__ void k_bicg_p(long long n, const double* __restrict__ r, const double* __restrict__ v,
                         double* __restrict__ p, const double* __restrict__ sc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double den = sc[SC_RHO_OLD] * sc[SC_OMEGA];
  const double beta = den != 0.0 ? (sc[SC_RHO_NEW] * sc[SC_ALPHA]) / den : 0.0;
  p[i] = r[i] + beta * (p[i] - sc[SC_OMEGA] * v[i]);
}

// alpha = rho_new / (rh, v), 0 at a breakdown
__device__ __forceinline__ double bicg_alpha(const double* sc) {
  return sc[SC_RV] != 0.0 ? sc[SC_RHO_NEW] / sc[SC_RV] : 0.0;
}

// s = r - alpha v
__global__ void k_bicg_s(long long n, const double* __restrict__ r, const double* __restrict__ v,
                         double* __restrict__ s, double* __restrict__ sc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double alpha = bicg_alpha(sc);
  if (i >= n) return;
  s[i] = r[i] - alpha * v[i];
}

// x += alpha p + omega s;  r = s - omega t;  omega = (t, s) / (t, t)
__global__ void k_bicg_xr(long long n, const double* __restrict__ p, const double* __restrict__ s,
                          const double* __restrict__ t, double* __restrict__ x, double* __restrict__ r,
                          double* __restrict__ sc) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const double alpha = bicg_alpha(sc);
  const double omega = sc[SC_TT] > 0.0 ? sc[SC_TS] / sc[SC_TT] : 0.0;
  if (i < n) {
    x[i] = x[i] + alpha * p[i] + omega * s[i];
    r[i] = s[i] - omega * t[i];
  }
}

// alpha, omega and rho_old of this iteration for the next one's beta (a
// kernel of its own: k_bicg_xr's threads read the previous values)
__global__ void k_bicg_scalars(double* __restrict__ sc) {
  if (threadIdx.x == 0) {
    sc[SC_ALPHA] = bicg_alpha(sc);
    sc[SC_OMEGA] = sc[SC_TT] > 0.0 ? sc[SC_TS] / sc[SC_TT] : 0.0;
    sc[SC_RHO_OLD] = sc[SC_RHO_NEW];
  }
}

// Conjugate gradients (every axis periodic or walled at both ends: the
// eliminated operator is symmetric positive definite, diag(1/(rho c^2)) +
// lambda^2 K^T tau K + lambda G^T (1/(2a)) G with K the central difference
// of the two face averages and G the face difference.  At a wall the ghost
// Pi is the wall cell's, so the wall face's Pi* is that cell's Pi, and the
// wall face's u* is 0; the ghost velocity feeds nothing else, and the
// operator stays symmetric.  Outflow copies make u* at the boundary face
// the edge cell's velocity, which breaks the symmetry: BiCGSTAB there.)
// The operator is a star stencil of radius 2 on the unknowns (neighbour
// indices wrapped on periodic axes, clamped on walled ones).  In 3D an
// iteration is two streaming kernels: (1) p = r + beta p_old and q = A p
// on the fly, with the block sums of (p, q); (2) x += alpha p,
// r -= alpha q, with those of (r, r).  In 2D it is one kernel
// (k_cg_iter_2d, through an LDS tile): the previous iteration's x, r
// updates are done on the fly as well.  Each kernel starts by adding the
// block sums it needs itself, every block in the same fixed order (so every
// block forms the same alpha and beta bit for bit, and no one-block launch
// sits between kernels).  A last-block-arrives reduction would need
// device-scope fences (one per block, an L2 write-back each on a part whose
// XCDs have L2s of their own), which cost far more.

// Coefficients of the homogeneous operator per interior cell: tau, 1/(rho c)
// and 1/(rho c^2) (the rows' scale), out of the padded workspace.
template <int DIM>
__global__ void k_cg_coef(Params P, RefGrid G, const double* __restrict__ W, double* __restrict__ tau,
                          double* __restrict__ irc, double* __restrict__ irc2) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  const int cx = (int)(c % P.nx);
  const long long rr = c / P.nx;
  const int cy = (int)(rr % P.ny);
  const int cz = (int)(rr / P.ny);
  const long long q = G.pad(cx + 2, DIM == 3 ? cy + 2 : 0, cz + 2);
  const long long n = G.npad;
  tau[c] = W[R_R * n + q];
  irc[c] = W[R_IRC * n + q];
  irc2[c] = 1.0 / (W[R_RC * n + q] * W[R_C * n + q]);
}

// Index offsets of the neighbours k - 2, k - 1, k + 1, k + 2 of coordinate
// k on an axis of m >= 2 cells and stride st: periodic images, or on a
// walled axis the nearest interior cell (the ghost Pi is the wall cell's).
__device__ __forceinline__ void nb_offsets(int k, int m, int st, bool wall, int& om2, int& om1, int& op1, int& op2) {
  if (wall) {
    om2 = ((k >= 2 ? k - 2 : 0) - k) * st;
    om1 = ((k >= 1 ? k - 1 : 0) - k) * st;
    op1 = ((k + 1 < m ? k + 1 : m - 1) - k) * st;
    op2 = ((k + 2 < m ? k + 2 : m - 1) - k) * st;
  } else {
    om2 = (k >= 2 ? -2 : m - 2) * st;
    om1 = (k >= 1 ? -1 : m - 1) * st;
    op1 = (k + 1 < m ? 1 : 1 - m) * st;
    op2 = (k + 2 < m ? 2 : 2 - m) * st;
  }
}

// Block sum of s in a fixed order (a butterfly within each wave, then the
// waves' sums in order); every thread gets it.  The caller separates two
// calls with a barrier.
__device__ __forceinline__ double block_sum(double s) {
  __shared__ double sh[BS / 64];
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) s = s + __shfl_xor(s, m, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = sh[0];
#pragma unroll
  for (int w = 1; w < BS / 64; ++w) t = t + sh[w];
  return t;
}

// Sum of a reduction's block sums in a fixed order, in one block (thread 0
// holds it).
__device__ __forceinline__ double sum_parts(const double* __restrict__ part, int nb) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += BS) s = s + part[i];
  return block_sum(s);
}

// beta = (r, r) / (r, r) of the previous iteration (0 in the first) from
// the nb block sums of (r, r); every block adds them in the same order, and
// block 0 keeps this iteration's (r, r) for the next one and for alpha.
__device__ __forceinline__ double cg_beta(const double* __restrict__ part_rr, int nb, double* __restrict__ sc, int it) {
  double beta = 0.0;
  if (it > 0) {
    const double rr = sum_parts(part_rr, nb);
    const double old = sc[SC_CG_RR + ((it - 1) & 1)];
    beta = old != 0.0 ? rr / old : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[SC_CG_RR + (it & 1)] = rr;
    __syncthreads();
  }
  return beta;
}

// Work units of k_cg_apply: a row of x cells (fixed y, z) cut into chunks
// of BS; each block takes a contiguous run of units, and the runs of the
// blocks one XCD receives (blocks go to the XCDs in turn) are contiguous, so
// the rows a row's stencil reaches are mostly read through the same L2.
// Cell indices are 32-bit (the host takes this path below 2^31 cells).
template <int DIM>
__global__ __launch_bounds__(BS) void k_cg_apply(Params P, const double* __restrict__ d_dt, const double* __restrict__ r,
                                                 const double* __restrict__ pold, double* __restrict__ pnew,
                                                 const double* __restrict__ tau, const double* __restrict__ irc,
                                                 const double* __restrict__ irc2, double* __restrict__ q,
                                                 const double* __restrict__ part_rr, int nb_rr,
                                                 double* __restrict__ part_pq, double* __restrict__ sc, int it,
                                                 int wallmask) {
  const double beta = cg_beta(part_rr, nb_rr, sc, it);
  const double dt = *d_dt;
  const int axes[3] = {0, DIM == 3 ? 1 : 2, 2};
  const int ext[3] = {P.nx, P.ny, P.nz};
  const int str[3] = {1, P.nx, P.nx * P.ny};
  double lam[DIM];
#pragma unroll
  for (int t = 0; t < DIM; ++t) lam[t] = dt / P.dx[axes[t]];
  const double hK = P.hK;
  const int nch = (P.nx + BS - 1) / BS;
  const int units = P.ny * P.nz * nch;
  const unsigned G = gridDim.x, b = blockIdx.x;
  const unsigned lw = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int u0 = (int)((long long)units * lw / G), u1 = (int)((long long)units * (lw + 1) / G);
  double s = 0.0;
  for (int u = u0; u < u1; ++u) {
    const int row = u / nch;
    const int cx = (u - row * nch) * BS + (int)threadIdx.x;
    if (cx >= P.nx) continue;
    const int crd[3] = {cx, DIM == 3 ? row % P.ny : 0, DIM == 3 ? row / P.ny : row};
    const int c = row * P.nx + cx;
    const double P0 = r[c] + beta * pold[c];
    const double t0 = tau[c], i0 = irc[c];
    double div = 0.0;
#pragma unroll
    for (int t = 0; t < DIM; ++t) {
      const int a = axes[t];
      const bool wall = (wallmask >> a) & 1;
      int om2, om1, op1, op2;
      nb_offsets(crd[a], ext[a], str[a], wall, om2, om1, op1, op2);
      const double Pm2 = r[c + om2] + beta * pold[c + om2];
      const double Pm1 = r[c + om1] + beta * pold[c + om1];
      const double Pp1 = r[c + op1] + beta * pold[c + op1];
      const double Pp2 = r[c + op2] + beta * pold[c + op2];
      // velocities of the cells c - e, c, c + e: u = -lambda tau [Pi*],
      // [Pi*] = (Pi_{+1} - Pi_{-1}) / 2 of the cell's neighbours
      const double um = -(lam[t] * tau[c + om1]) * (0.5 * (P0 - Pm2));
      const double uc = -(lam[t] * t0) * (0.5 * (Pp1 - Pm1));
      const double up = -(lam[t] * tau[c + op1]) * (0.5 * (Pp2 - P0));
      // u* of the faces c - e | c and c | c + e (0 on a wall face)
      double usm = 0.5 * (um + uc) - (P0 - Pm1) * (hK * dmin2(irc[c + om1], i0));
      double usp = 0.5 * (uc + up) - (Pp1 - P0) * (hK * dmin2(i0, irc[c + op1]));
      if (wall && crd[a] == 0) usm = 0.0;
      if (wall && crd[a] == ext[a] - 1) usp = 0.0;
      div = div + lam[t] * (usp - usm);
    }
    const double y = P0 * irc2[c] + div;
    pnew[c] = P0;
    q[c] = y;
    s = s + P0 * y;
  }
  const double tot = block_sum(s);
  if (threadIdx.x == 0) part_pq[blockIdx.x] = tot;
}

// The 2D product goes through LDS: a tile of CT_X x CT_Z cells stages p
// with its halo of 2 (periodic images or, on a walled axis, the wall cell),
// and tau and 1/(rho c) with their halo of 1, so each value is read from
// memory once per tile instead of once per stencil point (29 loads a cell
// become about 8).  Tiles in row-major order, a contiguous run per block
// and the blocks of one XCD together, as above.
constexpr int CT_X = 64, CT_Z = 16;
constexpr int CP_X = CT_X + 4, CP_Z = CT_Z + 4;  // p with halo 2
constexpr int CC_X = CT_X + 2, CC_Z = CT_Z + 2;  // tau, 1/(rho c) with halo 1
static_assert((CT_X * CT_Z) % BS == 0 && CT_X % 64 == 0, "tile rows are whole waves");

// One whole CG iteration in 2D, i >= 0, in one kernel.  From the previous
// iteration's r, q = A p and p (stencil reads through the LDS tile) and the
// block sums of its (p, q), (r, q), (q, q), (r, r): alpha = (r, r) / (p, q),
// the new (r, r) = (r, r) - 2 alpha (r, q) + alpha^2 (q, q) (the expansion
// of |r - alpha q|^2 over one step from exact sums: no drift accumulates),
// beta = new (r, r) / (r, r); then at every cell r' = r - alpha q,
// p' = r' + beta p, x += alpha p (own cells), q' = A p', and the block sums
// of (p', q'), (r', q'), (q', q') and the exact (r', r').  Iteration 0 takes
// alpha = beta = 0 (r' = r, p' = r).  Four sums per block in the layout
// part[k * pstride + block].
__device__ __forceinline__ void block_sum4(double (&v)[4]) {
  __shared__ double sh4[4][BS / 64];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v[k] = v[k] + __shfl_xor(v[k], m, 64);
  }
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) sh4[k][threadIdx.x >> 6] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double t = sh4[k][0];
#pragma unroll
    for (int w = 1; w < BS / 64; ++w) t = t + sh4[k][w];
    v[k] = t;
  }
}

enum { CGS_PQ = 0, CGS_RQ, CGS_QQ, CGS_RR };

__global__ __launch_bounds__(BS) void k_cg_iter_2d(Params P, const double* __restrict__ d_dt,
                                                   const double* __restrict__ rin, const double* __restrict__ qin,
                                                   const double* __restrict__ pin, double* __restrict__ rout,
                                                   double* __restrict__ qout, double* __restrict__ pout,
                                                   double* __restrict__ x, const double* __restrict__ tau,
                                                   const double* __restrict__ irc, const double* __restrict__ irc2,
                                                   const double* __restrict__ pprev, double* __restrict__ pcur,
                                                   int pstride, double* __restrict__ sc, int it, int wallmask) {
  __shared__ double sP[CP_Z][CP_X];
  __shared__ double sT[CC_Z][CC_X];
  __shared__ double sI[CC_Z][CC_X];
  __shared__ double sR[CT_Z][CT_X];
  __shared__ int colm[CP_X];
  __shared__ int rowm[CP_Z];
  double alpha = 0.0, beta = 0.0;
  if (it > 0) {
    double v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double a = 0.0;
      for (int i = threadIdx.x; i < (int)gridDim.x; i += BS) a = a + pprev[k * pstride + i];
      v[k] = a;
    }
    block_sum4(v);
    const double rr = v[CGS_RR];
    alpha = v[CGS_PQ] != 0.0 ? rr / v[CGS_PQ] : 0.0;
    const double rrn = (rr - 2.0 * alpha * v[CGS_RQ]) + (alpha * alpha) * v[CGS_QQ];
    beta = rr != 0.0 ? rrn / rr : 0.0;
    __syncthreads();
  }
  const double dt = *d_dt;
  const double lx = dt / P.dx[0], lz = dt / P.dx[2], hK = P.hK;
  const int nx = P.nx, nz = P.nz;
  const bool wx = wallmask & 1, wz = (wallmask >> 2) & 1;
  const int tx = (nx + CT_X - 1) / CT_X;
  const int tiles = tx * ((nz + CT_Z - 1) / CT_Z);
  const unsigned G = gridDim.x, b = blockIdx.x;
  const unsigned lw = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const int t0 = (int)((long long)tiles * lw / G), t1 = (int)((long long)tiles * (lw + 1) / G);
  const int tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int t = t0; t < t1; ++t) {
    const int x0 = (t % tx) * CT_X, z0 = (t / tx) * CT_Z;
    if (tid < CP_X) {
      const int v = x0 + tid - 2;
      int g = v % nx;
      g = g < 0 ? g + nx : g;
      colm[tid] = wx ? (v < 0 ? 0 : (v < nx ? v : nx - 1)) : g;
    } else if (tid < CP_X + CP_Z) {
      const int v = z0 + (tid - CP_X) - 2;
      int g = v % nz;
      g = g < 0 ? g + nz : g;
      rowm[tid - CP_X] = (wz ? (v < 0 ? 0 : (v < nz ? v : nz - 1)) : g) * nx;
    }
    __syncthreads();
    for (int e = tid; e < CP_X * CP_Z; e += BS) {
      const int j = e / CP_X, i = e - j * CP_X;
      const int idx = rowm[j] + colm[i];
      const double pp = pin[idx];
      const double rv = rin[idx] - alpha * qin[idx];
      const double pv = rv + beta * pp;
      sP[j][i] = pv;
      if (j >= 2 && j < CT_Z + 2 && i >= 2 && i < CT_X + 2 && x0 + i - 2 < nx && z0 + j - 2 < nz) {
        rout[idx] = rv;
        pout[idx] = pv;
        x[idx] = x[idx] + alpha * pp;
        sR[j - 2][i - 2] = rv;
        acc[CGS_RR] = acc[CGS_RR] + rv * rv;
      }
    }
    for (int e = tid; e < CC_X * CC_Z; e += BS) {
      const int j = e / CC_X, i = e - j * CC_X;
      const int idx = rowm[j + 1] + colm[i + 1];
      sT[j][i] = tau[idx];
      sI[j][i] = irc[idx];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < CT_X * CT_Z / BS; ++k) {
      const int e = tid + k * BS;
      const int i = e % CT_X, j = e / CT_X;
      const int gx = x0 + i, gz = z0 + j;
      if (gx < nx && gz < nz) {
        const double P0 = sP[j + 2][i + 2], t0c = sT[j + 1][i + 1], i0 = sI[j + 1][i + 1];
        double div = 0.0;
        {  // x: velocities of the cells c - e, c, c + e, then u* of the two faces
          const double Pm2 = sP[j + 2][i], Pm1 = sP[j + 2][i + 1], Pp1 = sP[j + 2][i + 3], Pp2 = sP[j + 2][i + 4];
          const double um = -(lx * sT[j + 1][i]) * (0.5 * (P0 - Pm2));
          const double uc = -(lx * t0c) * (0.5 * (Pp1 - Pm1));
          const double up = -(lx * sT[j + 1][i + 2]) * (0.5 * (Pp2 - P0));
          double usm = 0.5 * (um + uc) - (P0 - Pm1) * (hK * dmin2(sI[j + 1][i], i0));
          double usp = 0.5 * (uc + up) - (Pp1 - P0) * (hK * dmin2(i0, sI[j + 1][i + 2]));
          if (wx && gx == 0) usm = 0.0;
          if (wx && gx == nx - 1) usp = 0.0;
          div = div + lx * (usp - usm);
        }
        {  // z
          const double Pm2 = sP[j][i + 2], Pm1 = sP[j + 1][i + 2], Pp1 = sP[j + 3][i + 2], Pp2 = sP[j + 4][i + 2];
          const double um = -(lz * sT[j][i + 1]) * (0.5 * (P0 - Pm2));
          const double uc = -(lz * t0c) * (0.5 * (Pp1 - Pm1));
          const double up = -(lz * sT[j + 2][i + 1]) * (0.5 * (Pp2 - P0));
          double usm = 0.5 * (um + uc) - (P0 - Pm1) * (hK * dmin2(sI[j][i + 1], i0));
          double usp = 0.5 * (uc + up) - (Pp1 - P0) * (hK * dmin2(i0, sI[j + 2][i + 1]));
          if (wz && gz == 0) usm = 0.0;
          if (wz && gz == nz - 1) usp = 0.0;
          div = div + lz * (usp - usm);
        }
        const int c = gz * nx + gx;
        const double y = P0 * irc2[c] + div;
        qout[c] = y;
        acc[CGS_PQ] = acc[CGS_PQ] + P0 * y;
        acc[CGS_RQ] = acc[CGS_RQ] + sR[j][i] * y;
        acc[CGS_QQ] = acc[CGS_QQ] + y * y;
      }
    }
    __syncthreads();  // the next tile overwrites the LDS
  }
  block_sum4(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) pcur[k * pstride + blockIdx.x] = acc[k];
  }
}

// (r, r) of the last fused 2D iteration, for the host's convergence test.
__global__ __launch_bounds__(BS) void k_cg_check_rr(const double* __restrict__ rr_parts, int nb,
                                                    double* __restrict__ sc) {
  const double rr = sum_parts(rr_parts, nb);
  if (threadIdx.x == 0) sc[SC_CG_CHK] = rr;
}

// alpha = (r, r) / (p, q), every block adding the block sums of (p, q) in
// the same order; then x += alpha p, r -= alpha q and the block sums of
// the new (r, r).
__global__ __launch_bounds__(BS) void k_cg_xr(long long n, const double* __restrict__ p, const double* __restrict__ q,
                                              double* __restrict__ x, double* __restrict__ r,
                                              const double* __restrict__ part_pq, int nb_pq,
                                              double* __restrict__ part_rr, const double* __restrict__ sc, int it) {
  const double pq = sum_parts(part_pq, nb_pq);
  const double alpha = pq != 0.0 ? sc[SC_CG_RR + (it & 1)] / pq : 0.0;
  __syncthreads();
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * BS + threadIdx.x; i < n; i += (long long)gridDim.x * BS) {
    x[i] = x[i] + alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    s = s + ri * ri;
  }
  const double tot = block_sum(s);
  if (threadIdx.x == 0) part_rr[blockIdx.x] = tot;
}

// (r, r) of the last iteration, for the host's convergence test.
__global__ __launch_bounds__(BS) void k_cg_check(const double* __restrict__ part_rr, int nb, double* __restrict__ sc) {
  const double rr = sum_parts(part_rr, nb);
  if (threadIdx.x == 0) sc[SC_CG_CHK] = rr;
}

// x0 = p^n of every interior cell.
template <int DIM>
__global__ void k_imex_x0(Params P, RefGrid G, const double* __restrict__ W, double* __restrict__ x) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  const int cxx = (int)(c % P.nx);
  const long long rr = c / P.nx;
  const int cyy = (int)(rr % P.ny);
  const int czz = (int)(rr / P.ny);
  x[c] = W[R_P * G.npad + G.pad(cxx + 2, DIM == 3 ? cyy + 2 : 0, czz + 2)];
}

__global__ void k_fill0(long long n, double* __restrict__ a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

__global__ void k_neg(long long n, double* __restrict__ a) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = -a[i];
}

__global__ void k_add_t(double* __restrict__ t, const double* __restrict__ dt) {
  if (threadIdx.x == 0) *t = *t + *dt;
}

unsigned nblk(long long n) { return (unsigned)((n + BS - 1) / BS); }

template <int DIM>
struct Imex {
  const Params& P;
  ImexLayout L;
  hipStream_t s;
  const double* d_dt;

  hipError_t apply(const double* xin, double* y, int cst) {
    const unsigned np = nblk(L.G.npad);
    hipLaunchKernelGGL(k_schur_extP<DIM>, dim3(np), dim3(BS), 0, s, P, L.G, L.W, xin, cst, L.ext);
    if (P.low_mach)
      hipLaunchKernelGGL((k_schur_u<DIM, true>), dim3(np), dim3(BS), 0, s, P, L.G, L.W, d_dt, cst, L.ext);
    else
      hipLaunchKernelGGL((k_schur_u<DIM, false>), dim3(np), dim3(BS), 0, s, P, L.G, L.W, d_dt, cst, L.ext);
    hipLaunchKernelGGL(k_schur_rows<DIM>, dim3(nblk(P.ncell)), dim3(BS), 0, s, P, L.G, L.W, L.ext, d_dt, xin, cst, y);
    return hipGetLastError();
  }
  void dot(const double* a, const double* b, int slot) {
    hipLaunchKernelGGL(k_dot_partial, dim3(DOT_BLOCKS), dim3(BS), 0, s, a, b, L.n, L.part);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(BS), 0, s, L.part, DOT_BLOCKS, L.sc + slot);
  }
  int read(int slot, double* h) {
    if (hipMemcpyAsync(h, L.sc + slot, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return ARS_EDEVICE;
    return hipStreamSynchronize(s) == hipSuccess ? ARS_OK : ARS_EDEVICE;
  }

  // Solve the implicit system of the state whose primitives and explicit
  // faces are in the workspace; returns iterations in *its.
  int solve(double tol, int max_iter, int* its) {
    const unsigned nb = nblk(L.n);
    // b = -F(0); x0 = explicit values; r = b - L x0
    hipLaunchKernelGGL(k_fill0, dim3(nb), dim3(BS), 0, s, L.n, L.t);
    if (apply(L.t, L.b, 1) != hipSuccess) return ARS_EDEVICE;
    hipLaunchKernelGGL(k_neg, dim3(nb), dim3(BS), 0, s, L.n, L.b);
    hipLaunchKernelGGL(k_imex_x0<DIM>, dim3(nblk(P.ncell)), dim3(BS), 0, s, P, L.G, L.W, L.x);
    if (apply(L.x, L.r, 0) != hipSuccess) return ARS_EDEVICE;
    hipLaunchKernelGGL(k_bicg_start, dim3(nb), dim3(BS), 0, s, L.n, L.b, L.r, L.rh, L.p, L.v, L.sc);
    dot(L.b, L.b, SC_BB);
    double bb = 0.0;
    if (read(SC_BB, &bb) != ARS_OK) return ARS_EDEVICE;
    const double target = tol * tol * (bb > 0.0 ? bb : 1.0);
    // the explicit pressure may already solve the system (an equilibrium)
    dot(L.r, L.r, SC_RR);
    double rr0 = 0.0;
    if (read(SC_RR, &rr0) != ARS_OK) return ARS_EDEVICE;
    if (!std::isfinite(rr0)) return ARS_ENOCONV;
    if (rr0 <= target) {
      if (its) *its = 0;
      return ARS_OK;
    }
    int it = 0;
    for (; it < max_iter; ++it) {
      dot(L.rh, L.r, SC_RHO_NEW);
      hipLaunchKernelGGL(k_bicg_p, dim3(nb), dim3(BS), 0, s, L.n, L.r, L.v, L.p, L.sc);
      if (apply(L.p, L.v, 0) != hipSuccess) return ARS_EDEVICE;
      dot(L.rh, L.v, SC_RV);
      hipLaunchKernelGGL(k_bicg_s, dim3(nb), dim3(BS), 0, s, L.n, L.r, L.v, L.sv, L.sc);
      if (apply(L.sv, L.t, 0) != hipSuccess) return ARS_EDEVICE;
      dot(L.t, L.sv, SC_TS);
      dot(L.t, L.t, SC_TT);
      hipLaunchKernelGGL(k_bicg_xr, dim3(nb), dim3(BS), 0, s, L.n, L.p, L.sv, L.t, L.x, L.r, L.sc);
      hipLaunchKernelGGL(k_bicg_scalars, dim3(1), dim3(64), 0, s, L.sc);
      if (it % 4 == 3 || it + 1 == max_iter) {
        dot(L.r, L.r, SC_RR);
        double rr = 0.0;
        if (read(SC_RR, &rr) != ARS_OK) return ARS_EDEVICE;
        if (!std::isfinite(rr)) return ARS_ENOCONV;
        if (rr <= target) {
          ++it;
          break;
        }
      }
    }
    if (its) *its = it;
    if (it >= max_iter) {
      double rr = 0.0;
      if (read(SC_RR, &rr) != ARS_OK) return ARS_EDEVICE;
      if (!(rr <= target)) return ARS_ENOCONV;
    }
    return hipGetLastError() == hipSuccess ? ARS_OK : ARS_EDEVICE;
  }

  // Conjugate gradients on the same system (every side periodic).  The
  // BiCGSTAB-only vectors hold the coefficients (rh: tau, sv: 1/(rho c),
  // t: 1/(rho c^2)) and b, once the first residual is formed, the second p.
  int solve_cg(double tol, int max_iter, int* its) {
    const unsigned nb = nblk(L.n);
    // bit a: the physical axis a is walled at both ends (a configuration
    // admits walls on the vertical axis only; the products take the mask
    // per axis all the same)
    const int wallmask = (P.bcx[0] == BC_WALL ? 1 : 0) | (DIM == 3 && P.bcy[0] == BC_WALL ? 2 : 0) |
                         (P.bcz[0] == BC_WALL ? 4 : 0);
    const unsigned gb = nb < (unsigned)CG_BLOCKS ? nb : (unsigned)CG_BLOCKS;  // k_cg_xr
    unsigned ga = gb;                                                          // the product
    if (DIM == 2) {
      const long long tiles = (long long)((P.nx + CT_X - 1) / CT_X) * ((P.nz + CT_Z - 1) / CT_Z);
      ga = tiles < CG_BLOCKS ? (unsigned)tiles : (unsigned)CG_BLOCKS;
    }
    hipLaunchKernelGGL(k_fill0, dim3(nb), dim3(BS), 0, s, L.n, L.t);
    if (apply(L.t, L.b, 1) != hipSuccess) return ARS_EDEVICE;
    hipLaunchKernelGGL(k_neg, dim3(nb), dim3(BS), 0, s, L.n, L.b);
    hipLaunchKernelGGL(k_imex_x0<DIM>, dim3(nblk(P.ncell)), dim3(BS), 0, s, P, L.G, L.W, L.x);
    if (apply(L.x, L.r, 0) != hipSuccess) return ARS_EDEVICE;
    // r = b - A x0 (also clears p and v, and copies r to rh, overwritten next)
    hipLaunchKernelGGL(k_bicg_start, dim3(nb), dim3(BS), 0, s, L.n, L.b, L.r, L.rh, L.p, L.v, L.sc);
    dot(L.b, L.b, SC_BB);
    double bb = 0.0;
    if (read(SC_BB, &bb) != ARS_OK) return ARS_EDEVICE;
    const double target = tol * tol * (bb > 0.0 ? bb : 1.0);
    dot(L.r, L.r, SC_CG_RR);  // (r, r) of iteration 0
    double rr0 = 0.0;
    if (read(SC_CG_RR, &rr0) != ARS_OK) return ARS_EDEVICE;
    if (!std::isfinite(rr0)) return ARS_ENOCONV;
    if (rr0 <= target) {
      if (its) *its = 0;
      return ARS_OK;
    }
    hipLaunchKernelGGL(k_cg_coef<DIM>, dim3(nblk(P.ncell)), dim3(BS), 0, s, P, L.G, L.W, L.rh, L.sv, L.t);
    if constexpr (DIM == 2) {
      return iterate_2d(target, max_iter, its, ga, wallmask);
    } else {
      return iterate_3d(target, max_iter, its, ga, gb, wallmask);
    }
  }

  // 3D: two kernels an iteration (k_cg_apply, k_cg_xr).
  int iterate_3d(double target, int max_iter, int* its, unsigned ga, unsigned gb, int wallmask) {
    double* const part_pq = L.part;
    double* const part_rr = L.part + (CG_BLOCKS > DOT_BLOCKS ? CG_BLOCKS : DOT_BLOCKS);
    double* pv[2] = {L.p, L.b};  // p = 0 on entry, so the first p is r
    int it = 0;
    for (; it < max_iter; ++it) {
      double* po = pv[it & 1];
      double* pn = pv[(it + 1) & 1];
      hipLaunchKernelGGL(k_cg_apply<3>, dim3(ga), dim3(BS), 0, s, P, d_dt, L.r, po, pn, L.rh, L.sv, L.t, L.v,
                         part_rr, (int)gb, part_pq, L.sc, it, wallmask);
      hipLaunchKernelGGL(k_cg_xr, dim3(gb), dim3(BS), 0, s, L.n, pn, L.v, L.x, L.r, part_pq, (int)ga, part_rr, L.sc,
                         it);
      if (it % CG_CHECK == CG_CHECK - 1 || it + 1 == max_iter) {
        hipLaunchKernelGGL(k_cg_check, dim3(1), dim3(BS), 0, s, part_rr, (int)gb, L.sc);
        double rr = 0.0;
        if (read(SC_CG_CHK, &rr) != ARS_OK) return ARS_EDEVICE;
        if (!std::isfinite(rr)) return ARS_ENOCONV;
        if (rr <= target) {
          ++it;
          break;
        }
      }
    }
    if (its) *its = it;
    if (it >= max_iter) {
      double rr = 0.0;
      if (read(SC_CG_CHK, &rr) != ARS_OK) return ARS_EDEVICE;
      if (!(rr <= target)) return ARS_ENOCONV;
    }
    return hipGetLastError() == hipSuccess ? ARS_OK : ARS_EDEVICE;
  }

  // 2D: one kernel an iteration (k_cg_iter_2d).  Iteration i reads the
  // residual, product and direction of set (i + 1) & 1 and writes set i & 1
  // (set 1 starts as r0, 0, 0: k_bicg_start zeroed p and v), and its four
  // block sums go to sum set i & 1.
  int iterate_2d(double target, int max_iter, int* its, unsigned ga, int wallmask) {
    const int ps = CG_BLOCKS > DOT_BLOCKS ? CG_BLOCKS : DOT_BLOCKS;
    double* R[2] = {L.r2, L.r};
    double* Q[2] = {L.q2, L.v};
    double* Pv[2] = {L.b, L.p};
    double* S[2] = {L.part, L.part + 4 * ps};
    int it = 0;
    for (; it < max_iter; ++it) {
      const int o = it & 1, in = o ^ 1;
      hipLaunchKernelGGL(k_cg_iter_2d, dim3(ga), dim3(BS), 0, s, P, d_dt, R[in], Q[in], Pv[in], R[o], Q[o], Pv[o],
                         L.x, L.rh, L.sv, L.t, S[in], S[o], ps, L.sc, it, wallmask);
      if (it % CG_CHECK == CG_CHECK - 1 || it + 1 == max_iter) {
        hipLaunchKernelGGL(k_cg_check_rr, dim3(1), dim3(BS), 0, s, S[o] + CGS_RR * ps, (int)ga, L.sc);
        double rr = 0.0;
        if (read(SC_CG_CHK, &rr) != ARS_OK) return ARS_EDEVICE;
        if (!std::isfinite(rr)) return ARS_ENOCONV;
        if (rr <= target) {
          ++it;
          break;
        }
      }
    }
    if (its) *its = it;
    if (it >= max_iter) {
      double rr = 0.0;
      if (read(SC_CG_CHK, &rr) != ARS_OK) return ARS_EDEVICE;
      if (!(rr <= target)) return ARS_ENOCONV;
    }
    return hipGetLastError() == hipSuccess ? ARS_OK : ARS_EDEVICE;
  }

  // The rest of the step with the implicit faces of x.
  hipError_t finish(double* Uout, Control* ctl) {
    const unsigned np = nblk(L.G.npad);
    hipLaunchKernelGGL(k_schur_extP<DIM>, dim3(np), dim3(BS), 0, s, P, L.G, L.W, L.x, 1, L.ext);
    if (P.low_mach) {
      hipLaunchKernelGGL((k_schur_u<DIM, true>), dim3(np), dim3(BS), 0, s, P, L.G, L.W, d_dt, 1, L.ext);
      hipLaunchKernelGGL((k_imex_faces<DIM, true>), dim3(np), dim3(BS), 0, s, P, L.G, L.W, L.ext);
    } else {
      hipLaunchKernelGGL((k_schur_u<DIM, false>), dim3(np), dim3(BS), 0, s, P, L.G, L.W, d_dt, 1, L.ext);
      hipLaunchKernelGGL((k_imex_faces<DIM, false>), dim3(np), dim3(BS), 0, s, P, L.G, L.W, L.ext);
    }
    hipLaunchKernelGGL(k_imex_cell<DIM>, dim3(np), dim3(BS), 0, s, P, L.G, d_dt, L.W);
    if (hipGetLastError() != hipSuccess) return hipErrorUnknown;
    return launch_ref_finish(P, L.W, Uout, d_dt, ctl, s);
  }
};

}  // namespace

size_t imex_workspace_bytes(const Params& P) {
  RefGrid G = make_grid(P);
  const long long n = P.ncell;
  auto al = [](size_t b) { return ((b + 255) / 256) * 256; };
  size_t s = al((size_t)R_NFIELD * G.npad * sizeof(double)) + al((size_t)(P.dim + 1) * G.npad * sizeof(double));
  s += 10 * al((size_t)n * sizeof(double));
  s += al(8 * (CG_BLOCKS > DOT_BLOCKS ? CG_BLOCKS : DOT_BLOCKS) * sizeof(double)) + al(SC_N * sizeof(double));
  return s;
}

template <int DIM>
static int imex_steps(const Params& P, double* d_state, double* d_tmp, Control* ctl, void* wimex, int nsteps,
                      const double* d_dt_sched, double* d_t, double tol, int max_iter, int* h_iters, hipStream_t s) {
  Imex<DIM> M{P, layout_of(P, wimex), s, nullptr};
  int total = 0;
  double* src = d_state;
  double* dst = d_tmp;
  for (int st = 0; st < nsteps; ++st) {
    M.d_dt = d_dt_sched + st;
    if (launch_ref_forward(P, src, M.L.W, M.d_dt, s) != hipSuccess) return ARS_EDEVICE;
    int its = 0;
    // conjugate gradients where the operator is symmetric: every axis
    // periodic or walled at both ends
    auto sym = [](const int* bc) {
      return (bc[0] == BC_PERIODIC && bc[1] == BC_PERIODIC) || (bc[0] == BC_WALL && bc[1] == BC_WALL);
    };
    const bool symmetric = sym(P.bcx) && sym(P.bcz) && (DIM == 2 || sym(P.bcy)) && P.nx >= 2 && P.nz >= 2 &&
                           (DIM == 2 || P.ny >= 2) && P.ncell < (1LL << 31) - (long long)BS;
    const int rc = symmetric ? M.solve_cg(tol, max_iter, &its) : M.solve(tol, max_iter, &its);
    total += its;
    if (rc != ARS_OK) {
      if (h_iters) *h_iters = total;
      return rc;
    }
    if (M.finish(dst, ctl) != hipSuccess) return ARS_EDEVICE;
    if (d_t) hipLaunchKernelGGL(k_add_t, dim3(1), dim3(64), 0, s, d_t, M.d_dt);
    double* w = src;
    src = dst;
    dst = w;
  }
  if (src != d_state &&
      hipMemcpyAsync(d_state, src, (size_t)(P.dim + 2) * P.ncell * sizeof(double), hipMemcpyDeviceToDevice, s) !=
          hipSuccess)
    return ARS_EDEVICE;
  if (h_iters) *h_iters = total;
  return hipGetLastError() == hipSuccess ? ARS_OK : ARS_EDEVICE;
}

int step_imex(const Params& P, double* d_state, double* d_tmp, Control* ctl, void* wimex, int nsteps,
              const double* d_dt_sched, double* d_t, double tol, int max_iter, int* h_iters, hipStream_t s) {
  return P.dim == 3 ? imex_steps<3>(P, d_state, d_tmp, ctl, wimex, nsteps, d_dt_sched, d_t, tol, max_iter, h_iters, s)
                    : imex_steps<2>(P, d_state, d_tmp, ctl, wimex, nsteps, d_dt_sched, d_t, tol, max_iter, h_iters, s);
}

}  // namespace ars
