// ars_api.hip -- the C ABI of include/ars.h: configuration checks, context,
// host-side initial states, and the launch sequences of the step,
// reductions and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/ars.h"
#include "ars_dev.h"
#include "ars_internal.h"

namespace {

constexpr size_t CTL_BYTES = 256;

int check(hipError_t e) { return e == hipSuccess ? ARS_OK : ARS_EDEVICE; }

bool lateral_ok(const ars_config* c, int a) {
  for (int s = 0; s < 2; ++s) {
    const int b = c->bc[a][s];
    if (b != ARS_BC_PERIODIC && b != ARS_BC_OUTFLOW) return false;
  }
  return (c->bc[a][0] == ARS_BC_PERIODIC) == (c->bc[a][1] == ARS_BC_PERIODIC);
}

// SplitMix64 generator (Steele, Lea and Flood 2014), one output per call.
uint64_t splitmix_out(uint64_t* s) {
  *s += 0x9E3779B97F4A7C15ULL;
  uint64_t v = *s;
  v ^= v >> 30;
  v *= 0xBF58476D1CE4E5B9ULL;
  v ^= v >> 27;
  v *= 0x94D049BB133111EBULL;
  v ^= v >> 31;
  return v;
}

ars::Params derive(const ars_config* c) {
  ars::Params P{};
  P.dim = c->dim;
  const int z = c->dim - 1;
  P.nx = c->n[0];
  P.ny = (c->dim == 3) ? c->n[1] : 1;
  P.nz = c->n[z];
  for (int s = 0; s < 2; ++s) {
    P.bcx[s] = c->bc[0][s];
    P.bcy[s] = (c->dim == 3) ? c->bc[1][s] : ars::BC_PERIODIC;
    P.bcz[s] = c->bc[z][s];
  }
  P.ncell = (long long)P.nx * P.ny * P.nz;
  const double hx = c->L[0] / (double)c->n[0];
  const double hy = (c->dim == 3) ? c->L[1] / (double)c->n[1] : 1.0;
  const double hz = c->L[z] / (double)c->n[z];
  const double h[3] = {hx, hy, hz};
  for (int a = 0; a < 3; ++a) {
    P.dx[a] = h[a];
    P.idx[a] = 1.0 / h[a];
    P.qidx[a] = 0.25 * P.idx[a];
  }
  P.gamma = c->gamma;
  P.gm1 = c->gamma - 1.0;
  P.g = c->g;
  P.K = c->K;
  P.hK = 0.5 / c->K;
  P.cfl = c->cfl;
  P.mu = c->mu;
  P.kappa = c->kappa;
  P.eta = (-2.0 * c->mu) / 3.0;
  const double dv = (4.0 * c->mu) / 3.0, dk = c->kappa * P.gm1;
  P.dmax = (dv < dk) ? dk : dv;
  double s2 = P.idx[0] * P.idx[0];
  if (c->dim == 3) s2 = s2 + P.idx[1] * P.idx[1];
  s2 = s2 + P.idx[2] * P.idx[2];
  P.sumidx2 = s2;
  for (int s = 0; s < 2; ++s) {
    P.Tw2[s] = 2.0 * c->T_wall[s];
    P.thermal[s] = c->thermal[s];
  }
  P.noslip = c->wall_noslip;
  P.dt_mode = c->dt_mode;
  P.low_mach = c->low_mach;
  P.diss = (c->mu > 0.0 || c->kappa > 0.0) ? 1 : 0;
  P.nc = c->energy_form == 1 ? 1 : 0;
  return P;
}

ars::Control* ctl_of(void* w) { return (ars::Control*)w; }

}  // namespace

// U^0 of a Rayleigh-Benard base with a temperature perturbation field: the
// density of d_state (the uploaded base) is kept, the energy is rebuilt from
// the level's linear temperature (the formula of the host initial state);
// rho of level k from the base column, staged in the first nz doubles of
// the x-momentum field (k_rb_mom overwrites them afterwards).
template <int DIM>
static __global__ void k_rb_dT(ars::Params P, double Tb, double Tt, double Lz, const double* __restrict__ dT,
                               double* __restrict__ U) {
  const long long N = P.ncell;
  const long long plane = (long long)P.nx * P.ny;
  const double* col = U + N;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const int k = (int)(i / plane);
    const double zk = ((double)k + 0.5) * P.dx[2];
    const double T = Tb + (Tt - Tb) * (zk / Lz);
    const double rho = col[k];
    U[i] = rho;
    U[(DIM + 1) * N + i] = (rho * (T + dT[i])) / P.gm1;
  }
}

// Momenta m = rho u0 (0 without u0) and, with u0, the kinetic energy added
// to E; runs after k_rb_dT.
template <int DIM>
static __global__ void k_rb_mom(ars::Params P, const double* __restrict__ u0, double* __restrict__ U) {
  const long long N = P.ncell;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x) {
    const double rho = U[i];
    double mm = 0.0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const double m = u0 ? rho * u0[a * N + i] : 0.0;
      U[(1 + a) * N + i] = m;
      mm = mm + m * m;
    }
    if (u0) U[(DIM + 1) * N + i] = U[(DIM + 1) * N + i] + (0.5 * mm) / rho;
  }
}

static __global__ void k_rb_dT_adjoint(long long N, int DIMv, double gm1, const double* __restrict__ U0,
                                const double* __restrict__ lam, double* __restrict__ g) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (long long)gridDim.x * blockDim.x)
    g[i] = (lam[(DIMv + 1) * N + i] * U0[i]) / gm1;
}

static unsigned flat_blocks(long long n) {
  const long long b = (n + 255) / 256;
  return (unsigned)std::max(1ll, std::min(b, 8192ll));
}

ars::Params ars::params_of(const ars_config* c) { return derive(c); }

int ars::default_zchunk(const Params& P, int tile3) {
  int zc;
  if (P.dim == 3) {
    // enough (tile, chunk) shares to fill 256 CUs several times over
    const int TX = TILE3_EX[tile3] - 4, TY = TILE3_EY[tile3] - 4;  // outputs per tile
    const long long tiles = ((P.nx + TX - 1) / TX) * (long long)((P.ny + TY - 1) / TY);
    const long long want = 1536;
    const long long nch = std::max(1ll, std::min((long long)P.nz, want / std::max(1ll, tiles)));
    zc = (int)((P.nz + nch - 1) / nch);
  } else {
    // 2D: (segment, plane) pairs per workgroup share ~ sqrt(pairs) / 13,
    // fitted to measured step times from 64 x 32 to 2048^2 (within a few
    // percent of the best share everywhere): small grids march one plane
    // per workgroup, since their step time is the latency of one march,
    // large ones longer shares that amortise the four halo planes
    const long long tiles = (P.nx + 59) / 60;
    const double pairs = (double)tiles * (double)P.nz;
    zc = (int)std::llround(std::sqrt(pairs) / 13.0);
    zc = std::max(1, std::min(zc, P.nz));
  }
  return std::max(1, zc);
}

extern "C" {

const char* ars_strerror(int s) {
  switch (s) {
    case ARS_OK: return "ok";
    case ARS_EINVAL: return "invalid argument or configuration";
    case ARS_ENOMEM: return "host allocation failed";
    case ARS_EDEVICE: return "HIP runtime or launch error";
    case ARS_ENONPHYS: return "non-physical state (rho, p or L not positive, or non-finite)";
    case ARS_EUNSUPPORTED: return "configuration not supported by this build";
    case ARS_ESCRATCH: return "state larger than the allocation-free scratch (ARS_NOALLOC_MAX_STATE doubles)";
    case ARS_ENOCONV: return "implicit acoustic solve did not converge";
    default: return "unknown status";
  }
}

int ars_validate(const ars_config* c) {
  if (!c) return ARS_EINVAL;
  if (c->dim < 1 || c->dim > 3) return ARS_EINVAL;
  const int z = c->dim - 1;
  for (int a = 0; a < c->dim; ++a) {
    if (c->n[a] < 1 || !(c->L[a] > 0.0) || !std::isfinite(c->L[a])) return ARS_EINVAL;
    if (a != z && !lateral_ok(c, a)) return ARS_EINVAL;
  }
  for (int s = 0; s < 2; ++s) {
    const int b = c->bc[z][s];
    if (b != ARS_BC_PERIODIC && b != ARS_BC_WALL && b != ARS_BC_OUTFLOW) return ARS_EINVAL;
  }
  if ((c->bc[z][0] == ARS_BC_PERIODIC) != (c->bc[z][1] == ARS_BC_PERIODIC)) return ARS_EINVAL;
  if (c->g != 0.0 && !(c->bc[z][0] == ARS_BC_WALL && c->bc[z][1] == ARS_BC_WALL)) return ARS_EINVAL;
  if (!(c->gamma > 1.0) || !(c->mu >= 0.0) || !(c->kappa >= 0.0) || !(c->K >= 1.0) || !(c->cfl > 0.0))
    return ARS_EINVAL;
  if (!std::isfinite(c->g) || !std::isfinite(c->mu) || !std::isfinite(c->kappa) || !std::isfinite(c->K) ||
      !std::isfinite(c->cfl) || !std::isfinite(c->gamma))
    return ARS_EINVAL;
  if (c->dt_mode != 0 && c->dt_mode != 1 && c->dt_mode != 2) return ARS_EINVAL;
  if (c->energy_form != 0 && c->energy_form != 1) return ARS_EINVAL;
  if (c->low_mach != 0 && c->low_mach != 1) return ARS_EINVAL;
  for (int s = 0; s < 2; ++s)
    if (c->thermal[s] != ARS_T_ADIABATIC && c->thermal[s] != ARS_T_FIXED) return ARS_EINVAL;
  long long cells = 1;
  for (int a = 0; a < c->dim; ++a) cells *= c->n[a];
  if (cells > (1ll << 31)) return ARS_EINVAL;
  return ARS_OK;
}

int ars_create(const ars_config* cfg, ars_ctx** out) {
  if (!out) return ARS_EINVAL;
  *out = nullptr;
  int rc = ars_validate(cfg);
  if (rc != ARS_OK) return rc;
  if (cfg->dim == 1) return ARS_EUNSUPPORTED;
  ars_ctx* c = new (std::nothrow) ars_ctx;
  if (!c) return ARS_ENOMEM;
  c->cfg = *cfg;
  c->P = derive(cfg);
  c->ts.tile3 = 0;
  c->ts.zchunk = ars::default_zchunk(c->P, 0);
  c->ts.num_cu = 0;
  c->ts.wg_per_cu = 0;
  c->len = (size_t)(cfg->dim + 2) * (size_t)c->P.ncell;
  *out = c;
  return ARS_OK;
}

void ars_destroy(ars_ctx* c) { delete c; }

size_t ars_state_len(const ars_ctx* c) { return c ? c->len : 0; }

size_t ars_workspace_bytes(const ars_ctx* c) {
  if (!c) return 0;
  return CTL_BYTES + ars::diag_partial_bytes(c->P) + 32 * sizeof(double);
}

size_t ars_workspace_bytes_ref(const ars_ctx* c) { return c ? ars::ref_workspace_bytes(c->P) : 0; }

int ars_set_zchunk(ars_ctx* c, int zchunk) {
  if (!c || zchunk < 1) return ARS_EINVAL;
  c->ts.zchunk = zchunk;
  return ARS_OK;
}

int ars_get_zchunk(const ars_ctx* c) { return c ? c->ts.zchunk : -1; }

int ars_set_tiling(ars_ctx* c, int zchunk, int wg_per_cu) {
  if (!c || zchunk < 1 || wg_per_cu < 0 || wg_per_cu > 32) return ARS_EINVAL;
  c->ts.zchunk = zchunk;
  c->ts.wg_per_cu = wg_per_cu;
  return ARS_OK;
}

int ars_get_tiling(const ars_ctx* c, int* zchunk, int* wg_per_cu) {
  if (!c) return ARS_EINVAL;
  if (zchunk) *zchunk = c->ts.zchunk;
  if (wg_per_cu) *wg_per_cu = c->ts.wg_per_cu;
  return ARS_OK;
}

int ars_set_tile3(ars_ctx* c, int tile) {
  if (!c || (tile != ARS_TILE3_32x10 && tile != ARS_TILE3_16x20)) return ARS_EINVAL;
  if (c->cfg.dim != 3) return tile == ARS_TILE3_32x10 ? ARS_OK : ARS_EUNSUPPORTED;
  if (c->ts.tile3 != tile) {
    c->ts.tile3 = tile;
    c->ts.zchunk = ars::default_zchunk(c->P, tile);
  }
  return ARS_OK;
}

int ars_get_tile3(const ars_ctx* c) { return c ? c->ts.tile3 : -1; }

int ars_workspace_init(ars_ctx* c, void* d_work, void* stream) {
  if (!c || !d_work) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (ars::launch_ctl_prep(ctl_of(d_work), 0, s) != hipSuccess) return ARS_EDEVICE;
  return check(ars::launch_ctl_prep(ctl_of(d_work), 2, s));
}

// -------------------------------------------------------------- init states
// Column profile of the discrete hydrostatic equilibrium: linear T (or
// T = 1), densities by the recursion of eq. well_balanced_formula with
// p = rho T (r0: the bottom density, <= 0 for T_bottom; ignored when iso).
static void hydrostatic_column(const ars_ctx* ctx, bool iso, double Tb, double Tt, double r0,
                               std::vector<double>& Tcol, std::vector<double>& rcol) {
  const ars_config& c = ctx->cfg;
  const ars::Params& P = ctx->P;
  const double dz = P.dx[2];
  const double Lz = c.L[c.dim - 1];
  auto phi = [&](int k) { return c.g * (((double)k + 0.5) * dz); };
  Tcol.resize(P.nz);
  rcol.resize(P.nz);
  for (int k = 0; k < P.nz; ++k) {
    const double zk = ((double)k + 0.5) * dz;
    Tcol[k] = Tb + (Tt - Tb) * (zk / Lz);
  }
  if (iso) r0 = std::exp(-(c.g * (0.5 * dz)));
  if (!(r0 > 0.0)) r0 = Tcol[0];
  rcol[0] = r0;
  for (int k = 1; k < P.nz; ++k) {
    const double delta = phi(k) - phi(k - 1);
    rcol[k] = (rcol[k - 1] * (Tcol[k - 1] - 0.5 * delta)) / (Tcol[k] + 0.5 * delta);
  }
}

int ars_init_state_host(const ars_ctx* ctx, int problem, const double* prm, int nprm, uint64_t seed,
                        double* h) {
  if (!ctx || !h || (nprm > 0 && !prm) || nprm < 0) return ARS_EINVAL;
  const ars_config& c = ctx->cfg;
  const ars::Params& P = ctx->P;
  const int D = c.dim;
  const long long N = P.ncell;
  const double gm1 = c.gamma - 1.0;
  auto param = [&](int i, double d) { return i < nprm ? prm[i] : d; };
  std::fill(h, h + (size_t)(D + 2) * N, 0.0);
  const double dz = P.dx[2];
  auto phi = [&](int k) { return c.g * (((double)k + 0.5) * dz); };
  switch (problem) {
    case ARS_PROB_UNIFORM: {
      const double rho = param(0, 1.0), p = param(4, 1.0);
      const double u[3] = {param(1, 0.0), param(2, 0.0), param(3, 0.0)};
      double kin = 0.0;
      for (int k = 0; k < D; ++k) kin = kin + u[k] * u[k];
      const double E = p / gm1 + 0.5 * rho * kin;
      for (long long i = 0; i < N; ++i) {
        h[i] = rho;
        for (int k = 0; k < D; ++k) h[(1 + k) * N + i] = rho * u[k];
        h[(D + 1) * N + i] = E;
      }
      return ARS_OK;
    }
    case ARS_PROB_RB:
    case ARS_PROB_ISOTHERMAL: {
      const bool iso = problem == ARS_PROB_ISOTHERMAL;
      const double Tb = iso ? 1.0 : param(0, 1.0);
      const double Tt = iso ? 1.0 : param(1, 0.5);
      const double amp = iso ? 0.0 : param(3, 0.0);
      std::vector<double> Tcol, rcol;
      hydrostatic_column(ctx, iso, Tb, Tt, param(2, -1.0), Tcol, rcol);
      uint64_t st = seed;
      const long long plane = (long long)P.nx * P.ny;
      for (long long i = 0; i < N; ++i) {
        const int k = (int)(i / plane);
        const uint64_t bits = splitmix_out(&st) >> 11;
        const double u01 = (double)bits * 0x1.0p-53;
        const double dT = amp * (2.0 * u01 - 1.0);
        h[i] = rcol[k];
        h[(D + 1) * N + i] = (rcol[k] * (Tcol[k] + dT)) / gm1;
      }
      return ARS_OK;
    }
    case ARS_PROB_GRESHO: {
      if (D != 2) return ARS_EINVAL;
      const double Ma = param(0, 1e-3);
      const double p0 = 1.0 / (c.gamma * Ma * Ma);
      const double xc = 0.5 * c.L[0], yc = 0.5 * c.L[1];
      const double hx = P.dx[0], hy = P.dx[2];
      for (int j = 0; j < P.nz; ++j) {
        const double y = ((double)j + 0.5) * hy - yc;
        for (int i = 0; i < P.nx; ++i) {
          const double x = ((double)i + 0.5) * hx - xc;
          const double r = std::sqrt(x * x + y * y);
          double ut, p;
          if (r < 0.2) {
            ut = 5.0 * r;
            p = p0 + 12.5 * r * r;
          } else if (r < 0.4) {
            ut = 2.0 - 5.0 * r;
            p = p0 + 12.5 * r * r + 4.0 - 20.0 * r + 4.0 * std::log(5.0 * r);
          } else {
            ut = 0.0;
            p = p0 - 2.0 + 4.0 * std::log(2.0);
          }
          // u_theta = 5 r vanishes at the centre: velocity 0 there
          const double ux = r > 0.0 ? -(ut * y) / r : 0.0, uy = r > 0.0 ? (ut * x) / r : 0.0;
          const long long cidx = i + (long long)P.nx * j;
          h[cidx] = 1.0;
          h[N + cidx] = 1.0 * ux;
          h[2 * N + cidx] = 1.0 * uy;
          h[3 * N + cidx] = p / gm1 + 0.5 * 1.0 * (ux * ux + uy * uy);
        }
      }
      return ARS_OK;
    }
    case ARS_PROB_SOD: {
      const double hx = P.dx[0];
      for (long long i = 0; i < N; ++i) {
        const int ix = (int)(i % P.nx);
        const double x = ((double)ix + 0.5) * hx;
        const bool left = x < 0.5 * c.L[0];
        h[i] = left ? 1.0 : 0.125;
        h[(D + 1) * N + i] = (left ? 1.0 : 0.1) / gm1;
      }
      return ARS_OK;
    }
    default:
      return ARS_EINVAL;
  }
}

int ars_init_state(ars_ctx* ctx, int problem, const double* prm, int nprm, uint64_t seed, double* d_state,
                   void* stream) {
  if (!ctx || !d_state) return ARS_EINVAL;
  std::vector<double> h;
  try {
    h.resize(ctx->len);
  } catch (...) {
    return ARS_ENOMEM;
  }
  int rc = ars_init_state_host(ctx, problem, prm, nprm, seed, h.data());
  if (rc != ARS_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(d_state, h.data(), ctx->len * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess)
    return ARS_EDEVICE;
  return check(hipStreamSynchronize(s));
}

int ars_init_rb_dT(ars_ctx* ctx, const double* prm, int nprm, const double* d_dT, const double* d_u0,
                   double* d_state, void* stream) {
  if (!ctx || !d_dT || !d_state || nprm < 0 || (nprm > 0 && !prm)) return ARS_EINVAL;
  const ars_config& c = ctx->cfg;
  const int z = c.dim - 1;
  if (c.bc[z][0] != ARS_BC_WALL || c.bc[z][1] != ARS_BC_WALL) return ARS_EINVAL;
  double base[3] = {1.0, 0.5, -1.0};
  for (int i = 0; i < nprm && i < 3; ++i) base[i] = prm[i];
  std::vector<double> Tcol, rcol;
  hydrostatic_column(ctx, false, base[0], base[1], base[2], Tcol, rcol);
  hipStream_t s = (hipStream_t)stream;
  // the column goes to the first nz doubles of the x-momentum field (the
  // caller's buffer; nz <= ncell), which k_rb_mom overwrites once k_rb_dT
  // has read it
  const long long N = ctx->P.ncell;
  if (hipMemcpyAsync(d_state + N, rcol.data(), (size_t)ctx->P.nz * sizeof(double), hipMemcpyHostToDevice, s) !=
      hipSuccess)
    return ARS_EDEVICE;
  const unsigned nb = flat_blocks(N);
  if (c.dim == 3) {
    hipLaunchKernelGGL(k_rb_dT<3>, dim3(nb), dim3(256), 0, s, ctx->P, base[0], base[1], c.L[z], d_dT, d_state);
    hipLaunchKernelGGL(k_rb_mom<3>, dim3(nb), dim3(256), 0, s, ctx->P, d_u0, d_state);
  } else {
    hipLaunchKernelGGL(k_rb_dT<2>, dim3(nb), dim3(256), 0, s, ctx->P, base[0], base[1], c.L[z], d_dT, d_state);
    hipLaunchKernelGGL(k_rb_mom<2>, dim3(nb), dim3(256), 0, s, ctx->P, d_u0, d_state);
  }
  if (hipGetLastError() != hipSuccess) return ARS_EDEVICE;
  return check(hipStreamSynchronize(s));
}

int ars_init_rb_dT_adjoint(ars_ctx* ctx, const double* d_state0, const double* d_lam, double* d_g_dT,
                           void* stream) {
  if (!ctx || !d_state0 || !d_lam || !d_g_dT) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_rb_dT_adjoint, dim3(flat_blocks(ctx->P.ncell)), dim3(256), 0, s, ctx->P.ncell,
                     ctx->cfg.dim, ctx->P.gm1, d_state0, d_lam, d_g_dT);
  return check(hipGetLastError());
}

// ---------------------------------------------------------------- stepping
int ars_compute_dt(ars_ctx* ctx, const double* d_state, void* d_work, double* d_dt, void* stream) {
  if (!ctx || !d_state || !d_work || !d_dt) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  ars::Control* ctl = ctl_of(d_work);
  if (ars::launch_ctl_prep(ctl, 0, s) != hipSuccess) return ARS_EDEVICE;
  if (ars::launch_rate_reduce(ctx->P, d_state, &ctl->lammax[0], s) != hipSuccess) return ARS_EDEVICE;
  return check(ars::launch_dt_finish(ctx->P, ctl, 0, d_dt, s));
}

int ars_step(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, int n, double* d_t, double* d_dt,
             double* d_dt_log, void* stream) {
  if (!ctx || !d_state || !d_tmp || !d_work || !d_dt || n < 0 || d_state == d_tmp) return ARS_EINVAL;
  if (n == 0) return ARS_OK;
  hipStream_t s = (hipStream_t)stream;
  ars::Control* ctl = ctl_of(d_work);
  if (ars::launch_ctl_prep(ctl, 1, s) != hipSuccess) return ARS_EDEVICE;
  double* src = d_state;
  double* dst = d_tmp;
  for (int st = 0; st < n; ++st) {
    ars::StepIO io{};
    io.rate_in = st == 0 ? nullptr : &ctl->lammax[st % 3];
    io.dt_in = d_dt;
    io.rate_out = &ctl->lammax[(st + 1) % 3];
    io.clear_slot = &ctl->lammax[(st + 2) % 3];
    io.t = d_t;
    io.dt_log = d_dt_log ? d_dt_log + st : nullptr;
    io.ctl = ctl;
    if (ars::launch_step_fused(ctx->P, src, dst, io, ctx->ts, s) != hipSuccess) return ARS_EDEVICE;
    std::swap(src, dst);
  }
  if (src != d_state) {
    if (hipMemcpyAsync(d_state, src, ctx->len * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ARS_EDEVICE;
  }
  return check(ars::launch_dt_finish(ctx->P, ctl, n % 3, d_dt, s));
}

int ars_step_sched(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, int n, const double* d_dt_sched,
                   double* d_t, void* stream) {
  if (!ctx || !d_state || !d_tmp || !d_work || !d_dt_sched || n < 0 || d_state == d_tmp) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  ars::Control* ctl = ctl_of(d_work);
  double* src = d_state;
  double* dst = d_tmp;
  for (int st = 0; st < n; ++st) {
    ars::StepIO io{};
    io.rate_in = nullptr;
    io.dt_in = d_dt_sched + st;
    io.rate_out = nullptr;
    io.clear_slot = nullptr;
    io.t = d_t;
    io.dt_log = nullptr;
    io.ctl = ctl;
    if (ars::launch_step_fused(ctx->P, src, dst, io, ctx->ts, s) != hipSuccess) return ARS_EDEVICE;
    std::swap(src, dst);
  }
  if (src != d_state) {
    if (hipMemcpyAsync(d_state, src, ctx->len * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ARS_EDEVICE;
  }
  return ARS_OK;
}

int ars_step_to(ars_ctx* ctx, const double* d_in, double* d_a, double* d_b, double* d_out, void* d_work, int n,
                double* d_t, double* d_dt, double* d_dt_log, void* stream) {
  if (!ctx || !d_in || !d_a || !d_b || !d_out || !d_work || !d_dt || n < 1 || d_a == d_b || d_in == d_a ||
      d_in == d_b || d_out == d_a || d_out == d_b || (n == 1 && d_out == d_in))
    return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  ars::Control* ctl = ctl_of(d_work);
  if (ars::launch_ctl_prep(ctl, 1, s) != hipSuccess) return ARS_EDEVICE;
  const double* src = d_in;
  for (int st = 0; st < n; ++st) {
    double* dst = st + 1 == n ? d_out : (st % 2 == 0 ? d_a : d_b);
    ars::StepIO io{};
    io.rate_in = st == 0 ? nullptr : &ctl->lammax[st % 3];
    io.dt_in = d_dt;
    io.rate_out = &ctl->lammax[(st + 1) % 3];
    io.clear_slot = &ctl->lammax[(st + 2) % 3];
    io.t = d_t;
    io.dt_log = d_dt_log ? d_dt_log + st : nullptr;
    io.ctl = ctl;
    if (ars::launch_step_fused(ctx->P, src, dst, io, ctx->ts, s) != hipSuccess) return ARS_EDEVICE;
    src = dst;
  }
  return check(ars::launch_dt_finish(ctx->P, ctl, n % 3, d_dt, s));
}

int ars_step_sched_to(ars_ctx* ctx, const double* d_in, double* d_a, double* d_b, double* d_out, void* d_work,
                      int n, const double* d_dt_sched, double* d_t, void* stream) {
  if (!ctx || !d_in || !d_a || !d_b || !d_out || !d_work || !d_dt_sched || n < 1 || d_a == d_b || d_in == d_a ||
      d_in == d_b || d_out == d_a || d_out == d_b || (n == 1 && d_out == d_in))
    return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  ars::Control* ctl = ctl_of(d_work);
  const double* src = d_in;
  for (int st = 0; st < n; ++st) {
    double* dst = st + 1 == n ? d_out : (st % 2 == 0 ? d_a : d_b);
    ars::StepIO io{};
    io.rate_in = nullptr;
    io.dt_in = d_dt_sched + st;
    io.rate_out = nullptr;
    io.clear_slot = nullptr;
    io.t = d_t;
    io.dt_log = nullptr;
    io.ctl = ctl;
    if (ars::launch_step_fused(ctx->P, src, dst, io, ctx->ts, s) != hipSuccess) return ARS_EDEVICE;
    src = dst;
  }
  return ARS_OK;
}

size_t ars_workspace_bytes_imex(const ars_ctx* c) { return c ? ars::imex_workspace_bytes(c->P) : 0; }

int ars_step_imex(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, void* d_work_imex, int n,
                  const double* d_dt_sched, double* d_t, double tol, int max_iter, int* h_iters, void* stream) {
  if (h_iters) *h_iters = 0;
  if (!ctx || !d_state || !d_tmp || !d_work || !d_work_imex || !d_dt_sched || n < 0 || d_state == d_tmp ||
      !(tol > 0.0) || max_iter < 1)
    return ARS_EINVAL;
  if (ctx->P.nc) return ARS_EUNSUPPORTED;
  if (n == 0) return ARS_OK;
  return ars::step_imex(ctx->P, d_state, d_tmp, ctl_of(d_work), d_work_imex, n, d_dt_sched, d_t, tol, max_iter,
                        h_iters, (hipStream_t)stream);
}

int ars_step_ref(ars_ctx* ctx, double* d_state, double* d_tmp, void* d_work, void* d_work_ref, int n,
                 const double* d_dt_sched, void* stream) {
  if (!ctx || !d_state || !d_tmp || !d_work || !d_work_ref || !d_dt_sched || n < 0 || d_state == d_tmp)
    return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  ars::Control* ctl = ctl_of(d_work);
  double* src = d_state;
  double* dst = d_tmp;
  for (int st = 0; st < n; ++st) {
    if (ars::launch_step_ref(ctx->P, src, dst, d_work_ref, d_dt_sched + st, ctl, s) != hipSuccess)
      return ARS_EDEVICE;
    std::swap(src, dst);
  }
  if (src != d_state) {
    if (hipMemcpyAsync(d_state, src, ctx->len * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ARS_EDEVICE;
  }
  return ARS_OK;
}

size_t ars_workspace_bytes_adjoint(const ars_ctx* c) { return c ? ars::adjoint_workspace_bytes(c->P) : 0; }
size_t ars_workspace_bytes_adjoint_ref(const ars_ctx* c) { return c ? ars::adjoint_ref_workspace_bytes(c->P) : 0; }

int ars_step_adjoint_ref(ars_ctx* ctx, const double* d_state_n, const double* d_lam_np1, double* d_lam_n,
                         const double* d_dt, double* d_param_grad, void* d_work_adj, void* stream) {
  if (!ctx || !d_state_n || !d_lam_np1 || !d_lam_n || !d_dt || !d_work_adj || d_lam_n == d_lam_np1)
    return ARS_EINVAL;
  return check(ars::launch_step_adjoint_ref(ctx->P, d_state_n, d_lam_np1, d_lam_n, d_dt, d_param_grad, d_work_adj,
                                            (hipStream_t)stream));
}

int ars_step_adjoint(ars_ctx* ctx, const double* d_state_n, const double* d_lam_np1, double* d_lam_n,
                     const double* d_dt, double* d_param_grad, void* d_work_adj, void* stream) {
  if (!ctx || !d_state_n || !d_lam_np1 || !d_lam_n || !d_dt || !d_work_adj || d_lam_n == d_lam_np1)
    return ARS_EINVAL;
  return check(ars::launch_step_adjoint(ctx->P, d_state_n, d_lam_np1, d_lam_n, d_dt, d_param_grad, d_work_adj,
                                        (hipStream_t)stream));
}

int ars_kinetic_energy(ars_ctx* ctx, const double* d_state, double* d_grad, double* d_ke, void* d_work,
                       void* stream) {
  if (!ctx || !d_state || !d_ke || !d_work) return ARS_EINVAL;
  char* w = (char*)d_work;
  double* partials = (double*)(w + CTL_BYTES);
  return check(ars::launch_ke(ctx->P, d_state, d_grad, partials, d_ke, (hipStream_t)stream));
}

int ars_nusselt(ars_ctx* ctx, const double* d_state, int side, double* d_grad, double* d_nu, void* d_work,
                void* stream) {
  if (!ctx || !d_state || !d_nu || !d_work || (side != 0 && side != 1)) return ARS_EINVAL;
  const ars_config& c = ctx->cfg;
  const int z = c.dim - 1;
  if (c.bc[z][0] != ARS_BC_WALL || c.bc[z][1] != ARS_BC_WALL || c.thermal[side] != ARS_T_FIXED) return ARS_EINVAL;
  const double dT = c.T_wall[0] - c.T_wall[1];
  if (!(dT != 0.0)) return ARS_EINVAL;
  const double ncol = (double)ctx->P.nx * (double)ctx->P.ny;
  const double C = (c.L[z] / dT) / ncol;
  char* w = (char*)d_work;
  double* partials = (double*)(w + CTL_BYTES);
  return check(ars::launch_nusselt(ctx->P, side, C, d_state, d_grad, partials, d_nu, (hipStream_t)stream));
}

int ars_spectrum_len(const ars_ctx* ctx) { return ctx ? ars::spectrum_shells(ctx->P) : 0; }

size_t ars_workspace_bytes_spectrum(const ars_ctx* ctx) { return ctx ? ars::spectrum_work_bytes(ctx->P) : 0; }

int ars_spectrum(ars_ctx* ctx, const double* d_state, int kz, double* d_spec, void* d_work_spec, void* stream) {
  if (!ctx || !d_state || !d_spec || !d_work_spec || kz < 0 || kz >= ctx->P.nz) return ARS_EINVAL;
  if (!ars::spectrum_supported(ctx->P)) return ARS_EUNSUPPORTED;
  return check(ars::launch_spectrum(ctx->P, d_state, kz, d_spec, d_work_spec, (hipStream_t)stream));
}

int ars_fault(ars_ctx* ctx, void* d_work, int64_t* fault_cell, void* stream) {
  if (!ctx || !d_work) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  ars::Control h{};
  if (hipMemcpyAsync(&h, d_work, sizeof(ars::Control), hipMemcpyDeviceToHost, s) != hipSuccess) return ARS_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return ARS_EDEVICE;
  if (fault_cell) *fault_cell = h.fault ? (int64_t)h.fault_cell : -1;
  if (h.fault) {
    if (ars::launch_ctl_prep(ctl_of(d_work), 2, s) != hipSuccess) return ARS_EDEVICE;
    return ARS_ENONPHYS;
  }
  return ARS_OK;
}

int ars_diagnostics(ars_ctx* ctx, const double* d_state, void* d_work, ars_diag* out, void* stream) {
  if (!ctx || !d_state || !d_work || !out) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  char* w = (char*)d_work;
  double* partials = (double*)(w + CTL_BYTES);
  double* res = (double*)(w + CTL_BYTES + ars::diag_partial_bytes(ctx->P));
  if (ars::launch_diag(ctx->P, d_state, partials, res, s) != hipSuccess) return ARS_EDEVICE;
  double r[16];
  if (hipMemcpyAsync(r, res, 13 * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess) return ARS_EDEVICE;
  int64_t fc = -1;
  const int frc = ars_fault(ctx, d_work, &fc, stream);
  if (frc == ARS_EDEVICE) return frc;
  const ars::Params& P = ctx->P;
  double dV = P.dx[0] * P.dx[2];
  if (P.dim == 3) dV = P.dx[0] * P.dx[1] * P.dx[2];
  std::memset(out, 0, sizeof(*out));
  out->mass = r[0] * dV;
  out->mom[0] = r[1] * dV;
  out->mom[1] = r[2] * dV;
  out->mom[2] = r[3] * dV;
  out->e_total = r[4] * dV;
  out->e_kin = r[5] * dV;
  out->e_int = r[6] * dV;
  out->e_grav = r[7] * dV;
  out->mean_u = r[8] / (double)P.ncell;
  out->max_u = r[9];
  out->max_mach = r[10];
  const ars_config& c = ctx->cfg;
  const int z = c.dim - 1;
  if (c.bc[z][0] == ARS_BC_WALL && c.bc[z][1] == ARS_BC_WALL) {
    const double dT = c.T_wall[0] - c.T_wall[1];
    const double ncol = (double)P.nx * (double)P.ny;
    if (dT != 0.0) {
      out->nu_bot = (r[11] / ncol) * c.L[z] / dT;
      out->nu_top = (r[12] / ncol) * c.L[z] / dT;
    }
  }
  out->fault = (frc == ARS_ENONPHYS) ? 1 : 0;
  out->fault_cell = fc;
  return frc;
}

}  // extern "C"
