// ars_reduce.hip -- reductions around the step: the CFL rate of a state
// (time-step kernel), control-block preparation, dt finalisation and the
// diagnostics of Sec. 4 (deterministic two-level sums).
#include "ars_dev.h"
#include "ars_internal.h"

namespace ars {

template <int DIM>
__global__ void __launch_bounds__(256) k_rate(Params P, const double* __restrict__ U, unsigned long long* slot) {
  constexpr int NV = DIM + 2;
  __shared__ double red[4];
  double m = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    double b[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) b[v] = U[c + v * P.ncell];
    const Prim<DIM> q = cons_to_prim<DIM>(P, b);
    const double l = cell_rate<DIM>(P, q);
    m = l > m ? l : m;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mm = red[0];
    for (int w = 1; w < 4; ++w) mm = red[w] > mm ? red[w] : mm;
    atomic_max_rate(slot, mm);
  }
}

hipError_t launch_rate_reduce(const Params& P, const double* U, unsigned long long* slot, hipStream_t s) {
  long long nb = (P.ncell + 255) / 256;
  if (nb > 2048) nb = 2048;
  if (P.dim == 3)
    hipLaunchKernelGGL(k_rate<3>, dim3((unsigned)nb), dim3(256), 0, s, P, U, slot);
  else
    hipLaunchKernelGGL(k_rate<2>, dim3((unsigned)nb), dim3(256), 0, s, P, U, slot);
  return hipGetLastError();
}

// mode 0: clear rate slots 0..3; mode 1: clear slots 1..3 (keep slot 0);
// mode 2: clear the fault latch.  A kernel, not a memset, so the call can
// sit inside a captured graph.
__global__ void k_ctl_prep(Control* ctl, int mode) {
  if (threadIdx.x == 0) {
    if (mode == 0 || mode == 1) {
      for (int i = (mode == 0 ? 0 : 1); i < 4; ++i) ctl->lammax[i] = 0ull;
    }
    if (mode == 2) {
      ctl->fault = 0u;
      ctl->fault_cell = ~0ull;
    }
  }
}

hipError_t launch_ctl_prep(Control* ctl, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_prep, dim3(1), dim3(64), 0, s, ctl, mode);
  return hipGetLastError();
}

__global__ void k_dt_finish(double cfl, const Control* ctl, int slot, double* d_dt) {
  if (threadIdx.x == 0) *d_dt = cfl / __longlong_as_double((long long)ctl->lammax[slot]);
}

hipError_t launch_dt_finish(const Params& P, Control* ctl, int slot, double* d_dt, hipStream_t s) {
  hipLaunchKernelGGL(k_dt_finish, dim3(1), dim3(64), 0, s, P.cfl, ctl, slot, d_dt);
  return hipGetLastError();
}

// ---------------------------------------------------------------- diagnostics
// partial layout per block (16 doubles):
//  0 mass, 1-3 mom, 4 e_total, 5 e_kin, 6 e_int, 7 e_grav, 8 sum|u|,
//  9 max|u|, 10 max Mach, 11 bottom wall flux sum, 12 top wall flux sum
constexpr int DIAG_NB = 1024;
constexpr int DIAG_NF = 16;

size_t diag_partial_bytes(const Params&) { return (size_t)DIAG_NB * DIAG_NF * sizeof(double); }

template <int DIM>
__global__ void __launch_bounds__(256) k_diag_partial(Params P, const double* __restrict__ U, double* partials) {
  constexpr int NV = DIM + 2;
  __shared__ double sh[256];
  double acc[DIAG_NF];
#pragma unroll
  for (int i = 0; i < DIAG_NF; ++i) acc[i] = 0.0;
  const long long plane = (long long)P.nx * P.ny;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    double b[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) b[v] = U[c + v * P.ncell];
    const Prim<DIM> q = cons_to_prim<DIM>(P, b);
    const int kz = (int)(c / plane);
    const double phi = phi_at(P, kz);
    double kin = 0.0, uu = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      kin += 0.5 * b[1 + k] * q.u[k];
      uu += q.u[k] * q.u[k];
    }
    const double um = sqrt(uu);
    acc[0] += b[0];
    acc[1] += b[1];
    acc[2] += b[2];
    if (DIM == 3) acc[3] += b[3];
    acc[4] += b[NV - 1] + b[0] * phi;
    acc[5] += kin;
    acc[6] += b[NV - 1] - kin;
    acc[7] += b[0] * phi;
    acc[8] += um;
    acc[9] = um > acc[9] ? um : acc[9];
    const double ma = um / q.c;
    acc[10] = ma > acc[10] ? ma : acc[10];
    if (kz == 0) acc[11] += 2.0 * (0.5 * P.Tw2[0] - q.T) / P.dx[2];
    if (kz == P.nz - 1) acc[12] += 2.0 * (q.T - 0.5 * P.Tw2[1]) / P.dx[2];
  }
  // block reduction, fixed order
  for (int f = 0; f < 13; ++f) {
    sh[threadIdx.x] = acc[f];
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) {
        const double a = sh[threadIdx.x], bb = sh[threadIdx.x + w];
        sh[threadIdx.x] = (f == 9 || f == 10) ? (bb > a ? bb : a) : a + bb;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x * DIAG_NF + f] = sh[0];
    __syncthreads();
  }
}

__global__ void __launch_bounds__(256) k_diag_final(int nblocks, const double* partials, double* out) {
  __shared__ double sh[256];
  for (int f = 0; f < 13; ++f) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
      const double x = partials[b * DIAG_NF + f];
      a = (f == 9 || f == 10) ? (x > a ? x : a) : a + x;
    }
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
      if ((int)threadIdx.x < w) {
        const double x = sh[threadIdx.x], y = sh[threadIdx.x + w];
        sh[threadIdx.x] = (f == 9 || f == 10) ? (y > x ? y : x) : x + y;
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) out[f] = sh[0];
    __syncthreads();
  }
}

// ------------------------------------------------- kinetic-energy objective
// KE = sum_cells (1/2) sum_k m_k u_k dV; optional gradient dKE/dU:
// d/drho = -|u|^2 dV / 2, d/dm_k = u_k dV, d/dE = 0.
template <int DIM>
__global__ void __launch_bounds__(256) k_ke(Params P, double dV, const double* __restrict__ U,
                                           double* __restrict__ grad, double* partials) {
  constexpr int NV = DIM + 2;
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < P.ncell;
       c += (long long)gridDim.x * blockDim.x) {
    const double rho = U[c];
    const double r = 1.0 / rho;
    double kin = 0.0, uu = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double m = U[c + (1 + k) * P.ncell];
      const double u = m * r;
      kin = (k == 0) ? m * u : kin + m * u;
      uu = (k == 0) ? u * u : uu + u * u;
      if (grad) grad[c + (1 + k) * P.ncell] = u * dV;
    }
    acc += 0.5 * kin;
    if (grad) {
      grad[c] = -0.5 * uu * dV;
      grad[c + (NV - 1) * P.ncell] = 0.0;
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void k_ke_final(int nb, double dV, const double* partials, double* out) {
  if (threadIdx.x == 0) {
    double a = 0.0;
    int b = 0;
    // eight loads in flight together, then added in order
    for (; b + 8 <= nb; b += 8) {
      double x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = partials[b + j];
#pragma unroll
      for (int j = 0; j < 8; ++j) a += x[j];
    }
    for (; b < nb; ++b) a += partials[b];
    *out = a * dV;
  }
}

hipError_t launch_ke(const Params& P, const double* U, double* grad, double* partials, double* out, hipStream_t s) {
  double dV = P.dx[0] * P.dx[2];
  if (P.dim == 3) dV = P.dx[0] * P.dx[1] * P.dx[2];
  long long nb = (P.ncell + 255) / 256;
  if (nb > DIAG_NB) nb = DIAG_NB;
  if (P.dim == 3)
    hipLaunchKernelGGL(k_ke<3>, dim3((unsigned)nb), dim3(256), 0, s, P, dV, U, grad, partials);
  else
    hipLaunchKernelGGL(k_ke<2>, dim3((unsigned)nb), dim3(256), 0, s, P, dV, U, grad, partials);
  hipLaunchKernelGGL(k_ke_final, dim3(1), dim3(64), 0, s, (int)nb, dV, partials, out);
  return hipGetLastError();
}

// ------------------------------------------------ Nusselt-number objective
// Nu = C sum_cols 2 (T_w - T_0)/dz (bottom) or C sum_cols 2 (T_{n-1} - T_w)/dz
// (top), C = depth / (dT ncol); optional gradient dNu/dU (zero except on the
// wall-adjacent plane): with T = (gamma-1)(E - kin) / rho,
// dT/dE = (gamma-1)/rho, dT/dm_k = -(gamma-1) u_k / rho,
// dT/drho = (gamma-1)|u|^2/(2 rho) - T/rho.
template <int DIM>
__global__ void __launch_bounds__(256) k_nu(Params P, int side, double C, const double* __restrict__ U,
                                           double* __restrict__ grad, double* partials) {
  constexpr int NV = DIM + 2;
  __shared__ double sh[256];
  const long long plane = (long long)P.nx * P.ny;
  const long long base = side == 0 ? 0 : plane * (P.nz - 1);
  const double sgn = side == 0 ? -1.0 : 1.0;  // d(flux)/dT of the wall-adjacent cell
  const double Tw = 0.5 * P.Tw2[side];
  double acc = 0.0;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < plane;
       c += (long long)gridDim.x * blockDim.x) {
    const long long i = base + c;
    double b[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) b[v] = U[i + v * P.ncell];
    const Prim<DIM> q = cons_to_prim<DIM>(P, b);
    const double f = side == 0 ? 2.0 * (Tw - q.T) / P.dx[2] : 2.0 * (q.T - Tw) / P.dx[2];
    acc += f;
    if (grad) {
      const double dNdT = C * (sgn * 2.0 / P.dx[2]);
      double uu = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        uu += q.u[k] * q.u[k];
        grad[i + (1 + k) * P.ncell] = dNdT * (-(P.gm1 * q.u[k]) * q.r);
      }
      grad[i] = dNdT * ((0.5 * (P.gm1 * uu)) * q.r - q.T * q.r);
      grad[i + (NV - 1) * P.ncell] = dNdT * (P.gm1 * q.r);
    }
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

__global__ void k_nu_final(int nb, double C, const double* partials, double* out) {
  if (threadIdx.x == 0) {
    double a = 0.0;
    int b = 0;
    // eight loads in flight together, then added in order
    for (; b + 8 <= nb; b += 8) {
      double x[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) x[j] = partials[b + j];
#pragma unroll
      for (int j = 0; j < 8; ++j) a += x[j];
    }
    for (; b < nb; ++b) a += partials[b];
    *out = a * C;
  }
}

__global__ void __launch_bounds__(256) k_fill(double* p, long long n, double v) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_nusselt(const Params& P, int side, double C, const double* U, double* grad, double* partials,
                          double* out, hipStream_t s) {
  const long long plane = (long long)P.nx * P.ny;
  long long nb = (plane + 255) / 256;
  if (nb > DIAG_NB) nb = DIAG_NB;
  if (grad) {
    const long long n = (long long)(P.dim + 2) * P.ncell;
    long long fb = (n + 255) / 256;
    if (fb > 4096) fb = 4096;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)fb), dim3(256), 0, s, grad, n, 0.0);
  }
  if (P.dim == 3)
    hipLaunchKernelGGL(k_nu<3>, dim3((unsigned)nb), dim3(256), 0, s, P, side, C, U, grad, partials);
  else
    hipLaunchKernelGGL(k_nu<2>, dim3((unsigned)nb), dim3(256), 0, s, P, side, C, U, grad, partials);
  hipLaunchKernelGGL(k_nu_final, dim3(1), dim3(64), 0, s, (int)nb, C, partials, out);
  return hipGetLastError();
}

hipError_t launch_diag(const Params& P, const double* U, double* partials, double* out, hipStream_t s) {
  long long nb = (P.ncell + 255) / 256;
  if (nb > DIAG_NB) nb = DIAG_NB;
  if (P.dim == 3)
    hipLaunchKernelGGL(k_diag_partial<3>, dim3((unsigned)nb), dim3(256), 0, s, P, U, partials);
  else
    hipLaunchKernelGGL(k_diag_partial<2>, dim3((unsigned)nb), dim3(256), 0, s, P, U, partials);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, (int)nb, partials, out);
  return hipGetLastError();
}

}  // namespace ars
