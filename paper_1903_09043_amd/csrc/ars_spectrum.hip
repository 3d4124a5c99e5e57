// ars_spectrum.hip -- kinetic-energy spectrum of one horizontal plane, the
// diagnostic of the 3D Rayleigh-Benard runs (Sec. 4.5, 3D case).
//
// For w_c = sqrt(rho) u_c on the plane at vertical index kz (every velocity
// component), W_c(k) = sum_x w_c(x) exp(-2 pi i k.x / n) and
//   E(s) = sum_{k : round(|k|) = s} sum_c |W_c(k)|^2 / (2 N^2),
// k integer wave vectors in the FFT order (k_j = j for j < (n+1)/2, else
// j - n), N the cell count of the plane; sum_s E(s) is then the plane mean of
// rho |u|^2 / 2 (Parseval).  In 2D the plane is a line along x.
//
// The transform is a direct DFT, rows then columns, with the twiddle table
// of each length in LDS and the exponent k x reduced modulo n exactly in
// integers; the plane is at most 2048 x 2048, so the O(N (n_x + n_y)) cost
// stays in the milliseconds.  Shell sums visit the plane in a fixed order
// and reduce through a fixed tree: the result is deterministic.
#include "ars_dev.h"
#include "ars_internal.h"

namespace ars {

constexpr int SPEC_MAXN = 2048;

__device__ __forceinline__ int fft_wavenumber(int j, int n) { return j < (n + 1) / 2 ? j : j - n; }

// tw[j] = exp(-2 pi i j / n), j < n, cos in tw[0..n), -sin in tw[n..2n).
__device__ __forceinline__ void fill_twiddles(double* tw, int n) {
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)j / (double)n, &s, &c);
    tw[j] = c;
    tw[n + j] = -s;
  }
}

// Row transforms: block (y, c) loads w_c on row y of the plane and writes
// X_c(y, kx) = sum_x w_c(x, y) exp(-2 pi i kx x / nx).
__global__ void __launch_bounds__(256) k_spec_rows(Params P, const double* __restrict__ U, int kz,
                                                   double* __restrict__ Xr, double* __restrict__ Xi) {
  extern __shared__ double sm[];
  const int nx = P.nx, y = blockIdx.x, c = blockIdx.y;
  double* w = sm;
  double* tw = sm + nx;
  const long long base = ((long long)kz * P.ny + y) * nx;
  for (int x = threadIdx.x; x < nx; x += blockDim.x) {
    const double rho = U[base + x];
    const double m = U[(long long)(1 + c) * P.ncell + base + x];
    w[x] = sqrt(rho) * (m / rho);
  }
  fill_twiddles(tw, nx);
  __syncthreads();
  const long long o = ((long long)c * P.ny + y) * nx;
  for (int kx = threadIdx.x; kx < nx; kx += blockDim.x) {
    double ar = 0.0, ai = 0.0;
    int e = 0;  // kx x mod nx
    for (int x = 0; x < nx; ++x) {
      ar += w[x] * tw[e];
      ai += w[x] * tw[nx + e];
      e += kx;
      if (e >= nx) e -= nx;
    }
    Xr[o + kx] = ar;
    Xi[o + kx] = ai;
  }
}

// Column transforms of component c: block kx loads X_c(., kx) and adds
// |Y_c(ky, kx)|^2 to Pw(ky, kx) (stored when c == 0), with
// Y_c(ky, kx) = sum_y X_c(y, kx) exp(-2 pi i ky y / ny).  The components are
// launched in order, so Pw = |Y_0|^2 + |Y_1|^2 + |Y_2|^2 in that order.
__global__ void __launch_bounds__(256) k_spec_cols(Params P, int c, const double* __restrict__ Xr,
                                                   const double* __restrict__ Xi, double* __restrict__ Pw) {
  extern __shared__ double sm[];
  const int nx = P.nx, ny = P.ny, kx = blockIdx.x;
  double* vr = sm;
  double* vi = sm + ny;
  double* tw = sm + 2 * ny;
  const long long o = (long long)c * ny * nx;
  for (int y = threadIdx.x; y < ny; y += blockDim.x) {
    vr[y] = Xr[o + (long long)y * nx + kx];
    vi[y] = Xi[o + (long long)y * nx + kx];
  }
  fill_twiddles(tw, ny);
  __syncthreads();
  for (int ky = threadIdx.x; ky < ny; ky += blockDim.x) {
    double ar = 0.0, ai = 0.0;
    int e = 0;
    for (int y = 0; y < ny; ++y) {
      const double cr = tw[e], ci = tw[ny + e];
      ar += vr[y] * cr - vi[y] * ci;
      ai += vr[y] * ci + vi[y] * cr;
      e += ky;
      if (e >= ny) e -= ny;
    }
    const double p = ar * ar + ai * ai;
    const long long q = (long long)ky * nx + kx;
    Pw[q] = c == 0 ? p : Pw[q] + p;
  }
}

// Largest k >= 0 with 4 k^2 < q (q > 0), from a floating estimate corrected
// in integers.
__device__ __forceinline__ long long kmax_below(long long q) {
  long long k = (long long)sqrt((double)q * 0.25);
  while (k > 0 && 4 * k * k >= q) --k;
  while (4 * (k + 1) * (k + 1) < q) ++k;
  return k;
}

// Power of the wave vectors (kx, ky) of one row with |kx| = k, both signs
// where the FFT order holds them (+k at index k if k < (n+1)/2; -k at index
// n - k if 1 <= k <= n/2).
__device__ __forceinline__ double row_pair(const double* __restrict__ row, int n, long long k) {
  double s = 0.0;
  if (k < (n + 1) / 2) s += row[k];
  if (k >= 1 && k <= n / 2) s += row[n - k];
  return s;
}

// Shell sums: block s adds Pw over the wave vectors with round(|k|) = s,
// i.e. (2s - 1)^2 < 4 |k|^2 < (2s + 1)^2 (4 |k|^2 is even, so no bound is
// ever met exactly), and stores the sum / (2 N^2).  Thread t takes the rows
// t, t + 256, ...; in a row it walks only the |kx| of the annulus, in
// increasing order; a fixed tree then adds the threads: deterministic.
__global__ void __launch_bounds__(256) k_spec_shells(Params P, const double* __restrict__ Pw, double* __restrict__ E) {
  __shared__ double red[256];
  const int nx = P.nx, ny = P.ny, s = blockIdx.x;
  const long long N = (long long)nx * ny;
  const long long hi = (2LL * s + 1) * (2LL * s + 1);
  const long long lo = s == 0 ? -1 : (2LL * s - 1) * (2LL * s - 1);
  double acc = 0.0;
  for (int y = threadIdx.x; y < ny; y += blockDim.x) {
    const long long ky = fft_wavenumber(y, ny);
    const long long r = 4 * ky * ky;
    if (r >= hi) continue;
    const long long kb = kmax_below(hi - r);                    // 4 kx^2 < hi - r
    const long long ka = lo - r < 0 ? 0 : kmax_below(lo - r + 1) + 1;  // 4 kx^2 > lo - r
    const double* row = Pw + (long long)y * nx;
    for (long long k = ka; k <= kb; ++k) acc += row_pair(row, nx, k);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) E[s] = red[0] / (2.0 * (double)N * (double)N);
}

int spectrum_shells(const Params& P) {
  const double hx = (double)(P.nx / 2), hy = (double)(P.ny / 2);
  return (int)llrint(sqrt(hx * hx + hy * hy)) + 1;
}

size_t spectrum_work_bytes(const Params& P) {
  const size_t N = (size_t)P.nx * (size_t)P.ny;
  return (size_t)(2 * P.dim + 1) * N * sizeof(double);
}

bool spectrum_supported(const Params& P) { return P.nx <= SPEC_MAXN && P.ny <= SPEC_MAXN; }

hipError_t launch_spectrum(const Params& P, const double* U, int kz, double* E, void* work, hipStream_t s) {
  const long long N = (long long)P.nx * P.ny;
  double* Xr = (double*)work;
  double* Xi = Xr + (long long)P.dim * N;
  double* Pw = Xi + (long long)P.dim * N;
  hipLaunchKernelGGL(k_spec_rows, dim3((unsigned)P.ny, (unsigned)P.dim), dim3(256),
                     (size_t)3 * P.nx * sizeof(double), s, P, U, kz, Xr, Xi);
  for (int c = 0; c < P.dim; ++c)
    hipLaunchKernelGGL(k_spec_cols, dim3((unsigned)P.nx), dim3(256), (size_t)4 * P.ny * sizeof(double), s, P, c,
                       Xr, Xi, Pw);
  hipLaunchKernelGGL(k_spec_shells, dim3((unsigned)spectrum_shells(P)), dim3(256), 0, s, P, Pw, E);
  return hipGetLastError();
}

}  // namespace ars
