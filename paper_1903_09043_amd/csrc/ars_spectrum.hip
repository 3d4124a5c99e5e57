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
// When both sides are powers of two the transform is a radix-2 FFT, rows
// then columns, each transform staged in LDS (bit-reversed load, log2 n
// butterfly stages with a barrier each; the column kernel takes a tile of
// adjacent columns so its loads are row segments, and forms |Y|^2).
// Otherwise it is a dense DFT, rows then columns, and a DFT is a matrix
// product: the row transform is W (n_y x n_x) times the n_x x n_x twiddle
// matrix, the column transform the n_y x n_y twiddle matrix times X, so
// both run on the FP64 matrix cores (v_mfma_f64_16x16x4f64: one wave
// accumulates a 16 x 16 tile over K in steps of 4).  The twiddle matrices
// are never stored: entry (k, x) is read from an LDS table of
// exp(-2 pi i j / n) at j = k x mod n, the exponent carried exactly in
// integers.  Shell sums visit the plane in a fixed order and add the
// threads' sums in a fixed order: the result is deterministic.
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

typedef double dbl4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 FP64 matrix step: C (16 x 16) += A (16 x 4) B (4 x 16).
// Lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]; it holds
// C[l / 16 + 4 r][l % 16] in element r.
__device__ __forceinline__ dbl4 mma16(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// w_c = sqrt(rho) u_c on the plane, W[c][y][x].
__global__ void __launch_bounds__(256) k_spec_w(Params P, const double* __restrict__ U, int kz,
                                                double* __restrict__ W) {
  const long long N = (long long)P.nx * P.ny;
  const long long base = (long long)kz * N;
  for (long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x; f < N * P.dim;
       f += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(f / N);
    const long long i = f - c * N;
    const double rho = U[base + i];
    const double m = U[(long long)(1 + c) * P.ncell + base + i];
    W[f] = sqrt(rho) * (m / rho);
  }
}

// Row transforms X_c = W_c T_x, T_x(x, k) = exp(-2 pi i k x / n_x): block
// (kx group of 64, row tile of 16, component c), wave w the 16 x 16 tile of
// rows y0.. and wave numbers k0 = 64 bx + 16 w ..; real and imaginary
// parts in two accumulators.  Out-of-range rows, columns and K entries
// contribute zeros.
__global__ void __launch_bounds__(256) k_spec_rows(Params P, const double* __restrict__ W, double* __restrict__ Xr,
                                                   double* __restrict__ Xi) {
  extern __shared__ double tw[];
  const int nx = P.nx, ny = P.ny, c = blockIdx.z;
  fill_twiddles(tw, nx);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int y0 = blockIdx.y * 16, k0 = blockIdx.x * 64 + wave * 16;
  const int y = y0 + i, k = k0 + i;  // A row of this lane, B column of this lane
  const double* Wr = W + ((long long)c * ny + (y < ny ? y : 0)) * nx;
  const int dk = (int)((4LL * k) % nx);
  int e = (int)(((long long)k * q) % nx);  // k x mod n_x at x = q
  dbl4 ar = {0.0, 0.0, 0.0, 0.0}, ai = {0.0, 0.0, 0.0, 0.0};
  // K in blocks of 8 steps: all operand loads of a block are issued before
  // its 16 matrix steps
  for (int x0 = 0; x0 < nx; x0 += 32) {
    double a[8], br[8], bi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int x = x0 + 4 * j + q;
      const bool in = x < nx;
      a[j] = (in && y < ny) ? Wr[x] : 0.0;
      br[j] = (in && k < nx) ? tw[e] : 0.0;
      bi[j] = (in && k < nx) ? tw[nx + e] : 0.0;
      e += dk;
      if (e >= nx) e -= nx;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ar = mma16(a[j], br[j], ar);
      ai = mma16(a[j], bi[j], ai);
    }
  }
  const int kc = k0 + i;  // output column of this lane
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int yo = y0 + q + 4 * r;
    if (yo < ny && kc < nx) {
      const long long o = ((long long)c * ny + yo) * nx + kc;
      Xr[o] = ar[r];
      Xi[o] = ai[r];
    }
  }
}

// Column transforms Y_c = T_y X_c, T_y(ky, y) = exp(-2 pi i ky y / n_y),
// and Pc[c](ky, k) = |Y_c(ky, k)|^2: block (k group of 64, ky tile of 16,
// component c), wave w the 16 x 16 tile of ky0.. and k0 = 64 bx + 16 w ..
__global__ void __launch_bounds__(256) k_spec_cols(Params P, const double* __restrict__ Xr,
                                                   const double* __restrict__ Xi, double* __restrict__ Pc) {
  extern __shared__ double tw[];
  const int nx = P.nx, ny = P.ny, c = blockIdx.z;
  fill_twiddles(tw, ny);
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const int ky0 = blockIdx.y * 16, k0 = blockIdx.x * 64 + wave * 16;
  const int ky = ky0 + i, k = k0 + i;  // A row (ky) and B column (k) of this lane
  const long long o = (long long)c * ny * nx;
  const int dky = (int)((4LL * ky) % ny);
  int e = (int)(((long long)ky * q) % ny);  // ky y mod n_y at y = q
  dbl4 yr = {0.0, 0.0, 0.0, 0.0}, yi = {0.0, 0.0, 0.0, 0.0};
  for (int y0 = 0; y0 < ny; y0 += 32) {
    double tr[8], ti[8], xr[8], xi[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int y = y0 + 4 * j + q;
      const bool in = y < ny;
      tr[j] = (in && ky < ny) ? tw[e] : 0.0;
      ti[j] = (in && ky < ny) ? tw[ny + e] : 0.0;
      const bool bk = in && k < nx;
      xr[j] = bk ? Xr[o + (long long)y * nx + k] : 0.0;
      xi[j] = bk ? Xi[o + (long long)y * nx + k] : 0.0;
      e += dky;
      if (e >= ny) e -= ny;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      // (tr + i ti)(xr + i xi)
      yr = mma16(tr[j], xr[j], yr);
      yr = mma16(-ti[j], xi[j], yr);
      yi = mma16(tr[j], xi[j], yi);
      yi = mma16(ti[j], xr[j], yi);
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int kyo = ky0 + q + 4 * r;
    if (kyo < ny && k < nx) Pc[o + (long long)kyo * nx + k] = yr[r] * yr[r] + yi[r] * yi[r];
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
// The power of wave vector index f: |Y_0|^2 + |Y_1|^2 (+ |Y_2|^2), summed in
// component order.
__device__ __forceinline__ double power_at(const double* __restrict__ Pc, long long N, int D, long long f) {
  double p = Pc[f];
  for (int c = 1; c < D; ++c) p = p + Pc[c * N + f];
  return p;
}

__device__ __forceinline__ double row_pair(const double* __restrict__ Pc, long long N, int D, long long row, int n,
                                           long long k) {
  double s = 0.0;
  if (k < (n + 1) / 2) s += power_at(Pc, N, D, row + k);
  if (k >= 1 && k <= n / 2) s += power_at(Pc, N, D, row + n - k);
  return s;
}

// Shell sums: block s adds the power over the wave vectors with round(|k|) = s,
// i.e. (2s - 1)^2 < 4 |k|^2 < (2s + 1)^2 (4 |k|^2 is even, so no bound is
// ever met exactly), and stores the sum / (2 N^2).  Thread t takes the rows
// t, t + 256, ...; in a row it walks only the |kx| of the annulus, in
// increasing order; the threads are added in a fixed order: deterministic.
__global__ void __launch_bounds__(256) k_spec_shells(Params P, const double* __restrict__ Pc, double* __restrict__ E) {
  __shared__ double red[4];
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
    for (long long k = ka; k <= kb; ++k) acc += row_pair(Pc, N, P.dim, (long long)y * nx, nx, k);
  }
  // fixed order: a butterfly within each wave, then the four waves in order
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) acc = acc + __shfl_xor(acc, m, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) E[s] = (((red[0] + red[1]) + red[2]) + red[3]) / (2.0 * (double)N * (double)N);
}

// ---------------------------------------------------------------- FFT path
constexpr int FFT_LDS_DOUBLES = 8192;  // 64 KB of dynamic LDS

__device__ __forceinline__ int bit_reverse(int x, int logn) {
  return logn ? (int)(__brev((unsigned)x) >> (32 - logn)) : 0;
}

// tw[j] = exp(-2 pi i j / n) for j < n / 2: cos in tw[0..n/2), -sin in
// tw[n/2..n).
__device__ __forceinline__ void fill_half_twiddles(double* tw, int n) {
  const int h = n / 2;
  for (int j = threadIdx.x; j < h; j += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)j / (double)n, &sn, &cs);
    tw[j] = cs;
    tw[h + j] = -sn;
  }
}

// cw interleaved n-point transforms in LDS (element y of transform cc at
// y * cw + cc, loaded in bit-reversed order): the radix-2 stages, each a
// set of butterflies X_i, X_j <- X_i + w X_j, X_i - w X_j with
// w = exp(-2 pi i k / len), then a barrier.
__device__ void fft_stages(double* re, double* im, const double* tw, int n, int cw) {
  const int h = n / 2;
  for (int half = 1; half < n; half <<= 1) {
    const int len = 2 * half, step = n / len;
    for (int b = threadIdx.x; b < cw * h; b += blockDim.x) {
      const int cc = b % cw, t = b / cw;
      const int k = t % half, i = (t / half) * len + k;
      const int a = i * cw + cc, c2 = (i + half) * cw + cc;
      const double wr = tw[k * step], wi = tw[h + k * step];
      const double xr = re[c2], xi = im[c2];
      const double tr = wr * xr - wi * xi;
      const double ti = wr * xi + wi * xr;
      const double ar = re[a], ai = im[a];
      re[a] = ar + tr;
      im[a] = ai + ti;
      re[c2] = ar - tr;
      im[c2] = ai - ti;
    }
    __syncthreads();
  }
}

// Row transforms: block (row y, component c).
__global__ void __launch_bounds__(256) k_fft_rows(Params P, int logx, const double* __restrict__ W,
                                                  double* __restrict__ Xr, double* __restrict__ Xi) {
  extern __shared__ double sm[];
  const int n = P.nx, y = blockIdx.x, c = blockIdx.y;
  double* tw = sm;
  double* re = sm + n;
  double* im = re + n;
  fill_half_twiddles(tw, n);
  const long long o = ((long long)c * P.ny + y) * n;
  for (int x = threadIdx.x; x < n; x += blockDim.x) {
    const int j = bit_reverse(x, logx);
    re[j] = W[o + x];
    im[j] = 0.0;
  }
  __syncthreads();
  fft_stages(re, im, tw, n, 1);
  for (int k = threadIdx.x; k < n; k += blockDim.x) {
    Xr[o + k] = re[k];
    Xi[o + k] = im[k];
  }
}

// Column transforms and power: block (cw adjacent columns from k0, component
// c); Pc[c](ky, k) = |Y_c(ky, k)|^2.
__global__ void __launch_bounds__(256) k_fft_cols(Params P, int logy, int cw, const double* __restrict__ Xr,
                                                  const double* __restrict__ Xi, double* __restrict__ Pc) {
  extern __shared__ double sm[];
  const int nx = P.nx, n = P.ny, c = blockIdx.y, k0 = blockIdx.x * cw;
  double* tw = sm;
  double* re = sm + n;
  double* im = re + n * cw;
  fill_half_twiddles(tw, n);
  const long long o = (long long)c * n * nx;
  for (int e = threadIdx.x; e < cw * n; e += blockDim.x) {
    const int y = e / cw, cc = e - y * cw, k = k0 + cc;
    const int j = bit_reverse(y, logy) * cw + cc;
    const bool in = k < nx;
    re[j] = in ? Xr[o + (long long)y * nx + k] : 0.0;
    im[j] = in ? Xi[o + (long long)y * nx + k] : 0.0;
  }
  __syncthreads();
  fft_stages(re, im, tw, n, cw);
  for (int e = threadIdx.x; e < cw * n; e += blockDim.x) {
    const int ky = e / cw, cc = e - ky * cw, k = k0 + cc;
    if (k < nx) Pc[o + (long long)ky * nx + k] = re[e] * re[e] + im[e] * im[e];
  }
}

static int log2_exact(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return (1 << l) == n ? l : -1;
}

int spectrum_shells(const Params& P) {
  const double hx = (double)(P.nx / 2), hy = (double)(P.ny / 2);
  return (int)llrint(sqrt(hx * hx + hy * hy)) + 1;
}

size_t spectrum_work_bytes(const Params& P) {
  const size_t N = (size_t)P.nx * (size_t)P.ny;
  return (size_t)(4 * P.dim) * N * sizeof(double);
}

bool spectrum_supported(const Params& P) { return P.nx <= SPEC_MAXN && P.ny <= SPEC_MAXN; }

hipError_t launch_spectrum(const Params& P, const double* U, int kz, double* E, void* work, hipStream_t s) {
  const long long N = (long long)P.nx * P.ny;
  double* Wp = (double*)work;
  double* Xr = Wp + (long long)P.dim * N;
  double* Xi = Xr + (long long)P.dim * N;
  double* Pc = Xi + (long long)P.dim * N;
  long long nb = (N * P.dim + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(k_spec_w, dim3((unsigned)nb), dim3(256), 0, s, P, U, kz, Wp);
  const int lx = log2_exact(P.nx), ly = log2_exact(P.ny);
  if (lx >= 0 && ly >= 0) {
    // rows: n/2 twiddles + n complex; columns: cw of them beside the
    // twiddles, cw = 4 (measured at 256^2: 31.9 us a call against 33.5,
    // 32.6 and 36.0 with 1, 2 and 8 columns; wider tiles leave too few
    // workgroups) or fewer within the 64 KB
    int cw = 4;
    while (cw > 1 && P.ny + 2 * cw * P.ny > FFT_LDS_DOUBLES) cw /= 2;
    hipLaunchKernelGGL(k_fft_rows, dim3((unsigned)P.ny, (unsigned)P.dim), dim3(256),
                       (size_t)3 * P.nx * sizeof(double), s, P, lx, Wp, Xr, Xi);
    hipLaunchKernelGGL(k_fft_cols, dim3((unsigned)((P.nx + cw - 1) / cw), (unsigned)P.dim), dim3(256),
                       (size_t)(P.ny + 2 * cw * P.ny) * sizeof(double), s, P, ly, cw, Xr, Xi, Pc);
  } else {
    const dim3 g((unsigned)((P.nx + 63) / 64), (unsigned)((P.ny + 15) / 16), (unsigned)P.dim);
    hipLaunchKernelGGL(k_spec_rows, g, dim3(256), (size_t)2 * P.nx * sizeof(double), s, P, Wp, Xr, Xi);
    hipLaunchKernelGGL(k_spec_cols, g, dim3(256), (size_t)2 * P.ny * sizeof(double), s, P, Xr, Xi, Pc);
  }
  hipLaunchKernelGGL(k_spec_shells, dim3((unsigned)spectrum_shells(P)), dim3(256), 0, s, P, Pc, E);
  return hipGetLastError();
}

}  // namespace ars
