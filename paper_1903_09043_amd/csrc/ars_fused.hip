// ars_fused.hip -- fused explicit step of the all-regime, well-balanced
// scheme (arXiv 1903.09043, eq. all_regime_scheme with the dissipative
// fluxes of Sec. 2.2 and the relaxation step of Sec. 2.1.4) for gfx950.
//
// Design (MI355X-first, not the paper's flat Kokkos loop):
//  * One workgroup owns a tile of TX x TY columns (2D: TX columns) plus a
//    2-cell halo and marches along the vertical (gravity) axis.  The stencil
//    of one update is the radius-2 diamond (the upwinded transport value
//    b~ of a neighbour needs all faces of that neighbour), so the halo is 2.
//  * The vertical neighbours live in registers (a rolling window of planes);
//    lateral neighbours are exchanged through LDS once per plane:
//      XA  acoustic fields (rho c, c, p, u_lat) of the newest plane p
//      V   u, T of plane p-1 (viscous stencil), DZ  u(p) - u(p-2)
//      F   own +x/+y acoustic faces (u*, Pi*, Pi* u*) of plane p
//      B   transported values b~ of plane p-1
//      GX  own +x/+y total face fluxes of plane p-1
//    Per plane: faces at p, acoustic cell values at p-1, fluxes at p-1 and
//    the update of plane p-2; 2 barriers per plane.
//  * Every face is evaluated once; the only HBM traffic is the read of U^n
//    and the write of U^{n+1} (plus halo re-reads that hit L2).
//  * Epilogue: the rate of the NEW state for the next CFL time step is
//    reduced wave -> LDS -> one atomicMax per workgroup, so dt never leaves
//    the device and n steps need no host synchronisation.
//  * No MFMA: nothing here is a contraction.

#include "ars_fused.h"

namespace ars {

template <int DIM, bool LM, bool DISS, bool NC, int EX, int EY>
__global__ void __launch_bounds__(EX* EY) k_step_fused(Params P, const double* __restrict__ Uin,
                                                       double* __restrict__ Uout, StepIO io) {
  constexpr int NPOS = EX * EY;
  using Ly = FusedLayout<DIM>;
  __shared__ double sm[Ly::TOTAL * NPOS];
  constexpr int NW = (NPOS + 63) / 64;  // waves (the last one partial if 64 does not divide NPOS)
  __shared__ double red[NW];

  const int tid = threadIdx.x;
  // time step of this step
  double dt;
  if (io.rate_in)
    dt = P.cfl / __longlong_as_double((long long)*io.rate_in);
  else
    dt = *io.dt_in;
  const double lamx = dt / P.dx[0];
  const double lamy = (DIM == 3) ? dt / P.dx[1] : 0.0;
  const double lamz = dt / P.dx[2];
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) {
    if (io.clear_slot) *io.clear_slot = 0ull;
    if (io.t) *io.t = *io.t + dt;
    if (io.dt_log) *io.dt_log = dt;
  }

  // Persistent balanced schedule: the (tile, plane) pairs are laid end to
  // end (tile-major) and every workgroup takes one contiguous share; shares
  // of neighbouring workgroups on one XCD are neighbours in space, so halo
  // re-reads hit that XCD's L2.
  const long long total = (long long)io.ntx * io.nty * P.nz;
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int lw = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  long long cur = total * lw / G;
  const long long stop = total * (lw + 1) / G;
  double lmax = 0.0;
  unsigned long long badcell = ~0ull;
  while (cur < stop) {
    const int tile = (int)(cur / P.nz);
    const int z0 = (int)(cur % P.nz);
    const int z1 = (int)min((long long)P.nz, (long long)z0 + (stop - cur));
    cur += z1 - z0;
    const int tx = (DIM == 3) ? tile % io.ntx : tile * EY + (int)threadIdx.x / EX;
    const int ty = (DIM == 3) ? tile / io.ntx : 0;
    march_tile<DIM, LM, DISS, NC, EX, EY>(P, Uin, Uout, sm, tx, ty, 0, z0, z1, lamx, lamy, lamz, lmax, badcell);
  }

  // ---- workgroup reduction of the new-state rate, fault latch --------------
  if (badcell != ~0ull) {
    atomicOr(&io.ctl->fault, 1u);
    atomicMin(&io.ctl->fault_cell, badcell);
  }
  if (io.rate_out) {
    double m = lmax;
    if (NPOS % 64 != 0) {
      // a partial last wave has no lanes past NPOS to shuffle with: gather
      // every position's rate into wave 0 through LDS (free after the march)
      __syncthreads();
      sm[tid] = lmax;
      __syncthreads();
      m = 0.0;
      if (tid < 64)
        for (int j = tid; j < NPOS; j += 64) m = sm[j] > m ? sm[j] : m;
    }
    if (NPOS % 64 == 0 || tid < 64) {
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const double o2 = __shfl_xor(m, off, 64);
        m = o2 > m ? o2 : m;
      }
      if ((tid & 63) == 0) red[tid >> 6] = m;
    }
    __syncthreads();
    if (tid == 0) {
      double mm = red[0];
      for (int w = 1; w < (NPOS % 64 == 0 ? NW : 1); ++w) mm = red[w] > mm ? red[w] : mm;
      atomic_max_rate(io.rate_out, mm);
    }
  }
}

// --------------------------------------------------------------------------
// Host-side launch
// --------------------------------------------------------------------------
template <int DIM, bool LM, bool DISS, bool NC, int EX, int EY>
static hipError_t launch_fused_t(const Params& P, const double* Uin, double* Uout, StepIO io, const TileShape& ts,
                                 hipStream_t s) {
  constexpr int TX = EX - 4;
  constexpr int TY = (DIM == 3) ? EY - 4 : 1;
  io.ntx = (DIM == 3) ? (P.nx + TX - 1) / TX : (P.nx + TX * EY - 1) / (TX * EY);
  io.nty = (DIM == 3) ? (P.ny + TY - 1) / TY : 1;
  io.zchunk = ts.zchunk;
  const long long total = (long long)io.ntx * io.nty * P.nz;
  // one workgroup per (CU x resident blocks), each with an equal share of
  // planes; never more workgroups than shares of at least zchunk planes
  static int occ = 0;  // resident blocks per CU of this instance
  if (occ == 0) {
    int o = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, k_step_fused<DIM, LM, DISS, NC, EX, EY>, EX * EY, 0) !=
            hipSuccess ||
        o < 1)
      o = 1;
    occ = o;
  }
  int ncu = ts.num_cu;
  if (ncu <= 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
      ncu = 256;
  }
  long long nwg = (long long)(ts.wg_per_cu > 0 ? ts.wg_per_cu : occ) * ncu;
  const long long by_chunk = (total + ts.zchunk - 1) / ts.zchunk;
  if (by_chunk < nwg) nwg = by_chunk;
  if (nwg < 1) nwg = 1;
  hipLaunchKernelGGL((k_step_fused<DIM, LM, DISS, NC, EX, EY>), dim3((unsigned)nwg), dim3(EX * EY), 0, s, P, Uin, Uout,
                     io);
  return hipGetLastError();
}

template <int DIM, bool NC, int EX, int EY>
static hipError_t launch_variant(const Params& P, const double* Uin, double* Uout, StepIO io, const TileShape& ts,
                                 hipStream_t s) {
  const bool lm = P.low_mach != 0, ds = P.diss != 0;
  if (lm && ds) return launch_fused_t<DIM, true, true, NC, EX, EY>(P, Uin, Uout, io, ts, s);
  if (lm && !ds) return launch_fused_t<DIM, true, false, NC, EX, EY>(P, Uin, Uout, io, ts, s);
  if (!lm && ds) return launch_fused_t<DIM, false, true, NC, EX, EY>(P, Uin, Uout, io, ts, s);
  return launch_fused_t<DIM, false, false, NC, EX, EY>(P, Uin, Uout, io, ts, s);
}

hipError_t launch_step_fused(const Params& P, const double* Uin, double* Uout, StepIO io, const TileShape& ts,
                             hipStream_t s) {
  if (P.dim == 2)
    return P.nc ? launch_variant<2, true, 64, 1>(P, Uin, Uout, io, ts, s)
                : launch_variant<2, false, 64, 1>(P, Uin, Uout, io, ts, s);
  if (ts.tile3 == 1)
    return P.nc ? launch_variant<3, true, TILE3_EX[1], TILE3_EY[1]>(P, Uin, Uout, io, ts, s)
                : launch_variant<3, false, TILE3_EX[1], TILE3_EY[1]>(P, Uin, Uout, io, ts, s);
  return P.nc ? launch_variant<3, true, TILE3_EX[0], TILE3_EY[0]>(P, Uin, Uout, io, ts, s)
              : launch_variant<3, false, TILE3_EX[0], TILE3_EY[0]>(P, Uin, Uout, io, ts, s);
}

}  // namespace ars
