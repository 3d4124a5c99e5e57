// ars_batch.hip -- many independent 2D problems (uneven sizes, own
// transport coefficients and time steps) advanced by ONE persistent launch.
//
// Each workgroup owns one instance for the whole run (instances are handed
// out largest first), marches its tiles plane by plane with the same device
// code as the fused step (march_tile), reduces the new-state rate inside the
// workgroup for its next dt, and uses the workgroup barrier as the
// instance's step barrier: there is no inter-workgroup waiting, so the
// launch can neither deadlock nor depend on co-residency, and one launch
// (optionally captured in a hipGraph) replaces n_inst x n_steps launches.
// Results equal those of ars_step on each instance bit for bit.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/ars.h"
#include "ars_dev.h"
#include "ars_fused.h"
#include "ars_internal.h"

namespace ars {

// Mutable per-instance record; the instance's Params live in a separate
// read-only array of the table so the kernel reads them through a
// non-aliased constant pointer (uniform loads) instead of a private copy.
struct BatchInst {
  double* U;
  double* tmp;
  double t;                       // in/out: accumulated time
  double dt;                      // out: next step's dt
  unsigned long long fault_cell;  // out: smallest faulting cell (~0: none)
  int nxs;                        // x segments of TX columns
  int zc;                         // vertical chunks (divides nz)
  int lm, diss, nc, pad_;
};

template <int NPOS>
__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    v = o > v ? o : v;
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = red[0];
  for (int w = 1; w < NPOS / 64; ++w) m = red[w] > m ? red[w] : m;
  __syncthreads();
  return m;
}

// One workgroup per instance, for all steps.  A step is split into
// nxs * zc units (x segment, vertical chunk) of equal plane count; the EY
// rows of the workgroup take EY units per pass (rows past the last unit
// march a copy that writes nothing).
template <bool LM, bool DISS, bool NC, int EX, int EY>
__global__ void __launch_bounds__(EX* EY) k_batch(BatchInst* insts, const Params* __restrict__ params,
                                                  const int* __restrict__ order, int nsteps) {
  constexpr int NPOS = EX * EY;
  using Ly = FusedLayout<2>;
  __shared__ double sm[Ly::TOTAL * NPOS];
  __shared__ double red[NPOS / 64];
  __shared__ unsigned long long badsh;
  const int k = order[blockIdx.x];
  BatchInst* I = &insts[k];
  if ((I->lm != 0) != LM || (I->diss != 0) != DISS || (I->nc != 0) != NC) return;  // another variant's instance
  const Params& P = params[k];
  const int tid = threadIdx.x;
  const int py = tid / EX;
  const int nxs = I->nxs;
  const int units = nxs * I->zc;
  const int chunk = P.nz / I->zc;
  double* src = I->U;
  double* dst = I->tmp;
  if (tid == 0) badsh = ~0ull;
  // rate of the initial state
  double r0 = 0.0;
  for (long long c = tid; c < P.ncell; c += NPOS) {
    double b[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) b[v] = src[c + v * P.ncell];
    const double l = cell_rate<2>(P, cons_to_prim<2>(P, b));
    r0 = l > r0 ? l : r0;
  }
  double rate = block_max<NPOS>(r0, red);
  double t = I->t;
  unsigned long long bad = ~0ull;
  for (int s = 0; s < nsteps; ++s) {
    const double dt = P.cfl / rate;
    const double lamx = dt / P.dx[0];
    const double lamz = dt / P.dx[2];
    double lmax = 0.0;
    for (int u0 = 0; u0 < units; u0 += EY) {
      const int u = u0 + py;
      const bool live = u < units;
      const int tx = live ? u % nxs : nxs;  // past the last segment: no output
      const int zs = live ? (u / nxs) * chunk : 0;
      march_tile<2, LM, DISS, NC, EX, EY>(P, src, dst, sm, tx, 0, zs, 0, chunk, lamx, 0.0, lamz, lmax, bad);
    }
    rate = block_max<NPOS>(lmax, red);  // its barriers complete the new state
    t = t + dt;
    double* w = src;
    src = dst;
    dst = w;
  }
  if (src != I->U) {
    for (long long c = tid; c < 4 * P.ncell; c += NPOS) I->U[c] = src[c];
  }
  if (bad != ~0ull) atomicMin(&badsh, bad);
  __syncthreads();
  if (tid == 0) {
    I->t = t;
    I->dt = P.cfl / rate;
    I->fault_cell = badsh;
  }
}

}  // namespace ars

namespace {

constexpr int BEX = 64;  // positions per row segment (60 output columns)
constexpr int BTX = BEX - 4;

// table: [BatchInst x n][Params x n][order: int x n]
size_t params_offset(int n) { return ((size_t)n * sizeof(ars::BatchInst) + 255) / 256 * 256; }
size_t order_offset(int n) { return params_offset(n) + ((size_t)n * sizeof(ars::Params) + 255) / 256 * 256; }
size_t table_bytes(int n) { return order_offset(n) + (size_t)n * sizeof(int) + 256; }

}  // namespace

int ars::batch_segments(const Params& P) { return (P.nx + BTX - 1) / BTX; }

// Vertical chunk count minimising the marched planes of one step for a
// workgroup of `rows` segments: passes * (planes per chunk + 4 halo
// iterations), over powers of two dividing nz with at least 4 planes each.
int ars::batch_default_zc(const Params& P, int rows) {
  const int nxs = batch_segments(P);
  long long best = -1;
  int bz = 1;
  for (int zc = 1; zc <= P.nz; zc *= 2) {
    if (P.nz % zc != 0 || P.nz / zc < 4) break;
    const long long passes = (nxs * zc + rows - 1) / rows;
    const long long cost = passes * (P.nz / zc + 4);
    if (best < 0 || cost < best) {
      best = cost;
      bz = zc;
    }
  }
  return bz;
}

namespace {

template <bool NC, int EY>
void launch_rows_nc(ars_batch* b, ars::BatchInst* insts, const ars::Params* params, const int* order, int nsteps,
                    const bool (&have)[2][2][2], hipStream_t s) {
  const dim3 grid(b->n), block(BEX * EY);
  if (have[NC][1][1])
    hipLaunchKernelGGL((ars::k_batch<true, true, NC, BEX, EY>), grid, block, 0, s, insts, params, order, nsteps);
  if (have[NC][1][0])
    hipLaunchKernelGGL((ars::k_batch<true, false, NC, BEX, EY>), grid, block, 0, s, insts, params, order, nsteps);
  if (have[NC][0][1])
    hipLaunchKernelGGL((ars::k_batch<false, true, NC, BEX, EY>), grid, block, 0, s, insts, params, order, nsteps);
  if (have[NC][0][0])
    hipLaunchKernelGGL((ars::k_batch<false, false, NC, BEX, EY>), grid, block, 0, s, insts, params, order, nsteps);
}

template <int EY>
void launch_rows(ars_batch* b, ars::BatchInst* insts, const ars::Params* params, const int* order, int nsteps,
                 hipStream_t s) {
  // each instance is advanced by the variant matching its (energy form,
  // theta, dissipation) flags; the other variants' workgroups return at once
  bool have[2][2][2] = {};
  for (int k = 0; k < b->n; ++k) have[b->P[k].nc != 0][b->P[k].low_mach != 0][b->P[k].diss != 0] = true;
  launch_rows_nc<false, EY>(b, insts, params, order, nsteps, have, s);
  launch_rows_nc<true, EY>(b, insts, params, order, nsteps, have, s);
}

hipError_t launch_batch(ars_batch* b, void* table, int nsteps, hipStream_t s) {
  char* base = (char*)table;
  ars::BatchInst* insts = (ars::BatchInst*)base;
  const ars::Params* params = (const ars::Params*)(base + params_offset(b->n));
  const int* order = (const int*)(base + order_offset(b->n));
  if (b->rows == 8)
    launch_rows<8>(b, insts, params, order, nsteps, s);
  else
    launch_rows<4>(b, insts, params, order, nsteps, s);
  return hipGetLastError();
}

void drop_graph(ars_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->captured = false;
}

}  // namespace

extern "C" {

int ars_batch_create(int n_inst, const ars_config* cfgs, ars_batch** out) {
  if (!out || n_inst < 1 || !cfgs) return ARS_EINVAL;
  *out = nullptr;
  ars_batch* b = new (std::nothrow) ars_batch;
  if (!b) return ARS_ENOMEM;
  b->n = n_inst;
  b->rows = 4;
  b->graph = nullptr;
  b->exec = nullptr;
  b->captured = false;
  size_t total = 0;
  for (int k = 0; k < n_inst; ++k) {
    const int rc = ars_validate(&cfgs[k]);
    if (rc != ARS_OK || cfgs[k].dim != 2) {
      delete b;
      return rc != ARS_OK ? rc : ARS_EUNSUPPORTED;
    }
    b->cfg.push_back(cfgs[k]);
    b->P.push_back(ars::params_of(&cfgs[k]));
    b->zc.push_back(ars::batch_default_zc(b->P.back(), b->rows));
    b->off.push_back(total);
    total += (size_t)4 * (size_t)b->P.back().ncell;
  }
  b->total = total;
  b->order.resize(n_inst);
  std::iota(b->order.begin(), b->order.end(), 0);
  std::stable_sort(b->order.begin(), b->order.end(),
                   [&](int a, int c) { return b->P[a].ncell > b->P[c].ncell; });
  *out = b;
  return ARS_OK;
}

void ars_batch_destroy(ars_batch* b) {
  if (!b) return;
  drop_graph(b);
  delete b;
}

size_t ars_batch_state_len(const ars_batch* b) { return b ? b->total : 0; }

size_t ars_batch_state_offset(const ars_batch* b, int k) {
  if (!b || k < 0 || k >= b->n) return 0;
  return b->off[k];
}

size_t ars_batch_table_bytes(const ars_batch* b) { return b ? table_bytes(b->n) : 0; }

int ars_batch_set_tiling(ars_batch* b, int rows, const int* zc) {
  if (!b || (rows != 4 && rows != 8)) return ARS_EINVAL;
  if (zc) {
    for (int k = 0; k < b->n; ++k) {
      const int z = zc[k];
      if (z < 1 || z > b->P[k].nz || b->P[k].nz % z != 0) return ARS_EINVAL;
    }
  }
  b->rows = rows;
  for (int k = 0; k < b->n; ++k) b->zc[k] = zc ? zc[k] : ars::batch_default_zc(b->P[k], rows);
  drop_graph(b);
  return ARS_OK;
}

int ars_batch_get_tiling(const ars_batch* b, int* rows, int* zc) {
  if (!b) return ARS_EINVAL;
  if (rows) *rows = b->rows;
  if (zc)
    for (int k = 0; k < b->n; ++k) zc[k] = b->zc[k];
  return ARS_OK;
}

int ars_batch_bind(ars_batch* b, double* d_states, double* d_tmps, void* d_table, void* stream) {
  if (!b || !d_states || !d_tmps || !d_table) return ARS_EINVAL;
  std::vector<char> h(table_bytes(b->n), 0);
  ars::BatchInst* insts = (ars::BatchInst*)h.data();
  ars::Params* params = (ars::Params*)(h.data() + params_offset(b->n));
  for (int k = 0; k < b->n; ++k) {
    ars::BatchInst& I = insts[k];
    params[k] = b->P[k];
    I.U = d_states + b->off[k];
    I.tmp = d_tmps + b->off[k];
    I.t = 0.0;
    I.dt = 0.0;
    I.fault_cell = ~0ull;
    I.nxs = ars::batch_segments(b->P[k]);
    I.zc = b->zc[k];
    I.lm = b->P[k].low_mach;
    I.diss = b->P[k].diss;
    I.nc = b->P[k].nc;
  }
  std::memcpy(h.data() + order_offset(b->n), b->order.data(), (size_t)b->n * sizeof(int));
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(d_table, h.data(), h.size(), hipMemcpyHostToDevice, s) != hipSuccess) return ARS_EDEVICE;
  return hipStreamSynchronize(s) == hipSuccess ? ARS_OK : ARS_EDEVICE;
}

int ars_batch_step(ars_batch* b, void* d_table, int n_steps, void* stream) {
  if (!b || !d_table || n_steps < 0) return ARS_EINVAL;
  if (n_steps == 0) return ARS_OK;
  return launch_batch(b, d_table, n_steps, (hipStream_t)stream) == hipSuccess ? ARS_OK : ARS_EDEVICE;
}

int ars_batch_capture(ars_batch* b, void* d_table, int n_steps, void* stream) {
  if (!b || !d_table || n_steps < 1 || !stream) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  drop_graph(b);
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) return ARS_EDEVICE;
  const hipError_t le = launch_batch(b, d_table, n_steps, s);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(s, &g);
  if (le != hipSuccess || ee != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return ARS_EDEVICE;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    drop_graph(b);
    return ARS_EDEVICE;
  }
  b->captured = true;
  return ARS_OK;
}

int ars_batch_replay(ars_batch* b, void* stream) {
  if (!b || !b->captured) return ARS_EINVAL;
  return hipGraphLaunch(b->exec, (hipStream_t)stream) == hipSuccess ? ARS_OK : ARS_EDEVICE;
}

int ars_batch_read(const ars_batch* b, const void* d_table, double* h_t, double* h_dt, int64_t* h_fault_cell,
                   void* stream) {
  if (!b || !d_table) return ARS_EINVAL;
  std::vector<ars::BatchInst> h(b->n);
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(h.data(), d_table, (size_t)b->n * sizeof(ars::BatchInst), hipMemcpyDeviceToHost, s) !=
      hipSuccess)
    return ARS_EDEVICE;
  if (hipStreamSynchronize(s) != hipSuccess) return ARS_EDEVICE;
  int rc = ARS_OK;
  for (int k = 0; k < b->n; ++k) {
    if (h_t) h_t[k] = h[k].t;
    if (h_dt) h_dt[k] = h[k].dt;
    const bool f = h[k].fault_cell != ~0ull;
    if (h_fault_cell) h_fault_cell[k] = f ? (int64_t)h[k].fault_cell : -1;
    if (f) rc = ARS_ENONPHYS;
  }
  return rc;
}

}  // extern "C"
