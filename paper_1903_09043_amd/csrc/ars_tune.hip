// ars_tune.hip -- autotuner of the launch shapes: times candidate tilings
// of the fused step (vertical share per workgroup, resident workgroups per
// CU) and of the batched launch (row segments per workgroup, vertical
// chunking policy) on the caller's own problem, keeps the fastest, and
// remembers it in an optional text cache keyed by device and problem
// shape.  Results never depend on the tiling (every candidate computes the
// same bits), only time does.
//
// Cache file: one entry per line, "<key> <a> <b> <ms_per_step>", later lines
// winning.  Keys name the device (architecture, compute units) and what
// determines the kernel's work: dimension, grid, boundary kinds, theta and
// dissipation switches (step), or a hash of every instance's shape and
// switches (batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ars.h"
#include "ars_internal.h"

namespace {

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + ":cu" + std::to_string(prop.multiProcessorCount);
}

bool cache_lookup(const char* path, const std::string& key, int* a, int* b, double* ms, int* c = nullptr) {
  if (!path || !path[0]) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    char k[768];
    int x = 0, y = 0, z = 0;
    double m = 0.0;
    const int got = std::sscanf(line, "%767s %d %d %lf %d", k, &x, &y, &m, &z);
    if (got >= 4 && key == k) {
      *a = x;
      *b = y;
      *ms = m;
      if (c) *c = got == 5 ? z : 0;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void cache_store(const char* path, const std::string& key, int a, int b, double ms, int c = -1) {
  if (!path || !path[0]) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  if (c >= 0)
    std::fprintf(f, "%s %d %d %.6f %d\n", key.c_str(), a, b, ms, c);
  else
    std::fprintf(f, "%s %d %d %.6f\n", key.c_str(), a, b, ms);
  std::fclose(f);
}

uint64_t fnv1a(uint64_t h, long long v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (uint64_t)((v >> (8 * i)) & 0xff);
    h *= 0x100000001b3ULL;
  }
  return h;
}

// Milliseconds per step of `run(steps)` on stream s, after one untimed call.
template <class F>
int time_ms(F run, int steps, hipStream_t s, double* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return ARS_EDEVICE;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return ARS_EDEVICE;
  }
  int rc = run(1);
  if (rc == ARS_OK && hipEventRecord(e0, s) != hipSuccess) rc = ARS_EDEVICE;
  if (rc == ARS_OK) rc = run(steps);
  if (rc == ARS_OK && hipEventRecord(e1, s) != hipSuccess) rc = ARS_EDEVICE;
  float t = 0.f;
  if (rc == ARS_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess))
    rc = ARS_EDEVICE;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = (double)t / steps;
  return rc;
}

}  // namespace

extern "C" {

int ars_autotune(ars_ctx* ctx, const double* d_state, void* d_work, int trial_steps, const char* cache_path,
                 void* stream, ars_tune_result* out) {
  if (!ctx || !d_state || !d_work || trial_steps < 1) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const ars::Params& P = ctx->P;
  std::string key = "step:" + device_tag() + ":d" + std::to_string(P.dim) + ":" + std::to_string(P.nx) + "x" +
                    std::to_string(P.ny) + "x" + std::to_string(P.nz) + ":bc" + std::to_string(P.bcx[0]) +
                    std::to_string(P.bcy[0]) + std::to_string(P.bcz[0]) + ":lm" + std::to_string(P.low_mach) +
                    ":diss" + std::to_string(P.diss);
  ars_tune_result r{};
  int za = 0, wb = 0, tc = 0;
  double ms = 0.0;
  if (cache_lookup(cache_path, key, &za, &wb, &ms, &tc) && za >= 1 && wb >= 0 && (tc == 0 || (tc == 1 && P.dim == 3))) {
    ctx->ts.tile3 = tc;
    ctx->ts.zchunk = za;
    ctx->ts.wg_per_cu = wb;
    r.tile3 = tc;
    r.zchunk = za;
    r.wg_per_cu = wb;
    r.ms_per_step = ms;
    r.from_cache = 1;
    if (out) *out = r;
    return ARS_OK;
  }
  // candidates: the 3D tiles; for each, vertical shares per workgroup
  // around that tile's default; workgroups per CU (0 = as many as are
  // resident at once, else that many per CU, queued beyond residency)
  std::vector<int> tiles = {ctx->ts.tile3};
  if (P.dim == 3) tiles = {0, 1};
  std::vector<int> ws = {0, 2, 4};
  if (P.dim == 2) ws = {0, 4, 8, 16};
  double* buf = nullptr;
  double* dd = nullptr;
  const size_t bytes = ctx->len * sizeof(double);
  if (hipMalloc((void**)&buf, 2 * bytes + 4 * sizeof(double)) != hipSuccess) return ARS_EDEVICE;
  double* A = buf;
  double* B = buf + ctx->len;
  dd = buf + 2 * ctx->len;  // t, dt
  const ars::TileShape keep = ctx->ts;
  int rc = ARS_OK;
  double best = -1.0;
  ars::TileShape bestts = keep;
  int ncand = 0;
  for (int tl : tiles) {
    std::vector<int> zs;
    const int z0 = tl == keep.tile3 ? keep.zchunk : ars::default_zchunk(P, tl);
    for (int z : {z0, 1, 2, 4, 8, 16, 32, 64, std::max(1, z0 / 2), z0 * 2})
      if (z >= 1 && z <= P.nz && std::find(zs.begin(), zs.end(), z) == zs.end()) zs.push_back(z);
    for (int z : zs) {
      for (int w : ws) {
        ctx->ts.tile3 = tl;
        ctx->ts.zchunk = z;
        ctx->ts.wg_per_cu = w;
        // every candidate starts from the caller's state
        if (hipMemcpyAsync(A, d_state, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) rc = ARS_EDEVICE;
        if (rc == ARS_OK) rc = ars_compute_dt(ctx, A, d_work, dd + 1, s);
        double m = 0.0;
        if (rc == ARS_OK)
          rc = time_ms([&](int n) { return ars_step(ctx, A, B, d_work, n, dd, dd + 1, nullptr, s); }, trial_steps,
                       s, &m);
        if (rc != ARS_OK) break;
        ++ncand;
        if (best < 0.0 || m < best) {
          best = m;
          bestts = ctx->ts;
        }
      }
      if (rc != ARS_OK) break;
    }
    if (rc != ARS_OK) break;
  }
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (rc != ARS_OK) {
    ctx->ts = keep;
    return rc;
  }
  // the trial runs used the workspace's rate slots and fault latch
  rc = ars_workspace_init(ctx, d_work, stream);
  if (rc != ARS_OK) {
    ctx->ts = keep;
    return rc;
  }
  ctx->ts = bestts;
  cache_store(cache_path, key, bestts.zchunk, bestts.wg_per_cu, best, bestts.tile3);
  r.tile3 = bestts.tile3;
  r.zchunk = bestts.zchunk;
  r.wg_per_cu = bestts.wg_per_cu;
  r.ms_per_step = best;
  r.n_candidates = ncand;
  if (out) *out = r;
  return ARS_OK;
}

int ars_batch_autotune(ars_batch* b, double* d_states, double* d_tmps, void* d_table, int trial_steps,
                       const char* cache_path, void* stream, ars_tune_result* out) {
  if (!b || !d_states || !d_tmps || !d_table || trial_steps < 1) return ARS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  uint64_t h = 0xcbf29ce484222325ULL;
  for (int k = 0; k < b->n; ++k) {
    h = fnv1a(h, b->P[k].nx);
    h = fnv1a(h, b->P[k].nz);
    h = fnv1a(h, b->P[k].low_mach * 2 + b->P[k].diss);
    h = fnv1a(h, b->P[k].bcx[0] * 16 + b->P[k].bcz[0]);
  }
  char hx[32];
  std::snprintf(hx, sizeof hx, "%016llx", (unsigned long long)h);
  const std::string key = "batch:" + device_tag() + ":n" + std::to_string(b->n) + ":" + hx;
  // policies: 0 cost model, 1 no vertical chunks, 2 twice the model's
  // chunks (when they divide nz), 3 half the model's chunks
  auto policy_zc = [&](int pol, int rows) {
    std::vector<int> zc(b->n);
    for (int k = 0; k < b->n; ++k) {
      const int m = ars::batch_default_zc(b->P[k], rows);
      int z = m;
      if (pol == 1) z = 1;
      if (pol == 2 && b->P[k].nz % (2 * m) == 0 && b->P[k].nz / (2 * m) >= 2) z = 2 * m;
      if (pol == 3) z = std::max(1, m / 2);
      zc[k] = z;
    }
    return zc;
  };
  ars_tune_result r{};
  int ra = 0, pb = 0;
  double ms = 0.0;
  int rc = ARS_OK;
  if (cache_lookup(cache_path, key, &ra, &pb, &ms) && (ra == 4 || ra == 8) && pb >= 0 && pb <= 3) {
    const std::vector<int> zc = policy_zc(pb, ra);
    rc = ars_batch_set_tiling(b, ra, zc.data());
    if (rc == ARS_OK) rc = ars_batch_bind(b, d_states, d_tmps, d_table, stream);
    r.rows = ra;
    r.zc_policy = pb;
    r.ms_per_step = ms;
    r.from_cache = 1;
    if (out) *out = r;
    return rc;
  }
  const size_t bytes = b->total * sizeof(double);
  double* save = nullptr;
  if (hipMalloc((void**)&save, bytes) != hipSuccess) return ARS_EDEVICE;
  if (hipMemcpyAsync(save, d_states, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) rc = ARS_EDEVICE;
  double best = -1.0;
  int brow = b->rows, bpol = 0, ncand = 0;
  for (int rows : {4, 8}) {
    for (int pol = 0; pol < 4 && rc == ARS_OK; ++pol) {
      const std::vector<int> zc = policy_zc(pol, rows);
      if (pol > 0 && zc == policy_zc(0, rows)) continue;  // same as the model
      rc = ars_batch_set_tiling(b, rows, zc.data());
      if (rc == ARS_OK) rc = ars_batch_bind(b, d_states, d_tmps, d_table, stream);
      if (rc == ARS_OK && hipMemcpyAsync(d_states, save, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
        rc = ARS_EDEVICE;
      double m = 0.0;
      if (rc == ARS_OK)
        rc = time_ms([&](int n) { return ars_batch_step(b, d_table, n, stream); }, trial_steps, s, &m);
      if (rc != ARS_OK) break;
      ++ncand;
      if (best < 0.0 || m < best) {
        best = m;
        brow = rows;
        bpol = pol;
      }
    }
  }
  if (rc == ARS_OK && hipMemcpyAsync(d_states, save, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess)
    rc = ARS_EDEVICE;
  (void)hipStreamSynchronize(s);
  (void)hipFree(save);
  if (rc != ARS_OK) return rc;
  const std::vector<int> zc = policy_zc(bpol, brow);
  rc = ars_batch_set_tiling(b, brow, zc.data());
  if (rc == ARS_OK) rc = ars_batch_bind(b, d_states, d_tmps, d_table, stream);
  if (rc != ARS_OK) return rc;
  cache_store(cache_path, key, brow, bpol, best);
  r.rows = brow;
  r.zc_policy = bpol;
  r.ms_per_step = best;
  r.n_candidates = ncand;
  if (out) *out = r;
  return ARS_OK;
}

}  // extern "C"
