// ars_noalloc.hip -- ars_step_noalloc: the fused step with its scratch in a
// static device array of the library instead of caller buffers, for callers
// that cannot allocate device memory (code under graph capture, tight
// serving loops).
//
// The scratch of ars_step is a 256-byte control block (rate slots for the
// CFL maximum, fault latch) in the caller's workspace plus a second state
// buffer for the ping-pong of the march.  Here both live in `scratch`: the
// control block first, then room for a ping-pong state of at most
// ARS_NOALLOC_MAX_STATE doubles.  The kernels are those of ars_step.
//
// `scratch` names a host-side stand-in in host code; the device address of
// each GPU's copy is taken once per device with hipGetSymbolAddress (at the
// first call on that device, with that device current) and only that
// address is ever handed to a kernel or a copy.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/ars.h"
#include "ars_internal.h"

namespace {

constexpr size_t CTL_BYTES = 256;
constexpr size_t SCRATCH_BYTES = CTL_BYTES + (size_t)ARS_NOALLOC_MAX_STATE * sizeof(double);
static_assert(sizeof(ars::Control) <= CTL_BYTES, "control block exceeds its slot");

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {};

// Device address of this device's `scratch` (resolved once per device).
int scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) return ARS_EDEVICE;
  if (dev >= MAX_DEVICES) return ARS_EUNSUPPORTED;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ARS_EDEVICE;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return ARS_OK;
}

// Whole control block to its start values: rate slots 0, no fault.  A kernel
// rather than a memset, so that the call can be captured in a graph.
__global__ void k_noalloc_prep(ars::Control* ctl) {
  if (threadIdx.x == 0) {
    for (int i = 0; i < 4; ++i) ctl->lammax[i] = 0ull;
    ctl->fault = 0u;
    ctl->fault_cell = ~0ull;
  }
}

// Next dt from the last step's rate slot, NaN if a fault was latched.
__global__ void k_noalloc_finish(double cfl, const ars::Control* ctl, int slot, double* d_dt) {
  if (threadIdx.x == 0)
    *d_dt = ctl->fault ? __builtin_nan("") : cfl / __longlong_as_double((long long)ctl->lammax[slot]);
}

}  // namespace

extern "C" int ars_step_noalloc(ars_ctx* ctx, double* d_state, int n, double* d_t, double* d_dt, double* d_dt_log,
                                void* stream) {
  if (!ctx || !d_state || !d_dt || n < 0) return ARS_EINVAL;
  if (ctx->len > (size_t)ARS_NOALLOC_MAX_STATE) return ARS_ESCRATCH;
  if (n == 0) return ARS_OK;
  void* base = nullptr;
  const int rc = scratch_ptr(&base);
  if (rc != ARS_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  ars::Control* ctl = (ars::Control*)base;
  double* tmp = (double*)((char*)base + CTL_BYTES);
  hipLaunchKernelGGL(k_noalloc_prep, dim3(1), dim3(64), 0, s, ctl);
  if (hipGetLastError() != hipSuccess) return ARS_EDEVICE;
  double* src = d_state;
  double* dst = tmp;
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
    double* w = src;
    src = dst;
    dst = w;
  }
  if (src != d_state) {
    if (hipMemcpyAsync(d_state, src, ctx->len * sizeof(double), hipMemcpyDeviceToDevice, s) != hipSuccess)
      return ARS_EDEVICE;
  }
  hipLaunchKernelGGL(k_noalloc_finish, dim3(1), dim3(64), 0, s, ctx->P.cfl, (const ars::Control*)ctl, n % 3, d_dt);
  return hipGetLastError() == hipSuccess ? ARS_OK : ARS_EDEVICE;
}
