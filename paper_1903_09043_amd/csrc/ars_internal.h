// ars_internal.h -- host/device interfaces between the library's translation
// units (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include "ars_dev.h"

namespace ars {

// Per-launch inputs/outputs of one fused step.
struct StepIO {
  const unsigned long long* rate_in;  // dt = cfl / rate (if non-null)
  const double* dt_in;                // else dt = *dt_in
  unsigned long long* rate_out;       // atomic max of the new state's rates (nullable)
  unsigned long long* clear_slot;     // zeroed by one thread (slot used two steps later)
  double* t;                          // t += dt (nullable)
  double* dt_log;                     // dt written here (nullable)
  Control* ctl;                       // fault latch
  int zchunk, ntx, nty;
};

struct TileShape {
  int zchunk;     // minimum share of planes per workgroup
  int num_cu;     // compute units of the device (queried at first launch)
  int wg_per_cu;  // resident workgroups per CU of the chosen kernel
};

hipError_t launch_step_fused(const Params& P, const double* Uin, double* Uout, StepIO io, const TileShape& ts,
                             hipStream_t s);

// Reference (phase-by-phase) step on padded arrays; see ars_ref.hip.
size_t ref_workspace_bytes(const Params& P);
hipError_t launch_step_ref(const Params& P, const double* Uin, double* Uout, void* wref, const double* d_dt,
                           Control* ctl, hipStream_t s);

// Reductions (ars_reduce.hip).
hipError_t launch_rate_reduce(const Params& P, const double* U, unsigned long long* slot, hipStream_t s);
hipError_t launch_ctl_prep(Control* ctl, int mode, hipStream_t s);
hipError_t launch_dt_finish(const Params& P, Control* ctl, int slot, double* d_dt, hipStream_t s);
size_t diag_partial_bytes(const Params& P);
hipError_t launch_diag(const Params& P, const double* U, double* partials, double* out, hipStream_t s);

}  // namespace ars
