// ars_internal.h -- host/device interfaces between the library's translation
// units (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <vector>

#include "../../include/ars.h"
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

// Tiles of the 3D fused step (positions = outputs + the 2-cell halo on
// each side): ARS_TILE3_32x10 and ARS_TILE3_16x20 of include/ars.h.
constexpr int TILE3_EX[2] = {36, 20};
constexpr int TILE3_EY[2] = {14, 24};

struct TileShape {
  int tile3;      // 3D tile (index into TILE3_EX / TILE3_EY)
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
// forward phases only (primitives, faces, acoustic cell values) into wref
hipError_t launch_ref_forward(const Params& P, const double* Uin, void* wref, const double* d_dt, hipStream_t s);
// face fluxes and update from the faces and cell values in wref
hipError_t launch_ref_finish(const Params& P, void* wref, double* Uout, const double* d_dt, Control* ctl,
                             hipStream_t s);

// Implicit acoustic (IMEX) step (ars_imex.hip).
size_t imex_workspace_bytes(const Params& P);
int step_imex(const Params& P, double* d_state, double* d_tmp, Control* ctl, void* wimex, int nsteps,
              const double* d_dt_sched, double* d_t, double tol, int max_iter, int* h_iters, hipStream_t s);

// Adjoint step: the fused marches (ars_adjf.hip) where adjf_supported,
// else the phase kernels (ars_adjoint.hip), which are also the reference.
size_t adjoint_workspace_bytes(const Params& P);
hipError_t launch_step_adjoint(const Params& P, const double* Un, const double* lam_np1, double* lam_n,
                               const double* d_dt, double* d_param_grad, void* wadj, hipStream_t s);
size_t adjoint_ref_workspace_bytes(const Params& P);
hipError_t launch_step_adjoint_ref(const Params& P, const double* Un, const double* lam_np1, double* lam_n,
                                   const double* d_dt, double* d_param_grad, void* wadj, hipStream_t s);
bool adjf_supported(const Params& P);
size_t adjf_workspace_bytes(const Params& P);
hipError_t launch_step_adjoint_fused(const Params& P, const double* Un, const double* lam_np1, double* lam_n,
                                     const double* d_dt, double* d_param_grad, void* wadj, hipStream_t s);
hipError_t launch_adj_params_final(int nb, const double* partial, double* pgrad, hipStream_t s);

// Derived kernel parameters of a validated configuration (ars_api.hip).
Params params_of(const ars_config* c);
// Default vertical share per workgroup of the fused step for a tile.
int default_zchunk(const Params& P, int tile3);

// Batched problems (ars_batch.hip): x segments of one instance and the
// cost-model vertical chunk count for `rows` segments per workgroup.
int batch_segments(const Params& P);
int batch_default_zc(const Params& P, int rows);

// Reductions (ars_reduce.hip).
hipError_t launch_rate_reduce(const Params& P, const double* U, unsigned long long* slot, hipStream_t s);
hipError_t launch_ctl_prep(Control* ctl, int mode, hipStream_t s);
hipError_t launch_dt_finish(const Params& P, Control* ctl, int slot, double* d_dt, hipStream_t s);
size_t diag_partial_bytes(const Params& P);
hipError_t launch_diag(const Params& P, const double* U, double* partials, double* out, hipStream_t s);
hipError_t launch_ke(const Params& P, const double* U, double* grad, double* partials, double* out, hipStream_t s);
hipError_t launch_nusselt(const Params& P, int side, double C, const double* U, double* grad, double* partials,
                          double* out, hipStream_t s);
int spectrum_shells(const Params& P);
size_t spectrum_work_bytes(const Params& P);
bool spectrum_supported(const Params& P);
hipError_t launch_spectrum(const Params& P, const double* U, int kz, double* E, void* work, hipStream_t s);

}  // namespace ars

struct ars_ctx {
  ars_config cfg;
  ars::Params P;
  ars::TileShape ts;
  size_t len;
};

struct ars_batch {
  int n;
  int rows;                   // row segments per workgroup (4 or 8)
  std::vector<ars_config> cfg;
  std::vector<ars::Params> P;
  std::vector<int> zc;        // vertical chunks per instance
  std::vector<size_t> off;    // state offsets (doubles)
  std::vector<int> order;     // largest first
  size_t total;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool captured;
};
