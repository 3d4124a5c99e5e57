// ars_ref.h -- padded-grid layout shared by the phase-by-phase reference
// step and the adjoint step (two ghost layers per active axis).
#pragma once
#include "ars_dev.h"

namespace ars {

struct RefGrid {
  int D;
  int Px, Py, Pz;      // padded extents (Py = 1 in 2D)
  long long npad;
  __host__ __device__ long long pad(int qx, int qy, int qz) const {
    return qx + (long long)Px * (qy + (long long)Py * qz);
  }
};

// Field offsets (in units of npad doubles) inside the reference workspace.
enum {
  R_RHO = 0, R_R, R_UX, R_UY, R_UZ, R_P, R_C, R_RC, R_T, R_IC, R_IRC,  // primitives (11)
  R_CONS = 11,                                                         // 5 conserved
  R_FACE = 16,                                                         // 3 axes x (us, pi, P, S)
  R_WALL = 28,                                                         // 3 axes wall flags (as doubles)
  R_L = 31, R_SB = 32, R_BT = 33,                                      // L, S-bar, 5 b~
  R_G = 38,                                                            // 3 axes x 5 fluxes
  R_US = 53,                                                           // (uS)_i (non-conservative energy)
  R_NFIELD = 54
};

inline RefGrid make_grid(const Params& P) {
  RefGrid G;
  G.D = P.dim;
  G.Px = P.nx + 4;
  G.Py = (P.dim == 3) ? P.ny + 4 : 1;
  G.Pz = P.nz + 4;
  G.npad = (long long)G.Px * G.Py * G.Pz;
  return G;
}


__device__ __forceinline__ void decode(const RefGrid& G, long long i, int& qx, int& qy, int& qz) {
  qx = (int)(i % G.Px);
  long long r = i / G.Px;
  qy = (int)(r % G.Py);
  qz = (int)(r / G.Py);
}

// axis helpers: a = 0 (x), 1 (y, 3D only), 2 (vertical)
__device__ __forceinline__ long long astride(const RefGrid& G, int a) {
  return a == 0 ? 1 : (a == 1 ? (long long)G.Px : (long long)G.Px * G.Py);
}


// velocity component k (0..DIM-1) -> primitive field
__device__ __forceinline__ int ufield(int DIM, int k) { return k == DIM - 1 ? R_UZ : (k == 0 ? R_UX : R_UY); }

}  // namespace ars
