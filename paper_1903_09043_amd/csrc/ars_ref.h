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
  R_L = 28, R_SB = 29, R_BT = 30,                                      // L, S-bar, 5 b~
  R_G = 35,                                                            // 3 axes x 5 fluxes
  R_US = 50,                                                           // (uS)_i (non-conservative energy)
  R_NFIELD = 51
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


// Whether face (a, l | l + e_a) is a wall (lz: vertical padded index of l):
// only the vertical axis has walls, between the last ghost and the first
// interior plane at the bottom and between the last interior and the first
// ghost plane at the top.
__device__ __forceinline__ bool ref_wall(const Params& P, int a, int lz) {
  return a == 2 && ((lz == 1 && P.bcz[0] == BC_WALL) || (lz == P.nz + 1 && P.bcz[1] == BC_WALL));
}

// velocity component k (0..DIM-1) -> primitive field
__device__ __forceinline__ int ufield(int DIM, int k) { return k == DIM - 1 ? R_UZ : (k == 0 ? R_UX : R_UY); }

}  // namespace ars
