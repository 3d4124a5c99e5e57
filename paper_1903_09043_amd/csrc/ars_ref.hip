// ars_ref.hip -- the same explicit step as separate phase kernels on padded
// arrays (two ghost layers), each phase one thread per cell or face:
//   ghosts + primitives -> acoustic faces and cell values (L, b~), one
//   pass -> total face fluxes -> update (+ relaxation E = calE - rho Phi).
// It stores every intermediate in the workspace and exists to check the
// fused kernels bit for bit (and to expose the intermediates to tests).
#include "ars_dev.h"
#include "ars_internal.h"
#include "ars_ref.h"

namespace ars {

size_t ref_workspace_bytes(const Params& P) {
  RefGrid G = make_grid(P);
  return (size_t)R_NFIELD * (size_t)G.npad * sizeof(double);
}

template <int DIM>
__global__ void k_ref_prim(Params P, RefGrid G, const double* __restrict__ U, double* __restrict__ W) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.npad) return;
  constexpr int NV = DIM + 2;
  int qx, qy, qz;
  decode(G, i, qx, qy, qz);
  const int cx = resolve_lat(qx - 2, P.nx, P.bcx);
  const int cy = (DIM == 3) ? resolve_lat(qy - 2, P.ny, P.bcy) : 0;
  int kz = qz - 2;
  int ghost = -1;
  if (kz < 0 || kz >= P.nz) {
    const int side = kz < 0 ? 0 : 1;
    if (P.bcz[side] == BC_WALL) {
      ghost = side;
      kz = side == 0 ? 0 : P.nz - 1;
    } else {
      kz = resolve_lat(kz, P.nz, P.bcz);
    }
  }
  const long long cell = cx + (long long)P.nx * (cy + (long long)P.ny * kz);
  double b[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) b[v] = U[cell + v * P.ncell];
  Prim<DIM> q = cons_to_prim<DIM>(P, b);
  if (ghost >= 0) {
    const int kg = ghost == 0 ? -1 : P.nz;
    q = wall_ghost<DIM>(P, q, ghost, phi_at(P, kg) - phi_at(P, kz));
  }
  const long long n = G.npad;
  W[R_RHO * n + i] = q.rho;
  W[R_R * n + i] = q.r;
  W[R_UX * n + i] = q.u[0];
  W[R_UY * n + i] = (DIM == 3) ? q.u[1] : 0.0;
  W[R_UZ * n + i] = q.u[DIM - 1];
  W[R_P * n + i] = q.p;
  W[R_C * n + i] = q.c;
  W[R_RC * n + i] = q.rc;
  W[R_T * n + i] = q.T;
  W[R_IC * n + i] = q.ic;
  W[R_IRC * n + i] = q.irc;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    double x = 0.0;
    if (ghost < 0 && v < NV) x = b[v];
    W[(R_CONS + v) * n + i] = x;
  }
}


// Acoustic face (a, l | l + e_a) from the stored primitives of its two cells
// (lz: vertical padded index of l).
template <int DIM, bool LM>
__device__ __forceinline__ void ref_face_at(const Params& P, const RefGrid& G, const double* __restrict__ W,
                                            long long l, int lz, int a, double& us, double& pi, double& Pf,
                                            double& S) {
  const long long n = G.npad;
  const long long r = l + astride(G, a);
  const int k = (a == 2) ? DIM - 1 : a;  // normal velocity component
  const int uf = ufield(DIM, k);
  S = 0.0;
  if (a == 2) {
    const bool wall = ref_wall(P, a, lz);
    Prim<DIM> L, R;
    L.rho = W[R_RHO * n + l]; L.rc = W[R_RC * n + l]; L.irc = W[R_IRC * n + l]; L.ic = W[R_IC * n + l];
    L.p = W[R_P * n + l]; L.u[DIM - 1] = W[uf * n + l];
    R.rho = W[R_RHO * n + r]; R.rc = W[R_RC * n + r]; R.irc = W[R_IRC * n + r]; R.ic = W[R_IC * n + r];
    R.p = W[R_P * n + r]; R.u[DIM - 1] = W[uf * n + r];
    face_vert<LM, DIM>(P, L, R, phi_at(P, lz + 1 - 2) - phi_at(P, lz - 2), wall, us, pi, Pf, S);
  } else {
    face_lat<LM>(P, W[R_RC * n + l], W[R_IRC * n + l], W[R_IC * n + l], W[R_P * n + l], W[uf * n + l],
                 W[R_RC * n + r], W[R_IRC * n + r], W[R_IC * n + r], W[R_P * n + r], W[uf * n + r], us, pi, Pf);
  }
}

// Padded cell i: its acoustic +faces for every active axis (stored), then,
// in the cell range [1, P - 1) of every active axis, its acoustic cell
// values L, S-bar and b~ (acoustic step, Sec. 2.1.2), with the -faces
// formed again from the stored primitives instead of read back (one pass
// instead of a face pass and a cell pass).
template <int DIM, bool LM>
__global__ void k_ref_face_cell(Params P, RefGrid G, const double* __restrict__ d_dt, double* __restrict__ W) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.npad) return;
  constexpr int NV = DIM + 2;
  int qx, qy, qz;
  decode(G, i, qx, qy, qz);
  const long long n = G.npad;
  // active axes in order: x, (y), z
  const int axes[3] = {0, DIM == 3 ? 1 : 2, 2};
  // All faces are formed before anything is stored, so the primitive loads
  // they share (this cell's) are not repeated behind the stores.
  double pus[3], ppi[3], pP[3], pS[3];  // own +faces
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    const int a = axes[t];
    const int qa = a == 0 ? qx : (a == 1 ? qy : qz);
    const int Pa = a == 0 ? G.Px : (a == 1 ? G.Py : G.Pz);
    pus[t] = ppi[t] = pP[t] = pS[t] = 0.0;
    if (qa + 1 < Pa) ref_face_at<DIM, LM>(P, G, W, i, qz, a, pus[t], ppi[t], pP[t], pS[t]);
  }
  const bool cell = qx >= 1 && qx < G.Px - 1 && qz >= 1 && qz < G.Pz - 1 && (DIM == 2 || (qy >= 1 && qy < G.Py - 1));
  double mus[3], mpi[3], mP[3], mS[3];  // -faces (a, i - e_a | i)
  double rho = 0.0, mom[3] = {0.0, 0.0, 0.0}, E0 = 0.0;
  if (cell) {
#pragma unroll
    for (int t = 0; t < DIM; ++t) {
      const int a = axes[t];
      ref_face_at<DIM, LM>(P, G, W, i - astride(G, a), qz - (a == 2), a, mus[t], mpi[t], mP[t], mS[t]);
    }
    rho = W[R_CONS * n + i];
    for (int k = 0; k < DIM; ++k) mom[k] = W[(R_CONS + 1 + k) * n + i];
    E0 = W[(R_CONS + NV - 1) * n + i];
  }
#pragma unroll
  for (int t = 0; t < DIM; ++t) {
    const int a = axes[t];
    const int qa = a == 0 ? qx : (a == 1 ? qy : qz);
    const int Pa = a == 0 ? G.Px : (a == 1 ? G.Py : G.Pz);
    if (qa + 1 >= Pa) continue;
    const int f = R_FACE + 4 * a;
    W[(f + 0) * n + i] = pus[t];
    W[(f + 1) * n + i] = ppi[t];
    W[(f + 2) * n + i] = pP[t];
    W[(f + 3) * n + i] = pS[t];
  }
  if (!cell) return;
  const double dt = *d_dt;
  const double lam[3] = {dt / P.dx[0], DIM == 3 ? dt / P.dx[1] : 0.0, dt / P.dx[2]};
  constexpr int TZ = DIM - 1;  // slot of the vertical axis
  double Lc = 1.0;
  for (int t = 0; t < DIM; ++t) Lc = Lc + lam[axes[t]] * (pus[t] - mus[t]);
  const double sb = 0.5 * (pS[TZ] + mS[TZ]);
  double Am[3];
  for (int t = 0; t < DIM; ++t) {
    double dpi = ppi[t] - mpi[t];
    if (axes[t] == 2) dpi = dpi - sb;
    Am[t] = lam[axes[t]] * dpi;
  }
  double AE = 0.0;
  for (int t = 0; t < DIM; ++t) {
    const double term = lam[axes[t]] * (pP[t] - mP[t]);
    AE = (t == 0) ? term : AE + term;
  }
  double calE;
  if (P.nc) {
    // App. B: energy without the potential, acoustic source (uS)_i
    const double uS = 0.5 * (pus[TZ] * pS[TZ] + mus[TZ] * mS[TZ]);
    W[R_US * n + i] = uS;
    AE = AE - lam[2] * uS;
    calE = E0;
  } else {
    calE = E0 + rho * phi_at(P, qz - 2);
  }
  const double iL = rcp_nr(Lc);
  W[R_L * n + i] = Lc;
  W[R_SB * n + i] = sb;
  W[R_BT * n + i] = rho * iL;
  for (int k = 0; k < DIM; ++k) W[(R_BT + 1 + k) * n + i] = (mom[k] - Am[k]) * iL;
  W[(R_BT + NV - 1) * n + i] = (calE - AE) * iL;
}

template <int DIM, bool DISS>
__global__ void k_ref_flux(Params P, RefGrid G, int a, double* __restrict__ W) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= G.npad) return;
  constexpr int NV = DIM + 2;
  int qx, qy, qz;
  decode(G, i, qx, qy, qz);
  const int q[3] = {qx, qy, qz};
  const int Pd[3] = {G.Px, G.Py, G.Pz};
  // face axis a: q_a in [1, P_a - 2); other active axes interior [2, P - 2)
  for (int b = 0; b < 3; ++b) {
    if (DIM == 2 && b == 1) continue;
    if (b == a) {
      if (q[b] < 1 || q[b] >= Pd[b] - 2) return;
    } else {
      if (q[b] < 2 || q[b] >= Pd[b] - 2) return;
    }
  }
  const long long n = G.npad;
  const long long j = i + astride(G, a);
  const int f = R_FACE + 4 * a;
  const double us = W[(f + 0) * n + i];
  const double pi = W[(f + 1) * n + i];
  const bool wall = ref_wall(P, a, q[2]);
  const int dn = (a == 2) ? DIM - 1 : a;  // normal velocity component index
  double tr[NV];
  if (wall) {
    for (int v = 0; v < NV; ++v) tr[v] = 0.0;
  } else {
    const long long up = us >= 0.0 ? i : j;
    tr[0] = W[R_BT * n + up] * us;
    for (int k = 0; k < DIM; ++k) tr[1 + k] = W[(R_BT + 1 + k) * n + up] * us;
    tr[NV - 1] = (W[(R_BT + NV - 1) * n + up] + pi) * us;
  }
  double Gv[NV];
  Gv[0] = tr[0];
  for (int k = 0; k < DIM; ++k) Gv[1 + k] = (k == dn) ? tr[1 + k] + pi : tr[1 + k];
  Gv[NV - 1] = tr[NV - 1];
  if (DISS) {
    // physical axis of velocity component k
    int axk[3];
    for (int k = 0; k < DIM; ++k) axk[k] = (k == DIM - 1) ? 2 : k;
    double g[3][3];  // g[t][k]: derivative along active axis index t of u_k
    int tn = (a == 2) ? DIM - 1 : a;
    const double idn = P.idx[a];
    for (int k = 0; k < DIM; ++k) {
      const int uf = ufield(DIM, k);
      g[tn][k] = (W[uf * n + j] - W[uf * n + i]) * idn;
    }
    for (int t = 0; t < DIM; ++t) {
      if (t == tn) continue;
      const int b = axk[t];
      const long long sb_ = astride(G, b);
      const double qb = P.qidx[b];
      for (int k = 0; k < DIM; ++k) {
        const int uf = ufield(DIM, k);
        g[t][k] = ((W[uf * n + i + sb_] - W[uf * n + i - sb_]) + (W[uf * n + j + sb_] - W[uf * n + j - sb_])) * qb;
      }
    }
    double div = g[0][0];
    for (int t = 1; t < DIM; ++t) div = div + g[t][t];
    double Wk = 0.0;
    for (int k = 0; k < DIM; ++k) {
      double t = P.mu * (g[tn][k] + g[k][tn]);
      if (k == tn) t = t + P.eta * div;
      const int uf = ufield(DIM, k);
      const double ufc = 0.5 * (W[uf * n + i] + W[uf * n + j]);
      Wk = (k == 0) ? t * ufc : Wk + t * ufc;
      Gv[1 + k] = Gv[1 + k] - t;
    }
    const double Q = -(P.kappa * ((W[R_T * n + j] - W[R_T * n + i]) * idn));
    Gv[NV - 1] = (Gv[NV - 1] - Wk) + Q;
  }
  for (int v = 0; v < NV; ++v) W[(R_G + 5 * a + v) * n + i] = Gv[v];
}

template <int DIM>
__global__ void k_ref_update(Params P, RefGrid G, const double* __restrict__ d_dt, const double* __restrict__ W,
                             double* __restrict__ Uout, Control* ctl) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= P.ncell) return;
  constexpr int NV = DIM + 2;
  const int x = (int)(c % P.nx);
  const long long r = c / P.nx;
  const int y = (int)(r % P.ny);
  const int z = (int)(r / P.ny);
  const long long i = G.pad(x + 2, DIM == 3 ? y + 2 : 0, z + 2);
  const long long n = G.npad;
  const double dt = *d_dt;
  const double lam[3] = {dt / P.dx[0], DIM == 3 ? dt / P.dx[1] : 0.0, dt / P.dx[2]};
  const int axes[3] = {0, DIM == 3 ? 1 : 2, 2};
  const double phic = phi_at(P, z);
  double nb[NV];
  for (int v = 0; v < NV; ++v) {
    double s = W[(R_CONS + v) * n + i];
    if (v == NV - 1 && !P.nc) s = s + W[R_CONS * n + i] * phic;
    for (int t = 0; t < DIM; ++t) {
      const int a = axes[t];
      const long long m = i - astride(G, a);
      s = s - lam[a] * (W[(R_G + 5 * a + v) * n + i] - W[(R_G + 5 * a + v) * n + m]);
    }
    if (v == DIM) s = s + lam[2] * W[R_SB * n + i];
    if (v == NV - 1 && P.nc) s = s + lam[2] * W[R_US * n + i];
    nb[v] = s;
  }
  if (!P.nc) nb[NV - 1] = nb[NV - 1] - nb[0] * phic;
  for (int v = 0; v < NV; ++v) Uout[c + v * P.ncell] = nb[v];
  const Prim<DIM> qn = cons_to_prim<DIM>(P, nb);
  double kin = nb[1] * qn.u[0];
  for (int k = 1; k < DIM; ++k) kin = kin + nb[1 + k] * qn.u[k];
  const bool ok = (W[R_L * n + i] > 0.0) && (nb[0] > 0.0) && (qn.p > 0.0) && isfinite(nb[0]) && isfinite(qn.p) &&
                  isfinite(kin);
  if (!ok) {
    atomicOr(&ctl->fault, 1u);
    atomicMin(&ctl->fault_cell, (unsigned long long)c);
  }
}

template <int DIM>
static hipError_t ref_t(const Params& P, const double* Uin, double* Uout, void* wref, const double* d_dt,
                        Control* ctl, hipStream_t s) {
  RefGrid G = make_grid(P);
  double* W = (double*)wref;
  const int bs = 256;
  const unsigned nb = (unsigned)((G.npad + bs - 1) / bs);
  hipLaunchKernelGGL(k_ref_prim<DIM>, dim3(nb), dim3(bs), 0, s, P, G, Uin, W);
  if (P.low_mach)
    hipLaunchKernelGGL((k_ref_face_cell<DIM, true>), dim3(nb), dim3(bs), 0, s, P, G, d_dt, W);
  else
    hipLaunchKernelGGL((k_ref_face_cell<DIM, false>), dim3(nb), dim3(bs), 0, s, P, G, d_dt, W);
  const int axes[3] = {0, 1, 2};
  for (int t = 0; t < 3; ++t) {
    const int a = axes[t];
    if (DIM == 2 && a == 1) continue;
    if (P.diss)
      hipLaunchKernelGGL((k_ref_flux<DIM, true>), dim3(nb), dim3(bs), 0, s, P, G, a, W);
    else
      hipLaunchKernelGGL((k_ref_flux<DIM, false>), dim3(nb), dim3(bs), 0, s, P, G, a, W);
  }
  const unsigned nc = (unsigned)((P.ncell + bs - 1) / bs);
  hipLaunchKernelGGL(k_ref_update<DIM>, dim3(nc), dim3(bs), 0, s, P, G, d_dt, W, Uout, ctl);
  return hipGetLastError();
}

template <int DIM>
static hipError_t ref_forward_t(const Params& P, const double* Uin, void* wref, const double* d_dt, hipStream_t s) {
  RefGrid G = make_grid(P);
  double* W = (double*)wref;
  const int bs = 256;
  const unsigned nb = (unsigned)((G.npad + bs - 1) / bs);
  hipLaunchKernelGGL(k_ref_prim<DIM>, dim3(nb), dim3(bs), 0, s, P, G, Uin, W);
  if (P.low_mach)
    hipLaunchKernelGGL((k_ref_face_cell<DIM, true>), dim3(nb), dim3(bs), 0, s, P, G, d_dt, W);
  else
    hipLaunchKernelGGL((k_ref_face_cell<DIM, false>), dim3(nb), dim3(bs), 0, s, P, G, d_dt, W);
  return hipGetLastError();
}

// Fluxes and update from the faces and acoustic cell values already in wref.
template <int DIM>
static hipError_t ref_finish_t(const Params& P, void* wref, double* Uout, const double* d_dt, Control* ctl,
                               hipStream_t s) {
  RefGrid G = make_grid(P);
  double* W = (double*)wref;
  const int bs = 256;
  const unsigned nb = (unsigned)((G.npad + bs - 1) / bs);
  for (int a = 0; a < 3; ++a) {
    if (DIM == 2 && a == 1) continue;
    if (P.diss)
      hipLaunchKernelGGL((k_ref_flux<DIM, true>), dim3(nb), dim3(bs), 0, s, P, G, a, W);
    else
      hipLaunchKernelGGL((k_ref_flux<DIM, false>), dim3(nb), dim3(bs), 0, s, P, G, a, W);
  }
  const unsigned nc = (unsigned)((P.ncell + bs - 1) / bs);
  hipLaunchKernelGGL(k_ref_update<DIM>, dim3(nc), dim3(bs), 0, s, P, G, d_dt, W, Uout, ctl);
  return hipGetLastError();
}

hipError_t launch_ref_finish(const Params& P, void* wref, double* Uout, const double* d_dt, Control* ctl,
                             hipStream_t s) {
  return P.dim == 3 ? ref_finish_t<3>(P, wref, Uout, d_dt, ctl, s) : ref_finish_t<2>(P, wref, Uout, d_dt, ctl, s);
}

hipError_t launch_ref_forward(const Params& P, const double* Uin, void* wref, const double* d_dt, hipStream_t s) {
  return P.dim == 3 ? ref_forward_t<3>(P, Uin, wref, d_dt, s) : ref_forward_t<2>(P, Uin, wref, d_dt, s);
}

hipError_t launch_step_ref(const Params& P, const double* Uin, double* Uout, void* wref, const double* d_dt,
                           Control* ctl, hipStream_t s) {
  return P.dim == 3 ? ref_t<3>(P, Uin, Uout, wref, d_dt, ctl, s) : ref_t<2>(P, Uin, Uout, wref, d_dt, ctl, s);
}

}  // namespace ars
