// ars_fused.h -- the per-tile vertical march of the fused step, shared by
// the single-problem step kernel and the batched kernel.
#pragma once
#include "ars_dev.h"

#include "ars_internal.h"

namespace ars {

// Synchronisation of the march between its LDS stages.  A 3D tile shares
// LDS between all waves of the workgroup: a workgroup barrier.  In 2D every
// row segment is one wave (64 positions) whose LDS slots and neighbours
// never leave that wave, so ordering the wave's own LDS accesses is enough:
// a wave-scope fence around a wave barrier (no inter-wave wait; the waves
// of a batched workgroup march independently between step barriers).
template <int DIM>
__device__ __forceinline__ void plane_sync() {
  if constexpr (DIM == 3) {
    __syncthreads();
  } else {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

template <int DIM>
struct FusedLayout;
template <>
struct FusedLayout<3> {
  static constexpr int XA = 0, NXA = 6;   // rc, 1/rc, 1/c, p, ux, uy
  static constexpr int V = 6, NVV = 4;    // ux, uy, uz, T
  static constexpr int DZ = 10, NDZ = 3;  // dz ux, dz uy, dz uz
  static constexpr int F = 13, NF = 6;    // x: us, pi, P ; y: us, pi, P
  static constexpr int B = 19, NB = 5;
  static constexpr int GX = 24, NG = 10;  // x: 5 ; y: 5
  static constexpr int TOTAL = 34;
};
template <>
struct FusedLayout<2> {
  static constexpr int XA = 0, NXA = 5;   // rc, 1/rc, 1/c, p, ux
  static constexpr int V = 5, NVV = 3;    // ux, uy, T
  static constexpr int DZ = 8, NDZ = 2;   // dy ux, dy uy
  static constexpr int F = 10, NF = 3;
  static constexpr int B = 13, NB = 4;
  static constexpr int GX = 17, NG = 4;
  static constexpr int TOTAL = 21;
};

// Vertical plane resolution: which plane to load and whether it is a wall
// ghost (0 bottom, 1 top) built from that plane.
__device__ __forceinline__ int plane_src(const Params& P, int q, int& ghost) {
  ghost = -1;
  if (q >= 0 && q < P.nz) return q;
  const int side = q < 0 ? 0 : 1;
  if (P.bcz[side] == BC_WALL) {
    ghost = side;
    return side == 0 ? 0 : P.nz - 1;
  }
  if (P.bcz[0] == BC_PERIODIC) {
    int m = q % P.nz;
    return m < 0 ? m + P.nz : m;
  }
  return side == 0 ? 0 : P.nz - 1;
}

__device__ __forceinline__ bool wall_face_below(const Params& P, int q) {
  // face between planes q and q+1
  return (q == -1 && P.bcz[0] == BC_WALL) || (q == P.nz - 1 && P.bcz[1] == BC_WALL);
}

// One workgroup marches one tile through planes [z0, z1) of the vertical
// axis: every output cell of the tile in those planes is written to Uout,
// the largest rate of the new state is folded into lmax and the smallest
// faulting cell into badcell.  Shared by the step kernel and the batched
// kernel.  (tx, ty) is the tile of this thread's row and zs a vertical
// shift of its planes: 3D tiles are TX x TY columns (tx, ty uniform over
// the workgroup, zs = 0); in 2D each of the EY rows is an independent
// segment of TX columns with its own tile and shift (plane p of the march
// is plane zs + p of the grid), so a workgroup can advance several
// segments or vertical chunks of one problem at once.
template <int DIM, bool LM, bool DISS, bool NC, int EX, int EY>
__device__ __forceinline__ void march_tile(const Params& P, const double* __restrict__ Uin,
                                           double* __restrict__ Uout, double* __restrict__ sm, const int tx,
                                           const int ty, const int zs, const int z0, const int z1,
                                           const double lamx, const double lamy, const double lamz,
                                           double& lmax, unsigned long long& badcell) {
  constexpr int NV = DIM + 2;
  constexpr int NPOS = EX * EY;
  constexpr int TX = EX - 4;
  // The stages run on all lanes (results of halo lanes are discarded, their
  // LDS slots never read by a needed position), so the code inside a stage
  // is one straight block in which the compiler interleaves independent
  // chains (the x and y faces, the cell values and the fluxes): 7 % faster
  // at 256^3 than guarding each stage per position, which splits the blocks
  // at every lane-divergent branch.  3D keeps the guards that are uniform
  // per wave for whole halo waves (the lateral-flux block, whose waves are
  // all-halo at the tile's ends: dropping that guard too measured 0.6 %
  // slower).
  constexpr bool UNI = (DIM == 2);
  static_assert(DIM == 3 || EX == 64, "a 2D row segment is exactly one wave (plane_sync relies on it)");
  constexpr int TY = (DIM == 3) ? EY - 4 : 1;
  constexpr int Z = DIM - 1;  // index of the vertical velocity component
  using Ly = FusedLayout<DIM>;
  const long long plane_stride = (long long)P.nx * P.ny;
  const long long N = P.ncell;
  const int tid = threadIdx.x;
  const int px = tid % EX;
  const int py = tid / EX;  // 3D: row of the tile; 2D: row segment

  // neighbour positions in LDS (clamped: edge positions compute values that
  // are never consumed by a needed position)
  const int pxp = px + 1 < EX ? tid + 1 : tid;
  const int pxm = px > 0 ? tid - 1 : tid;
  const int pyp = (DIM == 3 && py + 1 < EY) ? tid + EX : tid;
  const int pym = (DIM == 3 && py > 0) ? tid - EX : tid;
  const int pxpyp = (DIM == 3 && px + 1 < EX && py + 1 < EY) ? tid + EX + 1 : tid;
  const int pxpym = (DIM == 3 && px + 1 < EX && py > 0) ? tid - EX + 1 : tid;
  const int pxmyp = (DIM == 3 && px > 0 && py + 1 < EY) ? tid + EX - 1 : tid;
  // Positions that own a lateral face some output cell needs (the first
  // and the last wave of a 3D tile hold none and skip the flux stage).
  const bool inx1 = px >= 1 && px <= EX - 3;
  const bool inx2 = px >= 2 && px <= EX - 3;
  const bool iny1 = (DIM == 2) || (py >= 1 && py <= EY - 3);
  const bool iny2 = (DIM == 2) || (py >= 2 && py <= EY - 3);
  const bool needGx = inx1 && iny2;
  const bool needGy = (DIM == 3) && inx2 && iny1;

  const int x0 = tx * TX;
  const int y0 = ty * TY;
  const int gx = x0 + px - 2;
  const int gy = (DIM == 3) ? y0 + py - 2 : 0;
  const int cx = resolve_lat(gx, P.nx, P.bcx);
  const int cy = (DIM == 3) ? resolve_lat(gy, P.ny, P.bcy) : 0;
  const bool lat_out = (px >= 2 && px < EX - 2 && gx < P.nx) &&
                       (DIM == 2 || (py >= 2 && py < EY - 2 && gy < P.ny));
  const long long col = (long long)cx + (long long)P.nx * cy;

  // ---- rolling registers ---------------------------------------------------
  double Unx[NV];                 // conserved values of the next plane to use
  double U1[NV], U2[NV];          // conserved values of planes p-1, p-2
  Prim<DIM> q0, q1;               // primitives of planes p, p-1
  double u2[DIM], T2 = 0.0;       // u, T of plane p-2
  double zAus = 0, zApi = 0, zAP = 0, zAS = 0;  // z face (p-2|p-1)
  double zBus = 0, zBpi = 0, zBP = 0, zBS = 0;  // z face (p-1|p)
  double bt1[NV], bt2[NV];        // b~ of planes p-1, p-2
  double sb1 = 0.0, sb2 = 0.0;    // S-bar of planes p-1, p-2
  double uS1 = 0.0, uS2 = 0.0;    // (uS)_i of planes p-1, p-2 (non-conservative energy)
  double GzLo[NV];                // z-face flux (p-3|p-2)
  double Fo1[3 * (DIM - 1)];      // own lateral acoustic faces of plane p-1
  double dX2[4];                  // tangential differences at plane p-2
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    U1[v] = U2[v] = bt1[v] = bt2[v] = GzLo[v] = 0.0;
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) u2[k] = 0.0;
#pragma unroll
  for (int i = 0; i < 3 * (DIM - 1); ++i) Fo1[i] = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) dX2[i] = 0.0;
  q1 = Prim<DIM>{};

  int ghost_nx;
  {
    const int src = plane_src(P, zs + z0 - 2, ghost_nx);
    const double* base = Uin + col + plane_stride * src;
#pragma unroll
    for (int v = 0; v < NV; ++v) Unx[v] = base[v * N];
  }

  // One plane of the march.  In 3D the loop below takes two planes per trip
  // so that the rotation of the vertical window between them is a renaming
  // of registers, not a copy (the loop holds barriers, which the compiler's
  // own unrolling does not take; measured 1 % faster in 3D, 1 % slower for
  // the 2D row segments, which keep one plane per trip); z0 and z1 are
  // uniform over the workgroup, so every wave takes the same trips.
  auto plane = [&](const int p) __attribute__((always_inline)) {
    // ================= step 1: primitives of plane p ========================
    double Uc[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Uc[v] = Unx[v];
    const int ghost = ghost_nx;
    if (p + 1 <= z1 + 1) {  // prefetch plane p+1
      const int src = plane_src(P, zs + p + 1, ghost_nx);
      const double* base = Uin + col + plane_stride * src;
#pragma unroll
      for (int v = 0; v < NV; ++v) Unx[v] = base[v * N];
    }
    q0 = cons_to_prim<DIM>(P, Uc);
    if (ghost >= 0) {
      const int kg = ghost == 0 ? -1 : P.nz;
      const int ki = ghost == 0 ? 0 : P.nz - 1;
      q0 = wall_ghost<DIM>(P, q0, ghost, phi_at(P, kg) - phi_at(P, ki));
    }
    const double phip = phi_at(P, zs + p);
    const double phi1 = phi_at(P, zs + p - 1);
    const double phi2 = phi_at(P, zs + p - 2);
    // z face (p-1 | p)
    if (p >= z0 - 1) {
      face_vert<LM, DIM>(P, q1, q0, phip - phi1, wall_face_below(P, zs + p - 1), zBus, zBpi, zBP, zBS);
    }
    // LDS: acoustic fields of plane p; viscous fields of plane p-1
    sm[(Ly::XA + 0) * NPOS + tid] = q0.rc;
    sm[(Ly::XA + 1) * NPOS + tid] = q0.irc;
    sm[(Ly::XA + 2) * NPOS + tid] = q0.ic;
    sm[(Ly::XA + 3) * NPOS + tid] = q0.p;
    sm[(Ly::XA + 4) * NPOS + tid] = q0.u[0];
    if (DIM == 3) sm[(Ly::XA + 5) * NPOS + tid] = q0.u[1];
    if (DISS) {
#pragma unroll
      for (int k = 0; k < DIM; ++k) sm[(Ly::V + k) * NPOS + tid] = q1.u[k];
      sm[(Ly::V + DIM) * NPOS + tid] = q1.T;
#pragma unroll
      for (int k = 0; k < DIM; ++k) sm[(Ly::DZ + k) * NPOS + tid] = q0.u[k] - u2[k];
    }
    // Step 2a needs only the -x/-y faces of plane p-1 (published before the
    // previous barrier) and this column's z faces, so it runs before bar 1,
    // and F of plane p is published after bar 1, when every reader of F of
    // plane p-1 has passed it: two barriers per plane.  (With the stages on
    // every lane this is 1 % faster in 3D than running step 2a after bar 1
    // and publishing F behind a third barrier, which was the faster order
    // while 3D guarded its stages per position.)

    // ================= step 2a: acoustic cell values of plane p-1 ===========
    const bool doL = (p - 1 >= z0 - 1) && (p - 1 <= z1);
    if (doL) {
      double Lc = 1.0;
      // x faces: +x own (registers), -x from the left neighbour
      const double usxm = sm[(Ly::F + 0) * NPOS + pxm];
      const double pixm = sm[(Ly::F + 1) * NPOS + pxm];
      const double Pxm = sm[(Ly::F + 2) * NPOS + pxm];
      Lc = Lc + lamx * (Fo1[0] - usxm);
      double Amx = lamx * (Fo1[1] - pixm);
      double AE = lamx * (Fo1[2] - Pxm);
      double Amy = 0.0;
      if (DIM == 3) {
        const double usym = sm[(Ly::F + 3) * NPOS + pym];
        const double piym = sm[(Ly::F + 4) * NPOS + pym];
        const double Pym = sm[(Ly::F + 5) * NPOS + pym];
        Lc = Lc + lamy * (Fo1[3] - usym);
        Amy = lamy * (Fo1[4] - piym);
        AE = AE + lamy * (Fo1[5] - Pym);
      }
      Lc = Lc + lamz * (zBus - zAus);
      const double sb = 0.5 * (zBS + zAS);
      double dpz = zBpi - zApi;
      dpz = dpz - sb;
      const double Amz = lamz * dpz;
      AE = AE + lamz * (zBP - zAP);
      double calE;
      if (NC) {
        // App. B: the energy excludes the potential and its acoustic update
        // carries the source (uS)_i of the two vertical faces
        const double uS = 0.5 * (zBus * zBS + zAus * zAS);
        uS1 = uS;
        AE = AE - lamz * uS;
        calE = U1[NV - 1];
      } else {
        calE = U1[NV - 1] + U1[0] * phi1;
      }
      const double iL = rcp_nr(Lc);
      bt1[0] = U1[0] * iL;
      bt1[1] = (U1[1] - Amx) * iL;
      if (DIM == 3) {
        bt1[2] = (U1[2] - Amy) * iL;
        bt1[3] = (U1[3] - Amz) * iL;
      } else {
        bt1[2] = (U1[2] - Amz) * iL;
      }
      bt1[NV - 1] = (calE - AE) * iL;
      sb1 = sb;
#pragma unroll
      for (int v = 0; v < NV; ++v) sm[(Ly::B + v) * NPOS + tid] = bt1[v];
      if (lat_out && p - 1 >= z0 && p - 1 < z1 && !(Lc > 0.0)) {
        const unsigned long long cell = (unsigned long long)(col + plane_stride * (zs + p - 1));
        badcell = min(badcell, cell);
      }
    }
    plane_sync<DIM>();  // ------------------------------------------------ bar 1

    // ================= step 2b: own lateral acoustic faces of plane p =======
    double Fn[3 * (DIM - 1)];
    const bool doA = (p >= z0 - 1) && (p <= z1);
    if (doA) {
      face_lat<LM>(P, q0.rc, q0.irc, q0.ic, q0.p, q0.u[0], sm[(Ly::XA + 0) * NPOS + pxp],
                   sm[(Ly::XA + 1) * NPOS + pxp], sm[(Ly::XA + 2) * NPOS + pxp], sm[(Ly::XA + 3) * NPOS + pxp],
                   sm[(Ly::XA + 4) * NPOS + pxp], Fn[0], Fn[1], Fn[2]);
      if (DIM == 3)
        face_lat<LM>(P, q0.rc, q0.irc, q0.ic, q0.p, q0.u[1], sm[(Ly::XA + 0) * NPOS + pyp],
                     sm[(Ly::XA + 1) * NPOS + pyp], sm[(Ly::XA + 2) * NPOS + pyp], sm[(Ly::XA + 3) * NPOS + pyp],
                     sm[(Ly::XA + 5) * NPOS + pyp], Fn[3], Fn[4], Fn[5]);
    } else {
#pragma unroll
      for (int i = 0; i < 3 * (DIM - 1); ++i) Fn[i] = 0.0;
    }

    // ================= step 3 ==============================================
#pragma unroll
    for (int i = 0; i < 3 * (DIM - 1); ++i) sm[(Ly::F + i) * NPOS + tid] = Fn[i];

    // tangential differences of plane p-1 (for vertical viscous faces)
    double dX1[4] = {0.0, 0.0, 0.0, 0.0};
    if (DISS) {
      // 3D: dx ux, dx uz, dy uy, dy uz ; 2D: dx ux, dx uy
      dX1[0] = sm[(Ly::V + 0) * NPOS + pxp] - sm[(Ly::V + 0) * NPOS + pxm];
      dX1[1] = sm[(Ly::V + Z) * NPOS + pxp] - sm[(Ly::V + Z) * NPOS + pxm];
      if (DIM == 3) {
        dX1[2] = sm[(Ly::V + 1) * NPOS + pyp] - sm[(Ly::V + 1) * NPOS + pym];
        dX1[3] = sm[(Ly::V + 2) * NPOS + pyp] - sm[(Ly::V + 2) * NPOS + pym];
      }
    }

    // lateral total fluxes of plane p-1 (own +x / +y faces)
    // lateral fluxes are published only where computed; every reader of a
    // GX slot (an output cell or its -x/-y neighbour) has it computed
    double GXn[NV], GYn[NV];
    const bool doG = (p - 1 >= z0) && (p - 1 < z1);
    if (doG && (UNI || needGx || needGy)) {
#pragma unroll
      for (int dir = 0; dir < DIM - 1; ++dir) {
        const int nb = dir == 0 ? pxp : pyp;
        const double us = Fo1[3 * dir + 0];
        const double pi = Fo1[3 * dir + 1];
        double G[NV];
        const bool upL = us >= 0.0;
        double bu[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          // load the neighbour's value unconditionally and select: keeps the
          // upwind choice a v_cndmask instead of a divergent branch per field
          const double bn = sm[(Ly::B + v) * NPOS + nb];
          bu[v] = upL ? bt1[v] : bn;
        }
        G[0] = bu[0] * us;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          const double tr = bu[1 + k] * us;
          G[1 + k] = (k == dir) ? tr + pi : tr;
        }
        G[NV - 1] = (bu[NV - 1] + pi) * us;
        if (DISS) {
          // gradient rows at the face: g[a][k] = d u_k / d x_a
          double uR[DIM], TR;
#pragma unroll
          for (int k = 0; k < DIM; ++k) uR[k] = sm[(Ly::V + k) * NPOS + nb];
          TR = sm[(Ly::V + DIM) * NPOS + nb];
          double g[3][3];
          const double idn = P.idx[dir];
#pragma unroll
          for (int k = 0; k < DIM; ++k) g[dir][k] = (uR[k] - q1.u[k]) * idn;
          if (DIM == 3) {
            // the other lateral axis
            const int a = 1 - dir;
            const int pa_p = a == 1 ? pyp : pxp;
            const int pa_m = a == 1 ? pym : pxm;
            const int nb_p = a == 1 ? (dir == 0 ? pxpyp : pyp) : (dir == 1 ? pxpyp : pxp);
            const int nb_m = a == 1 ? (dir == 0 ? pxpym : pym) : (dir == 1 ? pxmyp : pxm);
            // needed: g[a][dir] and g[a][a]
            const double qa = P.qidx[a];
            g[a][dir] = ((sm[(Ly::V + dir) * NPOS + pa_p] - sm[(Ly::V + dir) * NPOS + pa_m]) +
                         (sm[(Ly::V + dir) * NPOS + nb_p] - sm[(Ly::V + dir) * NPOS + nb_m])) * qa;
            g[a][a] = ((sm[(Ly::V + a) * NPOS + pa_p] - sm[(Ly::V + a) * NPOS + pa_m]) +
                       (sm[(Ly::V + a) * NPOS + nb_p] - sm[(Ly::V + a) * NPOS + nb_m])) * qa;
          }
          // vertical tangential: needed g[Z][dir] and g[Z][Z]
          {
            const double qz = P.qidx[2];
            const double dzs_dir = q0.u[dir] - u2[dir];
            const double dzs_z = q0.u[Z] - u2[Z];
            g[Z][dir] = (dzs_dir + sm[(Ly::DZ + dir) * NPOS + nb]) * qz;
            g[Z][Z] = (dzs_z + sm[(Ly::DZ + Z) * NPOS + nb]) * qz;
          }
          double div = g[0][0];
          if (DIM == 3) div = div + g[1][1];
          div = div + g[Z][Z];
          double W = 0.0;
#pragma unroll
          for (int k = 0; k < DIM; ++k) {
            double t = P.mu * (g[dir][k] + g[k][dir]);
            if (k == dir) t = t + P.eta * div;
            const double uf = 0.5 * (q1.u[k] + uR[k]);
            W = (k == 0) ? t * uf : W + t * uf;
            G[1 + k] = G[1 + k] - t;
          }
          const double Q = -(P.kappa * ((TR - q1.T) * idn));
          G[NV - 1] = (G[NV - 1] - W) + Q;
        }
        if (dir == 0) {
#pragma unroll
          for (int v = 0; v < NV; ++v) GXn[v] = G[v];
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) GYn[v] = G[v];
        }
      }
    }

    // vertical total flux at (p-2 | p-1)
    double Gz[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Gz[v] = 0.0;
    const bool doGz = (p - 1 >= z0) && (p - 1 <= z1);
    if (doGz) {
      const bool wall = wall_face_below(P, zs + p - 2);
      double tr[NV];
      if (wall) {
#pragma unroll
        for (int v = 0; v < NV; ++v) tr[v] = 0.0;
      } else {
        const bool upL = zAus >= 0.0;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double b = upL ? bt2[v] : bt1[v];
          tr[v] = (v == NV - 1) ? (b + zApi) * zAus : b * zAus;
        }
      }
      Gz[0] = tr[0];
#pragma unroll
      for (int k = 0; k < DIM; ++k) Gz[1 + k] = (k == Z) ? tr[1 + k] + zApi : tr[1 + k];
      Gz[NV - 1] = tr[NV - 1];
      if (DISS) {
        double g[3][3];
        const double idn = P.idx[2];
#pragma unroll
        for (int k = 0; k < DIM; ++k) g[Z][k] = (q1.u[k] - u2[k]) * idn;
        // lateral tangential rows: g[0][Z], g[0][0] (and g[1][Z], g[1][1])
        g[0][0] = (dX2[0] + dX1[0]) * P.qidx[0];
        g[0][Z] = (dX2[1] + dX1[1]) * P.qidx[0];
        if (DIM == 3) {
          g[1][1] = (dX2[2] + dX1[2]) * P.qidx[1];
          g[1][Z] = (dX2[3] + dX1[3]) * P.qidx[1];
        }
        double div = g[0][0];
        if (DIM == 3) div = div + g[1][1];
        div = div + g[Z][Z];
        double W = 0.0;
#pragma unroll
        for (int k = 0; k < DIM; ++k) {
          double t = P.mu * (g[Z][k] + g[k][Z]);
          if (k == Z) t = t + P.eta * div;
          const double uf = 0.5 * (u2[k] + q1.u[k]);
          W = (k == 0) ? t * uf : W + t * uf;
          Gz[1 + k] = Gz[1 + k] - t;
        }
        const double Q = -(P.kappa * ((q1.T - T2) * idn));
        Gz[NV - 1] = (Gz[NV - 1] - W) + Q;
      }
    }

    // ================= update of plane p-2 ==================================
    const int o = p - 2;
    if (o >= z0 && o < z1 && lat_out) {
      double nb[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const double gxo = sm[(Ly::GX + v) * NPOS + tid];
        const double gxm = sm[(Ly::GX + v) * NPOS + pxm];
        double s = (v == NV - 1) ? (NC ? U2[NV - 1] : U2[NV - 1] + U2[0] * phi2) : U2[v];
        s = s - lamx * (gxo - gxm);
        if (DIM == 3) {
          const double gyo = sm[(Ly::GX + NV + v) * NPOS + tid];
          const double gym = sm[(Ly::GX + NV + v) * NPOS + pym];
          s = s - lamy * (gyo - gym);
        }
        s = s - lamz * (Gz[v] - GzLo[v]);
        if (v == 1 + Z) s = s + lamz * sb2;
        if (NC && v == NV - 1) s = s + lamz * uS2;
        nb[v] = s;
      }
      if (!NC) nb[NV - 1] = nb[NV - 1] - nb[0] * phi2;  // relaxation step: E = calE - rho Phi
      const long long cell = col + plane_stride * (zs + o);
#pragma unroll
      for (int v = 0; v < NV; ++v) Uout[cell + v * N] = nb[v];
      // epilogue: rate of the new state and validity
      const Prim<DIM> qn = cons_to_prim<DIM>(P, nb);
      double kin = nb[1] * qn.u[0];
#pragma unroll
      for (int k = 1; k < DIM; ++k) kin = kin + nb[1 + k] * qn.u[k];
      const double l = cell_rate<DIM>(P, qn);
      lmax = l > lmax ? l : lmax;
      const bool ok = (nb[0] > 0.0) && (qn.p > 0.0) && isfinite(nb[0]) && isfinite(qn.p) && isfinite(kin);
      if (!ok) badcell = min(badcell, (unsigned long long)cell);
    }
    plane_sync<DIM>();  // -------------------------------------------- bar 2

    // ================= step 4: publish lateral fluxes of plane p-1 ==========
    if (doG && (UNI || needGx)) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sm[(Ly::GX + v) * NPOS + tid] = GXn[v];
    }
    if (DIM == 3 && doG && (UNI || needGy)) {
#pragma unroll
      for (int v = 0; v < NV; ++v) sm[(Ly::GX + NV + v) * NPOS + tid] = GYn[v];
    }
    // rotate the vertical window
#pragma unroll
    for (int k = 0; k < DIM; ++k) u2[k] = q1.u[k];
    T2 = q1.T;
    q1 = q0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      U2[v] = U1[v];
      U1[v] = Uc[v];
      bt2[v] = bt1[v];
      GzLo[v] = Gz[v];
    }
    zAus = zBus; zApi = zBpi; zAP = zBP; zAS = zBS;
    sb2 = sb1;
    uS2 = uS1;
#pragma unroll
    for (int i = 0; i < 3 * (DIM - 1); ++i) Fo1[i] = Fn[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) dX2[i] = dX1[i];
  };
  int p = z0 - 2;
  if constexpr (DIM == 3) {
    for (; p + 1 <= z1 + 1; p += 2) {
      plane(p);
      plane(p + 1);
    }
    if (p <= z1 + 1) plane(p);
  } else {
    for (; p <= z1 + 1; ++p) plane(p);
  }

}

}  // namespace ars
