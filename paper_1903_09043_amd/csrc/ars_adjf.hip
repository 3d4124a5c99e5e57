// ars_adjf.hip -- fused reverse (adjoint) of one explicit step at a frozen
// time step, for 3D problems with periodic lateral sides and walls (or, with
// g = 0, periodic ends) along the vertical axis:
//   lam^n = (dU^{n+1}/dU^n)^T lam^{n+1},  <lam^{n+1}, dU^{n+1}/d(mu, kappa)>.
//
// Three tile marches along the vertical axis replace the phase kernels of
// ars_adjoint.hip (which stay as the reference path and serve every other
// configuration):
//
//  A  (halo 2) recomputes the acoustic part of the step of eq.
//     all_regime_scheme plane by plane exactly as the fused step does
//     (primitives, acoustic faces, acoustic cell values b~ = (b - A)/L),
//     forms the flux adjoints Gb = lam_a (nbar(R) - nbar(L)) from
//     lam^{n+1}, reverses the transport fluxes (u*, Pi* adjoints of every
//     face, b~ adjoint of every cell) and the acoustic cell values (adjoints
//     of L, A, S-bar and the direct conserved-value term).  It writes per
//     cell the adjoints of (L, A_m, A_E, S-bar) and the (u*, Pi*) adjoints
//     of its +x, +y, +z faces (12 fields), and lam^n = lam^{n+1} + the
//     direct term.
//  V  (halo 2) reverses the viscous and heat fluxes of Sec. 2.2: every face
//     publishes through LDS what it owes the cells of its stencil, every
//     cell collects in a fixed order; the velocity and temperature adjoints
//     of each cell (with those of its wall ghosts, through the ghost map)
//     are written as 5 more fields, and the mu/kappa derivatives are summed
//     per workgroup.
//  B  (halo 1) reverses the acoustic face solver (Sec. 2.1.2 with eq.
//     low_mach_correction and the gravity source of eq. well_balanced_formula)
//     of every face from those 12 fields and the recomputed primitives,
//     gathers the primitive adjoints of each cell (and of its wall ghosts),
//     adds the viscous ones of V, takes the sum through the primitive map
//     and adds it to lam^n.  Every plane's inputs are loaded one plane
//     ahead.
//
// Periodic lateral sides make every position of a tile a distinct cell of
// the grid (at least 5 cells per lateral axis), so every face is one
// physical face whose adjoint carries lam^{n+1} of both of its cells and no
// image has to be folded back.  Faces and cells are each reversed by one
// owner in a fixed order, and the mu/kappa partial sums go through one slot
// per workgroup: the result is deterministic.  Non-smooth operations take
// the branch of the forward step (max/min: first argument on ties; |x|: sign
// of x >= 0; upwind: u* >= 0 takes the left cell), as everywhere else.
#include <algorithm>

#include "ars_fused.h"

namespace ars {

// Workspace fields (each ncell doubles, interior layout).
enum {
  AF_CB = 0,   // adjoints of L, A_mx, A_my, A_mz, A_E, S-bar of the cell
  AF_FB = 6,   // (u*, Pi*) adjoints of the cell's +x, +y, +z faces from the flux reverse
  AF_PV = 12,  // (rho, u0, u1, u2, T) adjoints from the viscous and heat fluxes
  AF_NF = 17
};

// Tiles (positions = outputs + halo): A and V have a 2-cell halo, B a
// 1-cell halo.
constexpr int AF_AX = 36, AF_AY = 14;
constexpr int AF_VX = 36, AF_VY = 14;
constexpr int AF_BX = 32, AF_BY = 16;

bool adjf_supported(const Params& P) {
  if (P.dim != 3 || P.nc) return false;
  if (P.bcx[0] != BC_PERIODIC || P.bcy[0] != BC_PERIODIC) return false;
  if (P.nx < 5 || P.ny < 5) return false;
  const bool walls = P.bcz[0] == BC_WALL && P.bcz[1] == BC_WALL;
  const bool per = P.bcz[0] == BC_PERIODIC && P.g == 0.0 && P.nz >= 5;
  return walls || per;
}

static long long adjf_tiles(const Params& P, int EX, int EY, int halo) {
  const int TX = EX - 2 * halo, TY = EY - 2 * halo;
  return (long long)((P.nx + TX - 1) / TX) * ((P.ny + TY - 1) / TY);
}

static int adjf_num_cu() {
  static int ncu = 0;
  if (ncu == 0) {
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || n < 1)
      n = 256;
    ncu = n;
  }
  return ncu;
}

// Workgroups of a march: `per_cu` per compute unit (at most 1024 in all, so
// that the mu/kappa partials of V fit their slots), never more than
// (tile, plane) pairs / 8.
static int adjf_groups(const Params& P, int EX, int EY, int halo, int per_cu) {
  const long long pairs = adjf_tiles(P, EX, EY, halo) * P.nz;
  long long g = std::min(per_cu * adjf_num_cu(), 1024);
  g = std::min(g, std::max(1ll, pairs / 8));
  return (int)g;
}

// Share of workgroup b: workgroups are dealt to the 8 XCDs in turn, so the
// shares of one XCD are made consecutive (neighbours in space, whose halo
// re-reads then hit that XCD's L2).
__device__ __forceinline__ int xcd_share(int b, int G) { return (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b; }

size_t adjf_workspace_bytes(const Params& P) {
  return (size_t)AF_NF * (size_t)P.ncell * sizeof(double) + 2 * 1024 * sizeof(double);
}

// ------------------------------------------------------------------------
// Reverse building blocks
// ------------------------------------------------------------------------

// Reverse of cons_to_prim at one cell: pb = adjoints of (rho, u0, u1, u2, p,
// rho c, 1/(rho c), 1/c, T), q the forward primitives, m the momenta.
__device__ __forceinline__ void prim_adj(const Params& P, const Prim<3>& q, const double* m, const double* pb,
                                         double* Ub) {
  double rho_b = pb[0];
  double p_b = pb[4];
  const double rc_b = pb[5], irc_b = pb[6], ic_b = pb[7], T_b = pb[8];
  // irc = r ic, rc = rho c, ic = 1/c
  double rb = irc_b * q.ic;
  const double icb = ic_b + irc_b * q.r;
  double cb = -icb * q.ic * q.ic;
  rho_b += rc_b * q.c;
  cb += rc_b * q.rho;
  // T = p r
  p_b += T_b * q.r;
  rb += T_b * q.p;
  // c = sqrt(gamma p r): dc/dX = 1/(2c) = ic/2
  const double Xb = (cb * 0.5) * q.ic;
  p_b += Xb * P.gamma * q.r;
  rb += Xb * P.gamma * q.p;
  // p = (gamma - 1)(E - kin), kin = sum m_k u_k / 2, u_k = m_k r
  const double Eb = P.gm1 * p_b;
  const double kinb = -P.gm1 * p_b;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double mb = 0.5 * kinb * q.u[k];
    const double ubt = pb[1 + k] + 0.5 * kinb * m[k];
    mb += ubt * q.r;
    rb += ubt * m[k];
    Ub[1 + k] = mb;
  }
  rho_b += -rb * q.r * q.r;
  Ub[0] = rho_b;
  Ub[4] = Eb;
}

// Reverse of wall_ghost: gb = adjoints of the ghost's primitives (layout of
// prim_adj), added to the adjoints of the interior cell's (rho, u, T) in ib.
__device__ __forceinline__ void ghost_adj(const Params& P, int side, double delta, const Prim<3>& in,
                                          const Prim<3>& g, const double* gb, double* ib) {
  const double hd = 0.5 * delta;
  const double den = g.T + hd;
  double rb = gb[6] * g.ic;
  const double icb = gb[7] + gb[6] * g.r;
  double cb = -icb * g.ic * g.ic;
  double rhob = gb[0] + gb[5] * g.c;
  cb += gb[5] * g.rho;
  const double Xb = (cb * 0.5) * g.ic;
  double pb = gb[4] + Xb * P.gamma * g.r;
  rb += Xb * P.gamma * g.p;
  rhob += -rb * g.r * g.r;
  // p = rho Tg, T = Tg
  rhob += pb * g.T;
  double Tgb = gb[8] + pb * g.rho;
  // rho_g = rho_i (T_i - hd) / (Tg + hd)
  const double numb = rhob / den;
  Tgb += -rhob * g.rho / den;
  ib[0] += numb * (in.T - hd);
  double Tib = numb * in.rho;
  Tib += (P.thermal[side] == TH_FIXED) ? -Tgb : Tgb;
  ib[8] += Tib;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const bool flip = P.noslip ? true : (k == 2);
    ib[1 + k] += flip ? -gb[1 + k] : gb[1 + k];
  }
}

// Reverse of the viscous and heat flux of a face normal to axis dn, from
// the flux adjoint Gb: g is the forward gradient (g[a][k] = d u_k / d x_a;
// the entries the flux uses), uL/uR, TL/TR the cell values.  Returns the
// adjoints of uL, uR, TL, TR, of the gradient entries (gb) and mu/kappa.
__device__ __forceinline__ void visc_adj(const Params& P, int dn, double idn, const double (&g)[3][3],
                                         const double* uL, const double* uR, double TL, double TR, const double* Gb,
                                         double* uLb, double* uRb, double& TLb, double& TRb, double (&gb)[3][3],
                                         double& mub, double& kappab) {
  double div = g[0][0];
  div = div + g[1][1];
  div = div + g[2][2];
  double tau[3], uf[3], taub[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double t = P.mu * (g[dn][k] + g[k][dn]);
    if (k == dn) t = t + P.eta * div;
    tau[k] = t;
    uf[k] = 0.5 * (uL[k] + uR[k]);
    taub[k] = -Gb[1 + k];
  }
  // G_E = (G_E - W) + Q, W = sum tau_k uf_k, Q = -(kappa (TR - TL) idn)
  const double Wb = -Gb[4];
  const double Qb = Gb[4];
  const double x = (TR - TL) * idn;
  kappab = -x * Qb;
  const double dTb = (-P.kappa * Qb) * idn;
  TRb = dTb;
  TLb = -dTb;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    taub[k] += Wb * uf[k];
    const double ufb = Wb * tau[k];
    uLb[k] = 0.5 * ufb;
    uRb[k] = 0.5 * ufb;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 3; ++k) gb[a][k] = 0.0;
  mub = 0.0;
  double etab = 0.0, divb = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    mub += (g[dn][k] + g[k][dn]) * taub[k];
    const double s = P.mu * taub[k];
    gb[dn][k] += s;
    gb[k][dn] += s;
    if (k == dn) {
      etab += div * taub[k];
      divb += P.eta * taub[k];
    }
  }
  mub += etab * (-2.0 / 3.0);  // Stokes: eta = -2 mu / 3
#pragma unroll
  for (int t = 0; t < 3; ++t) gb[t][t] += divb;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    uRb[k] += gb[dn][k] * idn;
    uLb[k] -= gb[dn][k] * idn;
  }
}

// Reverse of the acoustic face solver (face_lat / face_vert) from the
// adjoints of u*, Pi*, P = Pi* u* and S: bl / br = adjoints of (rho, u_n, p,
// rho c, 1/(rho c), 1/c) of the left / right cell.
template <bool LM>
__device__ __forceinline__ void face_adj(const Params& P, bool vert, bool wall, double dphi, double us, double pi,
                                         double S, double uL, double pL, double rcL, double ircL, double icL,
                                         double uR, double pR, double rcR, double ircR, double icR, double usb,
                                         double pib, double Pb, double Sb, double* bl, double* br) {
  const double aa = P.K * dmax2(rcL, rcR);
  double theta = 1.0, ma = 0.0, cmin = 0.0;
  if (LM) {
    cmin = dmin2(icL, icR);
    ma = fabs(us) * cmin;
    theta = dmin2(ma, 1.0);
  }
  const double h = (0.5 * aa) * theta;
  const double du = uR - uL;
  double uLb = 0, uRb = 0, pLb = 0, pRb = 0, rcLb = 0, rcRb = 0, iLb = 0, iRb = 0, cLb = 0, cRb = 0;
  // P = Pi* u*
  pib += Pb * us;
  usb += Pb * pi;
  // Pi* = (pL + pR)/2 - h (uR - uL), h = (a/2) theta
  pLb += 0.5 * pib;
  pRb += 0.5 * pib;
  const double hb = -pib * du;
  const double dub = -pib * h;
  uRb += dub;
  uLb -= dub;
  const double ab = 0.5 * theta * hb;
  const double thetab = (0.5 * aa) * hb;
  if (LM && !wall) {
    const double mab = (ma <= 1.0) ? thetab : 0.0;
    const double absb = mab * cmin;
    const double cminb = mab * fabs(us);
    usb += (us >= 0.0) ? absb : -absb;
    if (icL <= icR)
      cLb += cminb;
    else
      cRb += cminb;
  }
  if (!wall) {
    // u* = (uL + uR)/2 - ((pR - pL) - S) (hK min(1/(rho c)))
    const double m = P.hK * dmin2(ircL, ircR);
    const double d1 = (pR - pL) - S;
    uLb += 0.5 * usb;
    uRb += 0.5 * usb;
    const double d1b = -usb * m;
    const double mb = -usb * d1;
    pRb += d1b;
    pLb -= d1b;
    Sb -= d1b;
    if (ircL <= ircR)
      iLb += P.hK * mb;
    else
      iRb += P.hK * mb;
  }
  double rLb = 0.0, rRb = 0.0;
  if (vert) {
    // S = -(rhoL + rhoR)/2 dphi
    const double rb = -0.5 * (Sb * dphi);
    rLb = rb;
    rRb = rb;
  }
  // a = K max(rho c)
  if (rcL >= rcR)
    rcLb += P.K * ab;
  else
    rcRb += P.K * ab;
  bl[0] = rLb; bl[1] = uLb; bl[2] = pLb; bl[3] = rcLb; bl[4] = iLb; bl[5] = cLb;
  br[0] = rRb; br[1] = uRb; br[2] = pRb; br[3] = rcRb; br[4] = iRb; br[5] = cRb;
}

__device__ __forceinline__ void nbar_of(const Params& P, int q, bool ghost, const double* lam, double* nb) {
  // adjoint of the update's pre-relaxation values nb (E' = nb_E - nb_rho Phi);
  // wall ghosts are not updated
  if (ghost) {
#pragma unroll
    for (int v = 0; v < 5; ++v) nb[v] = 0.0;
    return;
  }
  nb[0] = lam[0] - phi_at(P, q) * lam[4];
#pragma unroll
  for (int v = 1; v < 5; ++v) nb[v] = lam[v];
}

// ------------------------------------------------------------------------
// March A: acoustic and transport reverse
// ------------------------------------------------------------------------
struct AdjIOF {
  const double* U;     // U^n
  const double* lam1;  // lam^{n+1}
  double* lam0;        // lam^n (A writes the partial sum, V and B complete it)
  double* W;           // AF_NF fields
  double* partial;     // mu/kappa partials, 2 per workgroup of V
  const double* dt;
  int ntx, nty;
};

// nbar at a plane from lam^{n+1} (zero at wall ghosts, whose lam is zero)
__device__ __forceinline__ double nbar_v(const Params& P, int v, double phi, const double* l) {
  return v == 0 ? l[0] - phi * l[4] : l[v];
}

// LDS fields of march A (x NPOS doubles)
enum {
  LA_XA = 0,   // rc, 1/rc, 1/c, p, ux, uy of plane p
  LA_F = 6,    // own +x / +y faces of plane p: us, pi (x), us, pi (y)
  LA_B = 10,   // b~ of plane p-1
  LA_NB = 15,  // nbar of plane p-1, two slots (plane parity)
  LA_TOTAL = 25
};

template <bool LM, int EX, int EY>
__device__ __forceinline__ void adj_march_a(const Params& P, const AdjIOF& io, double* __restrict__ sm, const int tx,
                                            const int ty, const int z0, const int z1, const double lx,
                                            const double ly, const double lz) {
  constexpr int NV = 5;
  constexpr int NPOS = EX * EY;
  constexpr int TX = EX - 4, TY = EY - 4;
  const long long PS = (long long)P.nx * P.ny;
  const long long N = P.ncell;
  const int tid = threadIdx.x;
  const int px = tid % EX, py = tid / EX;
  const int pxp = px + 1 < EX ? tid + 1 : tid, pxm = px > 0 ? tid - 1 : tid;
  const int pyp = py + 1 < EY ? tid + EX : tid, pym = py > 0 ? tid - EX : tid;
  const int gx = tx * TX + px - 2, gy = ty * TY + py - 2;
  const int cx = resolve_lat(gx, P.nx, P.bcx), cy = resolve_lat(gy, P.ny, P.bcy);
  const long long col = (long long)cx + (long long)P.nx * cy;
  const bool out = px >= 2 && px < EX - 2 && gx < P.nx && py >= 2 && py < EY - 2 && gy < P.ny;
  const bool needL = px >= 1 && px <= EX - 2 && py >= 1 && py <= EY - 2;

  double Unx[NV], Lnx[NV];
  double U1[NV];                   // conserved values of plane p-1
  double l1[NV], l2[NV];           // lam^{n+1} of planes p-1, p-2 (0 at wall ghosts)
  Prim<3> q1;                      // primitives of plane p-1
  double zAus = 0, zApi = 0, zAP = 0, zAS = 0;
  double bt1[NV], bt2[NV], L1 = 1.0, L2 = 1.0;
  double Fo1[6];
  double btb2[NV];                 // b~ adjoint of plane p-2 (all but its top face)
#pragma unroll
  for (int v = 0; v < NV; ++v) U1[v] = l1[v] = l2[v] = bt1[v] = bt2[v] = btb2[v] = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) Fo1[i] = 0.0;
  q1 = Prim<3>{};
  int ghost_nx;
  {
    const int src = plane_src(P, z0 - 2, ghost_nx);
    const long long b = col + PS * src;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Unx[v] = io.U[b + v * N];
      Lnx[v] = io.lam1[b + v * N];  // a valid cell in every case; zeroed at wall ghosts when used
    }
  }
  for (int p = z0 - 2; p <= z1 + 1; ++p) {
    // ======================= phase 1 =======================================
    const int ghost = ghost_nx;
    double Uc[NV], l0[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Uc[v] = Unx[v];
      l0[v] = ghost >= 0 ? 0.0 : Lnx[v];  // wall ghosts are not updated: no lam
    }
    if (p + 1 <= z1 + 1) {
      const int src = plane_src(P, p + 1, ghost_nx);
      const long long b = col + PS * src;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Unx[v] = io.U[b + v * N];
        Lnx[v] = io.lam1[b + v * N];
      }
    }
    Prim<3> q0 = cons_to_prim<3>(P, Uc);
    if (ghost >= 0) {
      const int kg = ghost == 0 ? -1 : P.nz;
      const int ki = ghost == 0 ? 0 : P.nz - 1;
      q0 = wall_ghost<3>(P, q0, ghost, phi_at(P, kg) - phi_at(P, ki));
    }
    const double phip = phi_at(P, p), phi1 = phi_at(P, p - 1), phi2 = phi_at(P, p - 2);
    double zBus = 0, zBpi = 0, zBP = 0, zBS = 0;
    if (p >= z0 - 1) face_vert<LM, 3>(P, q1, q0, phip - phi1, wall_face_below(P, p - 1), zBus, zBpi, zBP, zBS);
    sm[(LA_XA + 0) * NPOS + tid] = q0.rc;
    sm[(LA_XA + 1) * NPOS + tid] = q0.irc;
    sm[(LA_XA + 2) * NPOS + tid] = q0.ic;
    sm[(LA_XA + 3) * NPOS + tid] = q0.p;
    sm[(LA_XA + 4) * NPOS + tid] = q0.u[0];
    sm[(LA_XA + 5) * NPOS + tid] = q0.u[1];
    const int nbs = LA_NB + 5 * (p & 1);
    double nb1[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      nb1[v] = nbar_v(P, v, phi1, l1);
      sm[(nbs + v) * NPOS + tid] = nb1[v];
    }
    __syncthreads();  // ------------------------------------------- bar 1

    // ======================= phase 2 =======================================
    // acoustic cell values of plane p-1 (forward)
    const bool doL = (p - 1 >= z0 - 1) && (p - 1 <= z1);
    if (doL) {
      const double usxm = sm[(LA_F + 0) * NPOS + pxm];
      const double pixm = sm[(LA_F + 1) * NPOS + pxm];
      const double Pxm = pixm * usxm;
      const double usym = sm[(LA_F + 2) * NPOS + pym];
      const double piym = sm[(LA_F + 3) * NPOS + pym];
      const double Pym = piym * usym;
      double Lc = 1.0;
      Lc = Lc + lx * (Fo1[0] - usxm);
      const double Amx = lx * (Fo1[1] - pixm);
      double AE = lx * (Fo1[2] - Pxm);
      Lc = Lc + ly * (Fo1[3] - usym);
      const double Amy = ly * (Fo1[4] - piym);
      AE = AE + ly * (Fo1[5] - Pym);
      Lc = Lc + lz * (zBus - zAus);
      const double sb = 0.5 * (zBS + zAS);
      double dpz = zBpi - zApi;
      dpz = dpz - sb;
      const double Amz = lz * dpz;
      AE = AE + lz * (zBP - zAP);
      const double calE = U1[NV - 1] + U1[0] * phi1;
      const double iL = rcp_nr(Lc);
      bt1[0] = U1[0] * iL;
      bt1[1] = (U1[1] - Amx) * iL;
      bt1[2] = (U1[2] - Amy) * iL;
      bt1[3] = (U1[3] - Amz) * iL;
      bt1[4] = (calE - AE) * iL;
      L1 = Lc;
#pragma unroll
      for (int v = 0; v < NV; ++v) sm[(LA_B + v) * NPOS + tid] = bt1[v];
    }
    // b~ adjoint of plane p-1 from its -x / -y faces when it is their upwind
    // (right) cell
    double btb1[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) btb1[v] = 0.0;
    if (p - 1 >= z0 && p - 1 < z1) {
      const double usxm = sm[(LA_F + 0) * NPOS + pxm];
      if (!(usxm >= 0.0)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) btb1[v] += (lx * (nb1[v] - sm[(nbs + v) * NPOS + pxm])) * usxm;
      }
      const double usym = sm[(LA_F + 2) * NPOS + pym];
      if (!(usym >= 0.0)) {
#pragma unroll
        for (int v = 0; v < NV; ++v) btb1[v] += (ly * (nb1[v] - sm[(nbs + v) * NPOS + pym])) * usym;
      }
    }
    // own lateral acoustic faces of plane p (forward)
    double Fn[6];
    if ((p >= z0 - 1) && (p <= z1)) {
      face_lat<LM>(P, q0.rc, q0.irc, q0.ic, q0.p, q0.u[0], sm[(LA_XA + 0) * NPOS + pxp],
                   sm[(LA_XA + 1) * NPOS + pxp], sm[(LA_XA + 2) * NPOS + pxp], sm[(LA_XA + 3) * NPOS + pxp],
                   sm[(LA_XA + 4) * NPOS + pxp], Fn[0], Fn[1], Fn[2]);
      face_lat<LM>(P, q0.rc, q0.irc, q0.ic, q0.p, q0.u[1], sm[(LA_XA + 0) * NPOS + pyp],
                   sm[(LA_XA + 1) * NPOS + pyp], sm[(LA_XA + 2) * NPOS + pyp], sm[(LA_XA + 3) * NPOS + pyp],
                   sm[(LA_XA + 5) * NPOS + pyp], Fn[3], Fn[4], Fn[5]);
    } else {
#pragma unroll
      for (int i = 0; i < 6; ++i) Fn[i] = 0.0;
    }
    __syncthreads();  // ------------------------------------------- bar 1b

    // ======================= phase 3 =======================================
    sm[(LA_F + 0) * NPOS + tid] = Fn[0];
    sm[(LA_F + 1) * NPOS + tid] = Fn[1];
    sm[(LA_F + 2) * NPOS + tid] = Fn[3];
    sm[(LA_F + 3) * NPOS + tid] = Fn[4];
    {
      // transport reverse of the own +x / +y faces of plane p-1
      const int m = p - 1;
      if (m >= z0 && m < z1) {
        const long long cell = col + PS * m;
#pragma unroll
        for (int dir = 0; dir < 2; ++dir) {
          const int nb = dir == 0 ? pxp : pyp;
          const double lam_a = dir == 0 ? lx : ly;
          const double us = Fo1[3 * dir + 0];
          const double pi = Fo1[3 * dir + 1];
          const bool upL = us >= 0.0;
          double Gb[NV], bu[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            Gb[v] = lam_a * (sm[(nbs + v) * NPOS + nb] - nb1[v]);
            const double bn = sm[(LA_B + v) * NPOS + nb];
            bu[v] = upL ? bt1[v] : bn;
          }
          double usb = 0.0;
#pragma unroll
          for (int v = 0; v < NV - 1; ++v) usb += Gb[v] * bu[v];
          usb += Gb[NV - 1] * (bu[NV - 1] + pi);
          const double pib = Gb[1 + dir] + Gb[NV - 1] * us;
          if (upL) {
#pragma unroll
            for (int v = 0; v < NV; ++v) btb1[v] += Gb[v] * us;
          }
          if (out) {
            io.W[(AF_FB + 2 * dir + 0) * N + cell] = usb;
            io.W[(AF_FB + 2 * dir + 1) * N + cell] = pib;
          }
        }
      }
      // transport reverse of the vertical face (p-2 | p-1)
      if ((p - 1 >= z0) && (p - 1 <= z1)) {
        const bool wall = wall_face_below(P, p - 2);
        double Gb[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Gb[v] = lz * (nb1[v] - nbar_v(P, v, phi2, l2));
        double usb = 0.0, pib = Gb[3];
        if (!wall) {
          const bool upL = zAus >= 0.0;
          double bu[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) bu[v] = upL ? bt2[v] : bt1[v];
#pragma unroll
          for (int v = 0; v < NV - 1; ++v) usb += Gb[v] * bu[v];
          usb += Gb[NV - 1] * (bu[NV - 1] + zApi);
          pib += Gb[NV - 1] * zAus;
          if (upL) {
#pragma unroll
            for (int v = 0; v < NV; ++v) btb2[v] += Gb[v] * zAus;
          } else {
#pragma unroll
            for (int v = 0; v < NV; ++v) btb1[v] += Gb[v] * zAus;
          }
        }
        if (out && p - 2 >= z0 && p - 2 < z1) {
          const long long cell = col + PS * (p - 2);
          io.W[(AF_FB + 4) * N + cell] = usb;
          io.W[(AF_FB + 5) * N + cell] = pib;
        }
      }
      // acoustic cell values of plane p-2, reversed; lam^n starts there
      if (p - 2 >= z0 && p - 2 < z1) {
        const double iL = rcp_nr(L2);
        double Lb = 0.0, Ab[NV], consb[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          consb[v] = btb2[v] * iL;
          Ab[v] = -btb2[v] * iL;
          Lb += btb2[v] * bt2[v];
        }
        Lb = -Lb * iL;
        consb[0] += phi2 * consb[NV - 1];  // calE = E + rho Phi
        // A_mz = lam_z ((Pi+ - Pi-) - S-bar); the update adds lam_z S-bar to m_z
        const double sbb = -lz * Ab[3] + lz * l2[3];
        const long long cell = col + PS * (p - 2);
        if (out) {
          io.W[(AF_CB + 0) * N + cell] = Lb;
          io.W[(AF_CB + 1) * N + cell] = Ab[1];
          io.W[(AF_CB + 2) * N + cell] = Ab[2];
          io.W[(AF_CB + 3) * N + cell] = Ab[3];
          io.W[(AF_CB + 4) * N + cell] = Ab[4];
          io.W[(AF_CB + 5) * N + cell] = sbb;
#pragma unroll
          for (int v = 0; v < NV; ++v) io.lam0[cell + v * N] = l2[v] + consb[v];
        }
      }
    }
    // rotate the vertical window
    q1 = q0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      U1[v] = Uc[v];
      l2[v] = l1[v];
      l1[v] = l0[v];
      bt2[v] = bt1[v];
      btb2[v] = btb1[v];
    }
    L2 = L1;
    zAus = zBus; zApi = zBpi; zAP = zBP; zAS = zBS;
#pragma unroll
    for (int i = 0; i < 6; ++i) Fo1[i] = Fn[i];
  }
}

template <bool LM, int EX, int EY>
__global__ void __launch_bounds__(EX* EY) k_adjf_a(Params P, AdjIOF io) {
  __shared__ double sm[LA_TOTAL * EX * EY];
  const double dt = *io.dt;
  const double lx = dt / P.dx[0], ly = dt / P.dx[1], lz = dt / P.dx[2];
  const long long total = (long long)io.ntx * io.nty * P.nz;
  const int G = gridDim.x, b = blockIdx.x;
  const int lw = xcd_share(b, G);
  long long cur = total * lw / G;
  const long long stop = total * (lw + 1) / G;
  while (cur < stop) {
    const int tile = (int)(cur / P.nz);
    const int z0 = (int)(cur % P.nz);
    const int z1 = (int)min((long long)P.nz, (long long)z0 + (stop - cur));
    cur += z1 - z0;
    adj_march_a<LM, EX, EY>(P, io, sm, tile % io.ntx, tile / io.ntx, z0, z1, lx, ly, lz);
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// March V: viscous and heat-flux reverse
// ------------------------------------------------------------------------
enum {
  LV_V = 0,    // ux, uy, uz, T of plane p-1
  LV_DZ = 4,   // u(p) - u(p-2)
  LV_NB = 7,   // nbar of plane p-1
  LV_MX = 12,  // messages of the +x face of plane p-1 (8)
  LV_MY = 20,  // messages of the +y face of plane p-1 (8)
  LV_MZ = 28,  // messages of the face (p-2 | p-1) (4)
  LV_TOTAL = 32
};

template <int EX, int EY>
__device__ __forceinline__ void adj_march_v(const Params& P, const AdjIOF& io, double* __restrict__ sm, const int tx,
                                            const int ty, const int z0, const int z1, const double lx,
                                            const double ly, const double lz, double& mu_acc, double& ka_acc) {
  constexpr int NV = 5;
  constexpr int NPOS = EX * EY;
  constexpr int TX = EX - 4, TY = EY - 4;
  const long long PS = (long long)P.nx * P.ny;
  const long long N = P.ncell;
  const int tid = threadIdx.x;
  const int px = tid % EX, py = tid / EX;
  const bool hxp = px + 1 < EX, hxm = px > 0, hyp = py + 1 < EY, hym = py > 0;
  const int pxp = hxp ? tid + 1 : tid, pxm = hxm ? tid - 1 : tid;
  const int pyp = hyp ? tid + EX : tid, pym = hym ? tid - EX : tid;
  const int pxpyp = (hxp && hyp) ? tid + EX + 1 : tid;
  const int pxpym = (hxp && hym) ? tid - EX + 1 : tid;
  const int pxmyp = (hxm && hyp) ? tid + EX - 1 : tid;
  const int pxmym = (hxm && hym) ? tid - EX - 1 : tid;
  const int gx = tx * TX + px - 2, gy = ty * TY + py - 2;
  const int cx = resolve_lat(gx, P.nx, P.bcx), cy = resolve_lat(gy, P.ny, P.bcy);
  const long long col = (long long)cx + (long long)P.nx * cy;
  const bool out = px >= 2 && px < EX - 2 && gx < P.nx && py >= 2 && py < EY - 2 && gy < P.ny;
  // owners of faces whose stencil reaches an output cell
  const bool visX = px >= 1 && px <= EX - 3 && py >= 1 && py <= EY - 2;
  const bool visY = px >= 1 && px <= EX - 2 && py >= 1 && py <= EY - 3;
  const bool visZ = px >= 1 && px <= EX - 2 && py >= 1 && py <= EY - 2;
  const bool zper = P.bcz[0] == BC_PERIODIC;
  const bool wlo = P.bcz[0] == BC_WALL, whi = P.bcz[1] == BC_WALL;
  const double qx = P.qidx[0], qy = P.qidx[1], qz = P.qidx[2];

  double Unx[NV], Lnx[NV];
  double l1[NV], l2[NV];           // lam^{n+1} of planes p-1, p-2 (0 at wall ghosts)
  double u1[3] = {0, 0, 0}, T1 = 0.0, u2[3] = {0, 0, 0}, T2 = 0.0;  // planes p-1, p-2
  double dX2[4] = {0, 0, 0, 0};    // tangential differences of plane p-2
  double vbB[4] = {0, 0, 0, 0}, vbC[4] = {0, 0, 0, 0};  // (u, T) adjoints of planes p-1, p-2
  double gcar[5] = {0, 0, 0, 0, 0};  // bottom wall ghost's (rho, u, T) share of plane 0
#pragma unroll
  for (int v = 0; v < NV; ++v) l1[v] = l2[v] = 0.0;
  int ghost_nx;
  {
    const int src = plane_src(P, z0 - 2, ghost_nx);
    const long long b = col + PS * src;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Unx[v] = io.U[b + v * N];
      Lnx[v] = io.lam1[b + v * N];  // a valid cell in every case; zeroed at wall ghosts when used
    }
  }
  for (int p = z0 - 2; p <= z1 + 1; ++p) {
    // ======================= phase 1 =======================================
    const int ghost = ghost_nx;
    double Uc[NV], l0[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Uc[v] = Unx[v];
      l0[v] = ghost >= 0 ? 0.0 : Lnx[v];  // wall ghosts are not updated: no lam
    }
    if (p + 1 <= z1 + 1) {
      const int src = plane_src(P, p + 1, ghost_nx);
      const long long b = col + PS * src;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        Unx[v] = io.U[b + v * N];
        Lnx[v] = io.lam1[b + v * N];
      }
    }
    Prim<3> q0 = cons_to_prim<3>(P, Uc);
    if (ghost >= 0) {
      const int kg = ghost == 0 ? -1 : P.nz;
      const int ki = ghost == 0 ? 0 : P.nz - 1;
      q0 = wall_ghost<3>(P, q0, ghost, phi_at(P, kg) - phi_at(P, ki));
    }
    const double phi1 = phi_at(P, p - 1), phi2 = phi_at(P, p - 2);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sm[(LV_V + k) * NPOS + tid] = u1[k];
      sm[(LV_DZ + k) * NPOS + tid] = q0.u[k] - u2[k];
    }
    sm[(LV_V + 3) * NPOS + tid] = T1;
    double nb1[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      nb1[v] = nbar_v(P, v, phi1, l1);
      sm[(LV_NB + v) * NPOS + tid] = nb1[v];
    }
    __syncthreads();  // ------------------------------------------- bar 1

    // ======================= phase 2 =======================================
    double vbA[4] = {0, 0, 0, 0};   // (u, T) adjoint of plane p
    double Mo[20];
#pragma unroll
    for (int i = 0; i < 20; ++i) Mo[i] = 0.0;
    // tangential differences of plane p-1 (vertical faces)
    double dX1[4] = {0.0, 0.0, 0.0, 0.0};
    {
      dX1[0] = sm[(LV_V + 0) * NPOS + pxp] - sm[(LV_V + 0) * NPOS + pxm];
      dX1[1] = sm[(LV_V + 2) * NPOS + pxp] - sm[(LV_V + 2) * NPOS + pxm];
      dX1[2] = sm[(LV_V + 1) * NPOS + pyp] - sm[(LV_V + 1) * NPOS + pym];
      dX1[3] = sm[(LV_V + 2) * NPOS + pyp] - sm[(LV_V + 2) * NPOS + pym];
    }
    // lateral faces of plane m = p-1
    const int m = p - 1;
    const bool latV = (zper || (m >= 0 && m < P.nz)) && m >= z0 - 1 && m <= z1;
    const bool own_m = out && m >= z0 && m < z1;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      if (!latV) continue;
      const int nb = dir == 0 ? pxp : pyp;
      const double lam_a = dir == 0 ? lx : ly;
      double Gb[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Gb[v] = lam_a * (sm[(LV_NB + v) * NPOS + nb] - nb1[v]);
      double uR[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) uR[k] = sm[(LV_V + k) * NPOS + nb];
      const double TR = sm[(LV_V + 3) * NPOS + nb];
      double g[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) g[a][k] = 0.0;
      const double idn = P.idx[dir];
#pragma unroll
      for (int k = 0; k < 3; ++k) g[dir][k] = (uR[k] - u1[k]) * idn;
      const int a = 1 - dir;
      const int pa_p = a == 1 ? pyp : pxp;
      const int pa_m = a == 1 ? pym : pxm;
      const int nb_p = a == 1 ? (dir == 0 ? pxpyp : pyp) : (dir == 1 ? pxpyp : pxp);
      const int nb_m = a == 1 ? (dir == 0 ? pxpym : pym) : (dir == 1 ? pxmyp : pxm);
      const double qa = P.qidx[a];
      g[a][dir] = ((sm[(LV_V + dir) * NPOS + pa_p] - sm[(LV_V + dir) * NPOS + pa_m]) +
                   (sm[(LV_V + dir) * NPOS + nb_p] - sm[(LV_V + dir) * NPOS + nb_m])) * qa;
      g[a][a] = ((sm[(LV_V + a) * NPOS + pa_p] - sm[(LV_V + a) * NPOS + pa_m]) +
                 (sm[(LV_V + a) * NPOS + nb_p] - sm[(LV_V + a) * NPOS + nb_m])) * qa;
      g[2][dir] = ((q0.u[dir] - u2[dir]) + sm[(LV_DZ + dir) * NPOS + nb]) * qz;
      g[2][2] = ((q0.u[2] - u2[2]) + sm[(LV_DZ + 2) * NPOS + nb]) * qz;
      double uLb[3], uRb[3], TLb, TRb, gb[3][3], mub, kab;
      visc_adj(P, dir, idn, g, u1, uR, T1, TR, Gb, uLb, uRb, TLb, TRb, gb, mub, kab);
#pragma unroll
      for (int k = 0; k < 3; ++k) vbB[k] += uLb[k];
      vbB[3] += TLb;
      // own column's share of the vertical tangential rows (planes p, p-2)
      vbA[dir] += qz * gb[2][dir];
      vbA[2] += qz * gb[2][2];
      vbC[dir] -= qz * gb[2][dir];
      vbC[2] -= qz * gb[2][2];
      double* M = Mo + 8 * dir;
      M[0] = uRb[0];
      M[1] = uRb[1];
      M[2] = uRb[2];
      M[3] = TRb;
      M[4] = gb[a][dir];
      M[5] = gb[a][a];
      M[6] = gb[2][dir];
      M[7] = gb[2][2];
      if (own_m) {
        mu_acc += mub;
        ka_acc += kab;
      }
    }
    // vertical face (p-2 | p-1)
    if ((p - 1 >= z0) && (p - 1 <= z1)) {
      double Gb[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Gb[v] = lz * (nb1[v] - nbar_v(P, v, phi2, l2));
      double g[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 0; k < 3; ++k) g[a][k] = 0.0;
      const double idn = P.idx[2];
#pragma unroll
      for (int k = 0; k < 3; ++k) g[2][k] = (u1[k] - u2[k]) * idn;
      g[0][0] = (dX2[0] + dX1[0]) * qx;
      g[0][2] = (dX2[1] + dX1[1]) * qx;
      g[1][1] = (dX2[2] + dX1[2]) * qy;
      g[1][2] = (dX2[3] + dX1[3]) * qy;
      double uLb[3], uRb[3], TLb, TRb, gb[3][3], mub, kab;
      visc_adj(P, 2, idn, g, u2, u1, T2, T1, Gb, uLb, uRb, TLb, TRb, gb, mub, kab);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        vbC[k] += uLb[k];
        vbB[k] += uRb[k];
      }
      vbC[3] += TLb;
      vbB[3] += TRb;
      Mo[16] = gb[0][0];
      Mo[17] = gb[0][2];
      Mo[18] = gb[1][1];
      Mo[19] = gb[1][2];
      const bool own = (p - 2 >= z0 && p - 2 < z1) || (p - 2 == -1 && z0 == 0 && wlo);
      if (out && own) {
        mu_acc += mub;
        ka_acc += kab;
      }
    }
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      sm[(LV_MX + i) * NPOS + tid] = Mo[i];
      sm[(LV_MY + i) * NPOS + tid] = Mo[8 + i];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) sm[(LV_MZ + i) * NPOS + tid] = Mo[16 + i];
    __syncthreads();  // ------------------------------------------- bar 2

    // ======================= phase 3 =======================================
    {
      // normal parts of the -x / -y faces of plane p-1
#pragma unroll
      for (int i = 0; i < 4; ++i) vbB[i] += sm[(LV_MX + i) * NPOS + pxm] + sm[(LV_MY + i) * NPOS + pym];
      // lateral tangential rows of the x faces (y rows) and y faces (x rows)
      vbB[0] += qy * ((sm[(LV_MX + 4) * NPOS + pym] - sm[(LV_MX + 4) * NPOS + pyp]) +
                      (sm[(LV_MX + 4) * NPOS + pxmym] - sm[(LV_MX + 4) * NPOS + pxmyp]));
      vbB[1] += qy * ((sm[(LV_MX + 5) * NPOS + pym] - sm[(LV_MX + 5) * NPOS + pyp]) +
                      (sm[(LV_MX + 5) * NPOS + pxmym] - sm[(LV_MX + 5) * NPOS + pxmyp]));
      vbB[1] += qx * ((sm[(LV_MY + 4) * NPOS + pxm] - sm[(LV_MY + 4) * NPOS + pxp]) +
                      (sm[(LV_MY + 4) * NPOS + pxmym] - sm[(LV_MY + 4) * NPOS + pxpym]));
      vbB[0] += qx * ((sm[(LV_MY + 5) * NPOS + pxm] - sm[(LV_MY + 5) * NPOS + pxp]) +
                      (sm[(LV_MY + 5) * NPOS + pxmym] - sm[(LV_MY + 5) * NPOS + pxpym]));
      // vertical tangential rows of the -x / -y faces (planes p and p-2)
      {
        const double a0 = qz * sm[(LV_MX + 6) * NPOS + pxm], a2 = qz * sm[(LV_MX + 7) * NPOS + pxm];
        const double b1 = qz * sm[(LV_MY + 6) * NPOS + pym], b2 = qz * sm[(LV_MY + 7) * NPOS + pym];
        vbA[0] += a0;
        vbA[2] += a2;
        vbA[1] += b1;
        vbA[2] += b2;
        vbC[0] -= a0;
        vbC[2] -= a2;
        vbC[1] -= b1;
        vbC[2] -= b2;
      }
      // lateral tangential rows of the vertical faces of the neighbouring columns
      {
        const double x0 = qx * (sm[(LV_MZ + 0) * NPOS + pxm] - sm[(LV_MZ + 0) * NPOS + pxp]);
        const double x2 = qx * (sm[(LV_MZ + 1) * NPOS + pxm] - sm[(LV_MZ + 1) * NPOS + pxp]);
        const double y1 = qy * (sm[(LV_MZ + 2) * NPOS + pym] - sm[(LV_MZ + 2) * NPOS + pyp]);
        const double y2 = qy * (sm[(LV_MZ + 3) * NPOS + pym] - sm[(LV_MZ + 3) * NPOS + pyp]);
        vbC[0] += x0;
        vbB[0] += x0;
        vbC[2] += x2;
        vbB[2] += x2;
        vbC[1] += y1;
        vbB[1] += y1;
        vbC[2] += y2;
        vbB[2] += y2;
      }
      if (p - 2 == -1 && z0 == 0 && wlo) {
        // bottom wall ghost (plane -1, built from plane 0 = p-1): its
        // adjoints go to the primitives of plane 0 through the ghost map
        double U0c[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) U0c[v] = io.U[col + v * N];
        const Prim<3> qi = cons_to_prim<3>(P, U0c);
        const double d = phi_at(P, -1) - phi_at(P, 0);
        const Prim<3> gq = wall_ghost<3>(P, qi, 0, d);
        const double gb[9] = {0.0, vbC[0], vbC[1], vbC[2], 0.0, 0.0, 0.0, 0.0, vbC[3]};
        double ib[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        ghost_adj(P, 0, d, qi, gq, gb, ib);
        gcar[0] = ib[0];
        gcar[1] = ib[1];
        gcar[2] = ib[2];
        gcar[3] = ib[3];
        gcar[4] = ib[8];
      }
      if (p - 2 >= z0 && p - 2 < z1) {
        // (rho, u, T) adjoints of plane p-2, for the primitive map of B
        const long long cell = col + PS * (p - 2);
        double pb[9] = {0.0, vbC[0], vbC[1], vbC[2], 0.0, 0.0, 0.0, 0.0, vbC[3]};
        if (p - 2 == P.nz - 1 && whi) {
          // top wall ghost (plane nz = p-1, built from this plane)
          double Uo[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) Uo[v] = io.U[cell + v * N];
          const Prim<3> qo = cons_to_prim<3>(P, Uo);
          const double d = phi_at(P, P.nz) - phi_at(P, P.nz - 1);
          const Prim<3> gq = wall_ghost<3>(P, qo, 1, d);
          const double gb[9] = {0.0, vbB[0], vbB[1], vbB[2], 0.0, 0.0, 0.0, 0.0, vbB[3]};
          ghost_adj(P, 1, d, qo, gq, gb, pb);
        }
        if ((p - 2 == 0) && wlo) {
          pb[0] += gcar[0];
          pb[1] += gcar[1];
          pb[2] += gcar[2];
          pb[3] += gcar[3];
          pb[8] += gcar[4];
        }
        if (out) {
          io.W[(AF_PV + 0) * N + cell] = pb[0];
          io.W[(AF_PV + 1) * N + cell] = pb[1];
          io.W[(AF_PV + 2) * N + cell] = pb[2];
          io.W[(AF_PV + 3) * N + cell] = pb[3];
          io.W[(AF_PV + 4) * N + cell] = pb[8];
        }
      }
    }
    // rotate the vertical window
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      u2[k] = u1[k];
      u1[k] = q0.u[k];
    }
    T2 = T1;
    T1 = q0.T;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      l2[v] = l1[v];
      l1[v] = l0[v];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      vbC[k] = vbB[k];
      vbB[k] = vbA[k];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) dX2[i] = dX1[i];
  }
}

template <int EX, int EY>
__global__ void __launch_bounds__(EX* EY) k_adjf_v(Params P, AdjIOF io) {
  constexpr int NPOS = EX * EY;
  __shared__ double sm[LV_TOTAL * NPOS];
  __shared__ double red[2][(NPOS + 63) / 64];
  const double dt = *io.dt;
  const double lx = dt / P.dx[0], ly = dt / P.dx[1], lz = dt / P.dx[2];
  const long long total = (long long)io.ntx * io.nty * P.nz;
  const int G = gridDim.x, b = blockIdx.x;
  const int lw = xcd_share(b, G);
  long long cur = total * lw / G;
  const long long stop = total * (lw + 1) / G;
  double mu_acc = 0.0, ka_acc = 0.0;
  while (cur < stop) {
    const int tile = (int)(cur / P.nz);
    const int z0 = (int)(cur % P.nz);
    const int z1 = (int)min((long long)P.nz, (long long)z0 + (stop - cur));
    cur += z1 - z0;
    adj_march_v<EX, EY>(P, io, sm, tile % io.ntx, tile / io.ntx, z0, z1, lx, ly, lz, mu_acc, ka_acc);
    __syncthreads();
  }
  // workgroup sums of the mu / kappa partials in a fixed order (a partial
  // last wave has no lanes past NPOS: its missing lanes add zeros)
  const int tid = threadIdx.x;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    mu_acc += __shfl_xor(mu_acc, off, 64);
    ka_acc += __shfl_xor(ka_acc, off, 64);
  }
  if ((tid & 63) == 0) {
    red[0][tid >> 6] = mu_acc;
    red[1][tid >> 6] = ka_acc;
  }
  __syncthreads();
  if (tid == 0) {
    double a = 0.0, c = 0.0;
    for (int w = 0; w < (NPOS + 63) / 64; ++w) {
      a += red[0][w];
      c += red[1][w];
    }
    io.partial[2 * b] = a;
    io.partial[2 * b + 1] = c;
  }
}
// ------------------------------------------------------------------------
// March B
// ------------------------------------------------------------------------
enum {
  LB_XA = 0,   // rc, 1/rc, 1/c, p, ux, uy of plane p
  LB_CB = 6,   // adjoints of L, A_mx, A_my, A_E of plane p
  LB_RX = 10,  // right-cell adjoints of the +x face of plane p (u_x, p, rc, 1/rc, 1/c)
  LB_RY = 15,  // same, +y face
  LB_TOTAL = 20
};

template <bool LM, int EX, int EY>
__device__ __forceinline__ void adj_march_b(const Params& P, const AdjIOF& io, double* __restrict__ sm, const int tx,
                                            const int ty, const int z0, const int z1, const double lx,
                                            const double ly, const double lz) {
  constexpr int NV = 5;
  constexpr int NPOS = EX * EY;
  constexpr int TX = EX - 2, TY = EY - 2;
  const long long PS = (long long)P.nx * P.ny;
  const long long N = P.ncell;
  const int tid = threadIdx.x;
  const int px = tid % EX, py = tid / EX;
  const int pxp = px + 1 < EX ? tid + 1 : tid, pxm = px > 0 ? tid - 1 : tid;
  const int pyp = py + 1 < EY ? tid + EX : tid, pym = py > 0 ? tid - EX : tid;
  const int gx = tx * TX + px - 1, gy = ty * TY + py - 1;
  const int cx = resolve_lat(gx, P.nx, P.bcx), cy = resolve_lat(gy, P.ny, P.bcy);
  const long long col = (long long)cx + (long long)P.nx * cy;
  const bool out = px >= 1 && px < EX - 1 && gx < P.nx && py >= 1 && py < EY - 1 && gy < P.ny;
  // owners of the lateral faces some output needs
  const bool ownX = px <= EX - 2 && py >= 1 && py <= EY - 2;
  const bool ownY = py <= EY - 2 && px >= 1 && px <= EX - 2;
  const bool wlo = P.bcz[0] == BC_WALL, whi = P.bcz[1] == BC_WALL;

  // plane data, loaded one plane ahead: U and the acoustic workspace fields
  // of plane q (zeroed at wall ghosts when used), and the partial lam^n and
  // viscous (rho, u, T) adjoints of plane q-1, finished in the trip that
  // uses them (all addresses valid: ghost and out-of-range planes load a
  // clamped plane that is never used)
  constexpr int NW = AF_PV;
  double Un[NV], Wn[NW], Ln[NV], Vn[5];
  int ghn;
  // Halo positions load only what they publish or use (U; L, A_mx, A_my,
  // A_E; the (u*, Pi*) adjoints of the lateral face they own): the rest is
  // read by output cells only.  The loads land one trip later, so the lanes
  // that skip them leave registers that are never read.
  const bool hx = !out && px == 0, hy = !out && py == 0;  // owners of an output's -x / -y face
  auto load = [&](int q) __attribute__((always_inline)) {
    const int src = plane_src(P, q, ghn);
    const long long cs = col + PS * src;
#pragma unroll
    for (int v = 0; v < NV; ++v) Un[v] = io.U[cs + v * N];
    if (ghn >= 0) {  // uniform: wall ghosts carry no adjoints
#pragma unroll
      for (int i = 0; i < NW; ++i) Wn[i] = 0.0;
    } else {
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const bool need = out || i == AF_CB + 0 || i == AF_CB + 1 || i == AF_CB + 2 || i == AF_CB + 4 ||
                          (hx && (i == AF_FB + 0 || i == AF_FB + 1)) || (hy && (i == AF_FB + 2 || i == AF_FB + 3));
        Wn[i] = need ? io.W[i * N + cs] : 0.0;
      }
    }
    if (out) {
      const long long cf = col + PS * min(max(q - 1, 0), P.nz - 1);
#pragma unroll
      for (int v = 0; v < NV; ++v) Ln[v] = io.lam0[cf + v * N];
#pragma unroll
      for (int k = 0; k < 5; ++k) Vn[k] = io.W[(AF_PV + k) * N + cf];
    }
  };
  Prim<3> q1 = Prim<3>{};
  double U1[NV] = {0, 0, 0, 0, 0};
  double pb1[8];                        // face adjoints of (rho, u, p, rc, 1/rc, 1/c) of plane p-1
  double cb1[4] = {0, 0, 0, 0};         // adjoints of L, A_mz, A_E, S-bar of plane p-1
  double fz1[2] = {0, 0};               // (u*, Pi*) adjoints of the face (p-1 | p)
#pragma unroll
  for (int k = 0; k < 8; ++k) pb1[k] = 0.0;
  load(z0 - 1);

  for (int p = z0 - 1; p <= z1; ++p) {
    const int ghost = ghn;
    double Uc[NV], w[NW], lo[NV], pv[5];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      Uc[v] = Un[v];
      lo[v] = Ln[v];
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = Wn[i];
#pragma unroll
    for (int k = 0; k < 5; ++k) pv[k] = Vn[k];
    const bool fin = out && p - 1 >= z0 && p - 1 < z1;
    if (p + 1 <= z1) load(p + 1);
    const double* cb = w + AF_CB;
    const double* fb = w + AF_FB;
    Prim<3> q0 = cons_to_prim<3>(P, Uc);
    if (ghost >= 0) {
      const int kg = ghost == 0 ? -1 : P.nz;
      const int ki = ghost == 0 ? 0 : P.nz - 1;
      q0 = wall_ghost<3>(P, q0, ghost, phi_at(P, kg) - phi_at(P, ki));
    }
    sm[(LB_XA + 0) * NPOS + tid] = q0.rc;
    sm[(LB_XA + 1) * NPOS + tid] = q0.irc;
    sm[(LB_XA + 2) * NPOS + tid] = q0.ic;
    sm[(LB_XA + 3) * NPOS + tid] = q0.p;
    sm[(LB_XA + 4) * NPOS + tid] = q0.u[0];
    sm[(LB_XA + 5) * NPOS + tid] = q0.u[1];
    sm[(LB_CB + 0) * NPOS + tid] = cb[0];
    sm[(LB_CB + 1) * NPOS + tid] = cb[1];
    sm[(LB_CB + 2) * NPOS + tid] = cb[2];
    sm[(LB_CB + 3) * NPOS + tid] = cb[4];
    __syncthreads();  // ------------------------------------------- bar 1

    double pb0[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) pb0[k] = 0.0;
    const bool lat = p >= z0 && p < z1;
#pragma unroll
    for (int dir = 0; dir < 2; ++dir) {
      if (!(lat && (dir == 0 ? ownX : ownY))) continue;
      const int nb = dir == 0 ? pxp : pyp;
      const double lam_a = dir == 0 ? lx : ly;
      const double rcR = sm[(LB_XA + 0) * NPOS + nb], ircR = sm[(LB_XA + 1) * NPOS + nb];
      const double icR = sm[(LB_XA + 2) * NPOS + nb], pR = sm[(LB_XA + 3) * NPOS + nb];
      const double uR = sm[(LB_XA + 4 + dir) * NPOS + nb];
      double us, pi, Pf;
      face_lat<LM>(P, q0.rc, q0.irc, q0.ic, q0.p, q0.u[dir], rcR, ircR, icR, pR, uR, us, pi, Pf);
      const double usb = fb[2 * dir] + lam_a * (cb[0] - sm[(LB_CB + 0) * NPOS + nb]);
      const double pib = fb[2 * dir + 1] + lam_a * (cb[1 + dir] - sm[(LB_CB + 1 + dir) * NPOS + nb]);
      const double Pb = lam_a * (cb[4] - sm[(LB_CB + 3) * NPOS + nb]);
      double bl[6], br[6];
      face_adj<LM>(P, false, false, 0.0, us, pi, 0.0, q0.u[dir], q0.p, q0.rc, q0.irc, q0.ic, uR, pR, rcR, ircR, icR,
                   usb, pib, Pb, 0.0, bl, br);
      pb0[1 + dir] += bl[1];
      pb0[4] += bl[2];
      pb0[5] += bl[3];
      pb0[6] += bl[4];
      pb0[7] += bl[5];
      const int R = dir == 0 ? LB_RX : LB_RY;
      sm[(R + 0) * NPOS + tid] = br[1];
      sm[(R + 1) * NPOS + tid] = br[2];
      sm[(R + 2) * NPOS + tid] = br[3];
      sm[(R + 3) * NPOS + tid] = br[4];
      sm[(R + 4) * NPOS + tid] = br[5];
    }
    // vertical face (p-1 | p)
    if (out && p >= z0 && p <= z1) {
      const bool wall = wall_face_below(P, p - 1);
      const double dphi = phi_at(P, p) - phi_at(P, p - 1);
      double us, pi, Pf, S;
      face_vert<LM, 3>(P, q1, q0, dphi, wall, us, pi, Pf, S);
      double usb = fz1[0], pib = fz1[1];
      if (p - 1 == -1 && wlo) {
        // bottom wall face: no transport; Pi* carries lam_z (nbar(0) - 0)
        usb = 0.0;
        pib = lz * io.lam1[col + 3 * N];
      }
      usb += lz * (cb1[0] - cb[0]);
      pib += lz * (cb1[1] - cb[3]);
      const double Pb = lz * (cb1[2] - cb[4]);
      const double Sb = 0.5 * cb1[3] + 0.5 * cb[5];
      double bl[6], br[6];
      face_adj<LM>(P, true, wall, dphi, us, pi, S, q1.u[2], q1.p, q1.rc, q1.irc, q1.ic, q0.u[2], q0.p, q0.rc,
                   q0.irc, q0.ic, usb, pib, Pb, Sb, bl, br);
      pb1[0] += bl[0];
      pb1[3] += bl[1];
      pb1[4] += bl[2];
      pb1[5] += bl[3];
      pb1[6] += bl[4];
      pb1[7] += bl[5];
      pb0[0] += br[0];
      pb0[3] += br[1];
      pb0[4] += br[2];
      pb0[5] += br[3];
      pb0[6] += br[4];
      pb0[7] += br[5];
    }
    __syncthreads();  // ------------------------------------------- bar 2
    if (out && lat) {
      pb0[1] += sm[(LB_RX + 0) * NPOS + pxm];
      pb0[4] += sm[(LB_RX + 1) * NPOS + pxm];
      pb0[5] += sm[(LB_RX + 2) * NPOS + pxm];
      pb0[6] += sm[(LB_RX + 3) * NPOS + pxm];
      pb0[7] += sm[(LB_RX + 4) * NPOS + pxm];
      pb0[2] += sm[(LB_RY + 0) * NPOS + pym];
      pb0[4] += sm[(LB_RY + 1) * NPOS + pym];
      pb0[5] += sm[(LB_RY + 2) * NPOS + pym];
      pb0[6] += sm[(LB_RY + 3) * NPOS + pym];
      pb0[7] += sm[(LB_RY + 4) * NPOS + pym];
    }
    if (out && p - 1 == -1 && wlo && z0 == 0) {
      // bottom wall ghost (plane -1 = p-1, built from plane 0 = p): its
      // share of lam^n of plane 0 joins the partial lam^n of plane 0 that
      // load(1) fetched at the top of this trip (z1 >= 1)
      const double gb[9] = {pb1[0], pb1[1], pb1[2], pb1[3], pb1[4], pb1[5], pb1[6], pb1[7], 0.0};
      double ib[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      ghost_adj(P, 0, phi_at(P, -1) - phi_at(P, 0), q0, q1, gb, ib);
      double gU[NV];
      prim_adj(P, q0, Uc + 1, ib, gU);
#pragma unroll
      for (int v = 0; v < NV; ++v) Ln[v] = Ln[v] + gU[v];
    }
    if (fin) {
      double pb[9] = {pb1[0], pb1[1], pb1[2], pb1[3], pb1[4], pb1[5], pb1[6], pb1[7], 0.0};
      if (p == P.nz && whi) {
        // top wall ghost (plane nz = p, built from plane nz-1 = p-1)
        const double gb[9] = {pb0[0], pb0[1], pb0[2], pb0[3], pb0[4], pb0[5], pb0[6], pb0[7], 0.0};
        ghost_adj(P, 1, phi_at(P, P.nz) - phi_at(P, P.nz - 1), q1, q0, gb, pb);
      }
      // viscous and heat-flux share (march V, which runs when diss)
      if (P.diss) {
        pb[0] += pv[0];
        pb[1] += pv[1];
        pb[2] += pv[2];
        pb[3] += pv[3];
        pb[8] += pv[4];
      }
      double Ub[NV];
      prim_adj(P, q1, U1 + 1, pb, Ub);
      const long long cell = col + PS * (p - 1);
#pragma unroll
      for (int v = 0; v < NV; ++v) io.lam0[cell + v * N] = lo[v] + Ub[v];
    }
    // rotate
    q1 = q0;
#pragma unroll
    for (int v = 0; v < NV; ++v) U1[v] = Uc[v];
#pragma unroll
    for (int k = 0; k < 8; ++k) pb1[k] = pb0[k];
    cb1[0] = cb[0];
    cb1[1] = cb[3];
    cb1[2] = cb[4];
    cb1[3] = cb[5];
    fz1[0] = fb[4];
    fz1[1] = fb[5];
  }
}
template <bool LM, int EX, int EY>
__global__ void __launch_bounds__(EX* EY) k_adjf_b(Params P, AdjIOF io) {
  __shared__ double sm[LB_TOTAL * EX * EY];
  const double dt = *io.dt;
  const double lx = dt / P.dx[0], ly = dt / P.dx[1], lz = dt / P.dx[2];
  const long long total = (long long)io.ntx * io.nty * P.nz;
  const int G = gridDim.x, b = blockIdx.x;
  const int lw = xcd_share(b, G);
  long long cur = total * lw / G;
  const long long stop = total * (lw + 1) / G;
  while (cur < stop) {
    const int tile = (int)(cur / P.nz);
    const int z0 = (int)(cur % P.nz);
    const int z1 = (int)min((long long)P.nz, (long long)z0 + (stop - cur));
    cur += z1 - z0;
    adj_march_b<LM, EX, EY>(P, io, sm, tile % io.ntx, tile / io.ntx, z0, z1, lx, ly, lz);
    __syncthreads();
  }
}

// ------------------------------------------------------------------------
// Host side
// ------------------------------------------------------------------------
template <bool LM, bool DISS>
static hipError_t adjf_t(const Params& P, const double* Un, const double* lam1, double* lam0, const double* d_dt,
                         double* pgrad, void* wadj, hipStream_t s) {
  AdjIOF io;
  io.U = Un;
  io.lam1 = lam1;
  io.lam0 = lam0;
  io.W = (double*)wadj;
  io.partial = io.W + (size_t)AF_NF * P.ncell;
  io.dt = d_dt;
  // A: lam^n = lam^{n+1} + direct term; L, A, S-bar and face adjoints
  io.ntx = (P.nx + AF_AX - 5) / (AF_AX - 4);
  io.nty = (P.ny + AF_AY - 5) / (AF_AY - 4);
  int g = adjf_groups(P, AF_AX, AF_AY, 2, 1);
  hipLaunchKernelGGL((k_adjf_a<LM, AF_AX, AF_AY>), dim3((unsigned)g), dim3(AF_AX * AF_AY), 0, s, P, io);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // V: + viscous and heat-flux terms, mu/kappa derivatives
  if (DISS) {
    io.ntx = (P.nx + AF_VX - 5) / (AF_VX - 4);
    io.nty = (P.ny + AF_VY - 5) / (AF_VY - 4);
    g = adjf_groups(P, AF_VX, AF_VY, 2, 1);
    hipLaunchKernelGGL((k_adjf_v<AF_VX, AF_VY>), dim3((unsigned)g), dim3(AF_VX * AF_VY), 0, s, P, io);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (pgrad) {
      e = launch_adj_params_final(g, io.partial, pgrad, s);
      if (e != hipSuccess) return e;
    }
  }
  // B: + acoustic face-solver terms
  io.ntx = (P.nx + AF_BX - 3) / (AF_BX - 2);
  io.nty = (P.ny + AF_BY - 3) / (AF_BY - 2);
  g = adjf_groups(P, AF_BX, AF_BY, 1, 1);
  hipLaunchKernelGGL((k_adjf_b<LM, AF_BX, AF_BY>), dim3((unsigned)g), dim3(AF_BX * AF_BY), 0, s, P, io);
  return hipGetLastError();
}

hipError_t launch_step_adjoint_fused(const Params& P, const double* Un, const double* lam_np1, double* lam_n,
                                     const double* d_dt, double* d_param_grad, void* wadj, hipStream_t s) {
  const bool lm = P.low_mach != 0, ds = P.diss != 0;
  if (lm && ds) return adjf_t<true, true>(P, Un, lam_np1, lam_n, d_dt, d_param_grad, wadj, s);
  if (lm) return adjf_t<true, false>(P, Un, lam_np1, lam_n, d_dt, d_param_grad, wadj, s);
  if (ds) return adjf_t<false, true>(P, Un, lam_np1, lam_n, d_dt, d_param_grad, wadj, s);
  return adjf_t<false, false>(P, Un, lam_np1, lam_n, d_dt, d_param_grad, wadj, s);
}

}  // namespace ars
