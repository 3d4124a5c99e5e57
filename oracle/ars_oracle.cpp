// ars_oracle.cpp -- plain serial FP64 CPU oracle of the all-regime,
// well-balanced finite-volume step of Padioleau, Tremblin, Audit, Kestener
// and Kokh, "A high performance and portable all-Mach regime flow solver code
// with well-balanced gravity" (arXiv 1903.09043).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
// calls this file; only the test-suite, the smoke check and the CPU baseline
// of the benchmark do.  It shares no code, header, table or constant with the
// HIP path.
//
// The oracle takes the method's steps in the paper's order, on padded
// arrays, one plain loop per step, no fusion and no tiling:
//   O1 ghosts          -- Sec. 4.3 (hydrostatic extrapolation + reflexive
//                         velocity), eq. (well_balanced_formula) solved for
//                         the ghost density; Sec. 4.5.3 fixed-T walls.
//   O2 primitives      -- ideal gas of Sec. 4, p = (gamma-1) rho e, T = p / rho
//                         (R = 1, as p = rho T of Sec. 4.3), c^2 = gamma p / rho.
//   O3 time step       -- CFL reduction ("time step kernel", Sec. 3.2); the
//                         paper gives no formula, the reading is additive
//                         hyperbolic + diffusive rate (dt_mode 2, for the
//                         IMEX step: transport + diffusive, no sound speed).
//   O4 faces           -- acoustic approximate Riemann solver (Sec. 2.1.2):
//                         u*, Pi*, a >= max(rho c), interface gravity S_{i+1/2};
//                         low-Mach factor theta of eq. (low_mach_correction).
//   O5 acoustic cells  -- L_i = 1 + dt/dx [u*]_i and the acoustic update of
//                         Sec. 2.1.2 giving the transported b~ = (b - A)/L.
//   O6 transport       -- upwind b~_{i+1/2} on the sign of u* (Sec. 2.1.3).
//   O7 dissipation     -- first-order viscous and heat fluxes (Sec. 2.2),
//                         Stokes hypothesis, Fourier law.
//   O8 update          -- eq. (all_regime_scheme) summed over directions,
//                         then the relaxation step Psi^{n+1} = Phi (Sec.
//                         2.1.4) realised as E = calE - rho Phi; or, with
//                         energy_form = 1, the non-conservative energy
//                         scheme of App. B (energy without the potential,
//                         source (uS)_i, no relaxation step).
//   O9 validity        -- L > 0, rho > 0, p > 0, finite.
//   IMEX               -- implicit acoustic step (the further work of the
//                         Conclusion): Sec. 2.1.2's acoustic step with its
//                         interface values at the end of the step, a linear
//                         system solved by a direct sparse solver in
//                         oracle/__init__.py; then O5-O9.  See the IMEX
//                         section for the reading and its one unpinned
//                         coefficient.
//
// Multi-dimensional form: unsplit (every face from U^n with one dt, L sums
// all directions), which is how the constant-potential limit (the all-regime
// scheme the paper extends) is posed.
//
// Every routine is templated on the scalar type so the same source, run on
// dual numbers, is the tangent-linear model (the time step is held fixed).
//
// Pins (tests/test_oracle_pins.py): published SplitMix64 outputs, discrete
// hydrostatic equilibrium and Table 1, conservation, closed-form special
// cases (uniform state, contact advection, shear wave, heat flux), exact
// Riemann solutions, the low-Mach behaviour of Sec. 4.2, geometric
// invariants, finite differences of the tangent-linear model and the
// dot-product identity of the dense adjoint, closed forms of the
// diagnostics (uniform states, the gravitational energy of a uniform column,
// Nu = 1 for the conductive profile).  Parity unpinned: the CFL rate and dt
// (orc_max_rate, orc_dt: the paper prints no formula, the rule here is a
// reading); for these only the GPU-versus-oracle comparison applies.
//
// State layout: SoA, var-major: [rho, m_0 .. m_{D-1}, E][cell],
// cell = i + n0*(j + n1*k), E = rho e + rho |u|^2 / 2 (no gravity).

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>
#include <algorithm>
#include <limits>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- scalars --
struct Dual {
  double v, d;
  Dual() : v(0.0), d(0.0) {}
  Dual(double x) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual sqrt_(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline double sqrt_(double a) { return std::sqrt(a); }

inline double val(double x) { return x; }
inline double val(const Dual& x) { return x.v; }

// Non-smooth helpers: the branch taken on the values is the one
// differentiated; ties take the first argument.
template <class S> inline S smax(const S& a, const S& b) { return val(a) >= val(b) ? a : b; }
template <class S> inline S smin(const S& a, const S& b) { return val(a) <= val(b) ? a : b; }
template <class S> inline S sabs(const S& a) { return val(a) >= 0.0 ? a : -a; }

// ----------------------------------------------------------------- config --
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_OUTFLOW = 2 };
enum { TH_ADIABATIC = 0, TH_FIXED = 1 };
enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENONPHYS = -4 };

}  // namespace

extern "C" {
// Same field order as the product's public config struct, defined here on
// its own so the two sides share no header.
typedef struct orc_config {
  int32_t dim;
  int32_t n[3];
  double L[3];
  double gamma, g, mu, kappa, K, cfl;
  int32_t low_mach;
  int32_t dt_mode;
  int32_t bc[3][2];
  int32_t wall_noslip;
  int32_t thermal[2];
  double T_wall[2];
  int32_t energy_form;  // 0: total energy with the relaxed potential; 1: App. B
  int32_t pad_;
} orc_config;
}

namespace {

struct Grid {
  int D, zax;             // number of axes, gravity axis (the last one)
  int n[3], P[3];         // interior and padded extents (2 ghost layers)
  long ncell, npad;
  double dx[3], idx[3];
  double gm1;
  explicit Grid(const orc_config& c) {
    D = c.dim;
    zax = D - 1;
    ncell = 1;
    npad = 1;
    for (int a = 0; a < 3; ++a) {
      if (a < D) {
        n[a] = c.n[a];
        P[a] = c.n[a] + 4;
        dx[a] = c.L[a] / (double)c.n[a];
        idx[a] = 1.0 / dx[a];
      } else {
        n[a] = 1;
        P[a] = 1;
        dx[a] = 1.0;
        idx[a] = 0.0;
      }
      ncell *= n[a];
      npad *= P[a];
    }
    gm1 = c.gamma - 1.0;
  }
  long pad(int q0, int q1, int q2) const { return q0 + (long)P[0] * (q1 + (long)P[1] * q2); }
  long cell(int i, int j, int k) const { return i + (long)n[0] * (j + (long)n[1] * k); }
  // Gravitational potential at the centre of the cell with (signed) index kz
  // along the gravity axis: Phi = g * z, z = (kz + 1/2) dz.
  double phi(const orc_config& c, int kz) const { return c.g * (((double)kz + 0.5) * dx[zax]); }
};

template <class S>
struct Prim {
  S rho, r, u[3], p, c, rc, T;
};

// O2: conservative -> primitive for one cell.
template <class S>
Prim<S> cons_to_prim(const orc_config& c, const Grid& G, const S* U, long cell) {
  const long N = G.ncell;
  Prim<S> q;
  q.rho = U[cell];
  q.r = S(1.0) / q.rho;
  S m[3] = {S(0.0), S(0.0), S(0.0)};
  for (int k = 0; k < G.D; ++k) {
    m[k] = U[(1 + k) * N + cell];
    q.u[k] = m[k] * q.r;
  }
  for (int k = G.D; k < 3; ++k) q.u[k] = S(0.0);
  S E = U[(1 + G.D) * N + cell];
  S kin = m[0] * q.u[0];
  for (int k = 1; k < G.D; ++k) kin = kin + m[k] * q.u[k];
  kin = S(0.5) * kin;
  q.p = S(G.gm1) * (E - kin);
  q.T = q.p / q.rho;              // p = rho T (R = 1)
  q.c = sqrt_(S(c.gamma) * q.T);  // c^2 = gamma p / rho = gamma T
  q.rc = q.rho * q.c;
  return q;
}

// Resolution of a padded index along a non-gravity axis (periodic wrap or
// outflow clamp); returns the padded index of the interior cell it copies.
inline int resolve_axis(const orc_config& c, const Grid& G, int a, int q) {
  const int n = G.n[a];
  if (q >= 2 && q < n + 2) return q;
  const int side = (q < 2) ? 0 : 1;
  if (c.bc[a][side] == BC_PERIODIC) return ((q - 2 + 2 * n) % n) + 2;
  return side == 0 ? 2 : n + 1;  // outflow: copy the nearest interior cell
}

template <class S>
struct State {
  std::vector<Prim<S>> prim;   // padded
  std::vector<S> cons;         // padded, [var][pad]
  std::vector<double> phi;     // padded index along zax -> Phi
};

// O1 + O2 on the whole padded grid.
template <class S>
void build_padded(const orc_config& c, const Grid& G, const S* U, State<S>& st) {
  const int nv = G.D + 2;
  st.prim.assign(G.npad, Prim<S>());
  st.cons.assign((size_t)nv * G.npad, S(0.0));
  st.phi.assign(G.P[G.zax], 0.0);
  for (int q = 0; q < G.P[G.zax]; ++q) st.phi[q] = G.phi(c, q - 2);
  const int z = G.zax;
  for (int q2 = 0; q2 < G.P[2]; ++q2)
    for (int q1 = 0; q1 < G.P[1]; ++q1)
      for (int q0 = 0; q0 < G.P[0]; ++q0) {
        int q[3] = {q0, q1, q2};
        // transverse axes first
        int rq[3] = {q0, q1, q2};
        for (int a = 0; a < G.D; ++a)
          if (a != z) rq[a] = resolve_axis(c, G, a, q[a]);
        const long dst = G.pad(q0, q1, q2);
        const int qz = q[z];
        const int nz = G.n[z];
        bool ghost_z = (qz < 2 || qz >= nz + 2);
        int side = (qz < 2) ? 0 : 1;
        if (ghost_z && c.bc[z][side] != BC_WALL) {
          rq[z] = resolve_axis(c, G, z, qz);
          ghost_z = false;
        }
        if (!ghost_z) {
          long cell = G.cell(rq[0] - (G.D > 0 ? 2 : 0), G.D > 1 ? rq[1] - 2 : 0, G.D > 2 ? rq[2] - 2 : 0);
          st.prim[dst] = cons_to_prim(c, G, U, cell);
          for (int v = 0; v < nv; ++v) st.cons[v * G.npad + dst] = U[v * G.ncell + cell];
          continue;
        }
        // Wall ghost (both ghost layers take the values of the first one).
        int qi = (side == 0) ? 2 : nz + 1;          // adjacent interior cell
        int qg = (side == 0) ? 1 : nz + 2;          // first ghost layer
        rq[z] = qi;
        long cell = G.cell(rq[0] - 2, G.D > 1 ? rq[1] - 2 : 0, G.D > 2 ? rq[2] - 2 : 0);
        Prim<S> in = cons_to_prim(c, G, U, cell);
        double delta = st.phi[qg] - st.phi[qi];
        S Ti = in.T;
        S Tg = (c.thermal[side] == TH_FIXED) ? S(2.0 * c.T_wall[side]) - Ti : Ti;
        Prim<S> gq;
        gq.rho = (in.rho * (Ti - S(0.5 * delta))) / (Tg + S(0.5 * delta));
        gq.r = S(1.0) / gq.rho;
        gq.p = gq.rho * Tg;
        gq.T = Tg;
        for (int k = 0; k < 3; ++k) {
          bool flip = c.wall_noslip ? true : (k == z);
          gq.u[k] = (k < G.D && flip) ? -in.u[k] : in.u[k];
        }
        gq.c = sqrt_(S(c.gamma) * Tg);
        gq.rc = gq.rho * gq.c;
        st.prim[dst] = gq;
        // conserved values of wall ghosts are never used (zero wall flux)
      }
}

template <class S>
struct Face {
  S a, S_, ustar, theta, pistar, P;
};

// O4: acoustic solver at the face between L and R = L + e_d (Sec. 2.1.2):
//   a  = K max(rho_L c_L, rho_R c_R)            (sub-characteristic condition)
//   S  = -(rho_L + rho_R)/2 (Phi_R - Phi_L)     (interface gravity source)
//   u* = (u_L + u_R)/2 - (Pi_R - Pi_L - S) / (2a)
//   Ma = |u*| / max(c_L, c_R),  theta = min(Ma, 1)   (eq. low_mach_correction)
//   Pi* = (Pi_L + Pi_R)/2 - (a theta / 2)(u_R - u_L)
// with the quotients written as the paper writes them.
template <class S>
Face<S> acoustic_face(const orc_config& c, const Grid& G, const Prim<S>& L, const Prim<S>& R,
                      int d, double phiL, double phiR, bool wall) {
  Face<S> f;
  f.a = S(c.K) * smax(L.rc, R.rc);
  if (d == G.zax)
    f.S_ = (S(-0.5) * (L.rho + R.rho)) * S(phiR - phiL);
  else
    f.S_ = S(0.0);
  if (wall)
    f.ustar = S(0.0);
  else
    f.ustar = S(0.5) * (L.u[d] + R.u[d]) - ((R.p - L.p) - f.S_) / (S(2.0) * f.a);
  if (c.low_mach) {
    S Ma = sabs(f.ustar) / smax(L.c, R.c);
    f.theta = smin(Ma, S(1.0));
  } else {
    f.theta = S(1.0);
  }
  f.pistar = S(0.5) * (L.p + R.p) - ((S(0.5) * f.a) * f.theta) * (R.u[d] - L.u[d]);
  f.P = f.pistar * f.ustar;
  return f;
}

template <class S>
struct StepArrays {
  std::vector<Face<S>> face[3];
  std::vector<unsigned char> wall[3];
  std::vector<S> L;                 // padded
  std::vector<S> bt;                // padded, [var][pad]
  std::vector<S> Gf[3];             // per axis: [var][pad]
  std::vector<S> tau[3];            // per axis: [k][pad] (dissipative only)
};

inline bool is_wall_face(const orc_config& c, const Grid& G, int d, int q) {
  // face between padded q and q+1 along d
  if (d != G.zax) return false;
  const int n = G.n[d];
  if (q == 1 && c.bc[d][0] == BC_WALL) return true;
  if (q == n + 1 && c.bc[d][1] == BC_WALL) return true;
  return false;
}

template <class S>
void imex_override(const orc_config& c, const Grid& G, const State<S>& st, StepArrays<S>& A, double dt,
                   const double* x);

template <class S>
int step_impl(const orc_config& c, const S* U, S* Uout, double dt, S mu, S kappa,
              int64_t* fault_cell, const double* imex_x = nullptr) {
  Grid G(c);
  const int D = G.D, z = G.zax, nv = D + 2;
  const long NP = G.npad;
  const bool diss = (val(mu) > 0.0) || (val(kappa) > 0.0);
  const S eta = (S(-2.0) * mu) / S(3.0);
  double lam[3];
  for (int d = 0; d < 3; ++d) lam[d] = (d < D) ? dt / G.dx[d] : 0.0;
  long stride[3] = {1, (long)G.P[0], (long)G.P[0] * G.P[1]};

  State<S> st;
  build_padded(c, G, U, st);
  StepArrays<S> A;

  // O4: faces between padded q and q+1 for q in [0, P-1) along each axis.
  for (int d = 0; d < D; ++d) {
    A.face[d].assign(NP, Face<S>());
    A.wall[d].assign(NP, 0);
#pragma omp parallel for schedule(static)
    for (int q2 = 0; q2 < G.P[2]; ++q2)
      for (int q1 = 0; q1 < G.P[1]; ++q1)
        for (int q0 = 0; q0 < G.P[0]; ++q0) {
          int q[3] = {q0, q1, q2};
          if (q[d] + 1 >= G.P[d]) continue;
          long p = G.pad(q0, q1, q2);
          long pr = p + stride[d];
          double phiL = st.phi[q[z]], phiR = st.phi[q[z] + (d == z ? 1 : 0)];
          bool w = is_wall_face(c, G, d, q[d]);
          A.wall[d][p] = w;
          A.face[d][p] = acoustic_face(c, G, st.prim[p], st.prim[pr], d, phiL, phiR, w);
        }
  }

  // Implicit acoustic step: the interface values u*, Pi* (and Pi* u*) of
  // every face come from the solution x of the implicit system instead.
  if (imex_x) imex_override(c, G, st, A, dt, imex_x);

  // O5: acoustic cell values for padded cells [1, P-1) along every axis.
  A.L.assign(NP, S(1.0));
  A.bt.assign((size_t)nv * NP, S(0.0));
  std::vector<S> Sbar(NP, S(0.0));
  // App. B (non-conservative energy): no relaxation of the potential; the
  // energy's acoustic update carries the source (uS)_i = (u*_{i+1/2}
  // S_{i+1/2} + u*_{i-1/2} S_{i-1/2}) / 2 of the gravity axis.
  const bool nc = c.energy_form == 1;
  std::vector<S> uSbar(nc ? NP : 0, S(0.0));
#pragma omp parallel for schedule(static)
  for (int q2 = (D > 2 ? 1 : 0); q2 < (D > 2 ? G.P[2] - 1 : 1); ++q2)
    for (int q1 = (D > 1 ? 1 : 0); q1 < (D > 1 ? G.P[1] - 1 : 1); ++q1)
      for (int q0 = 1; q0 < G.P[0] - 1; ++q0) {
        int q[3] = {q0, q1, q2};
        long p = G.pad(q0, q1, q2);
        S Lc = S(1.0);
        for (int d = 0; d < D; ++d)
          Lc = Lc + S(lam[d]) * (A.face[d][p].ustar - A.face[d][p - stride[d]].ustar);
        S sb = S(0.5) * (A.face[z][p].S_ + A.face[z][p - stride[z]].S_);
        Sbar[p] = sb;
        S Am[3];
        for (int k = 0; k < D; ++k) {
          S dpi = A.face[k][p].pistar - A.face[k][p - stride[k]].pistar;
          if (k == z) dpi = dpi - sb;
          Am[k] = S(lam[k]) * dpi;
        }
        S AE = S(lam[0]) * (A.face[0][p].P - A.face[0][p - stride[0]].P);
        for (int d = 1; d < D; ++d) AE = AE + S(lam[d]) * (A.face[d][p].P - A.face[d][p - stride[d]].P);
        S rho = st.cons[0 * NP + p];
        S calE;
        if (nc) {
          const Face<S>& fu = A.face[z][p];
          const Face<S>& fd = A.face[z][p - stride[z]];
          S uS = S(0.5) * (fu.ustar * fu.S_ + fd.ustar * fd.S_);
          uSbar[p] = uS;
          AE = AE - S(lam[z]) * uS;
          calE = st.cons[(1 + D) * NP + p];
        } else {
          calE = st.cons[(1 + D) * NP + p] + rho * S(st.phi[q[z]]);
        }
        // L~ b~ = b - A^b  (the acoustic update of Sec. 2.1.2)
        A.L[p] = Lc;
        A.bt[0 * NP + p] = rho / Lc;
        for (int k = 0; k < D; ++k) A.bt[(1 + k) * NP + p] = (st.cons[(1 + k) * NP + p] - Am[k]) / Lc;
        A.bt[(1 + D) * NP + p] = (calE - AE) / Lc;
      }

  // O6 + O7: total face flux G for faces between padded q and q+1,
  // q in [1, P-2) along d (every face of every interior cell).
  for (int d = 0; d < D; ++d) {
    A.Gf[d].assign((size_t)nv * NP, S(0.0));
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (a >= D) { lo[a] = 0; hi[a] = 1; }
      else if (a == d) { lo[a] = 1; hi[a] = G.P[a] - 2; }   // faces q|q+1, q in [1, n+2)
      else { lo[a] = 2; hi[a] = G.P[a] - 2; }               // interior rows only
    }
#pragma omp parallel for schedule(static)
    for (int q2 = lo[2]; q2 < hi[2]; ++q2)
      for (int q1 = lo[1]; q1 < hi[1]; ++q1)
        for (int q0 = lo[0]; q0 < hi[0]; ++q0) {
          long p = G.pad(q0, q1, q2);
          long pr = p + stride[d];
          const Face<S>& f = A.face[d][p];
          S tr[5];
          if (A.wall[d][p]) {
            for (int v = 0; v < nv; ++v) tr[v] = S(0.0);
          } else {
            long up = (val(f.ustar) >= 0.0) ? p : pr;
            tr[0] = A.bt[0 * NP + up] * f.ustar;
            for (int k = 0; k < D; ++k) tr[1 + k] = A.bt[(1 + k) * NP + up] * f.ustar;
            tr[1 + D] = (A.bt[(1 + D) * NP + up] + f.pistar) * f.ustar;
          }
          S Gv[5];
          Gv[0] = tr[0];
          for (int k = 0; k < D; ++k) Gv[1 + k] = (k == d) ? tr[1 + k] + f.pistar : tr[1 + k];
          Gv[1 + D] = tr[1 + D];
          if (diss) {
            const Prim<S>& PL = st.prim[p];
            const Prim<S>& PR = st.prim[pr];
            S grad[3][3];  // grad[a][k] = d u_k / d x_a at the face
            for (int k = 0; k < D; ++k) grad[d][k] = (PR.u[k] - PL.u[k]) * S(G.idx[d]);
            for (int a = 0; a < D; ++a) {
              if (a == d) continue;
              const Prim<S>& Lp = st.prim[p + stride[a]];
              const Prim<S>& Lm = st.prim[p - stride[a]];
              const Prim<S>& Rp = st.prim[pr + stride[a]];
              const Prim<S>& Rm = st.prim[pr - stride[a]];
              for (int k = 0; k < D; ++k)
                grad[a][k] = ((Lp.u[k] - Lm.u[k]) + (Rp.u[k] - Rm.u[k])) * S(0.25 * G.idx[a]);
            }
            S div = grad[0][0];
            for (int a = 1; a < D; ++a) div = div + grad[a][a];
            S W = S(0.0);
            for (int k = 0; k < D; ++k) {
              S t = mu * (grad[d][k] + grad[k][d]);
              if (k == d) t = t + eta * div;
              S uf = S(0.5) * (PL.u[k] + PR.u[k]);
              W = (k == 0) ? t * uf : W + t * uf;
              Gv[1 + k] = Gv[1 + k] - t;
            }
            S Q = -(kappa * ((PR.T - PL.T) * S(G.idx[d])));
            Gv[1 + D] = (Gv[1 + D] - W) + Q;
          }
          for (int v = 0; v < nv; ++v) A.Gf[d][v * NP + p] = Gv[v];
        }
  }

  // O8 + O9: update interior cells.
  long first_bad = std::numeric_limits<long>::max();
  const double gm1 = G.gm1;
#pragma omp parallel for schedule(static) reduction(min : first_bad)
  for (int k = 0; k < G.n[2]; ++k)
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        int q[3] = {i + 2, D > 1 ? j + 2 : 0, D > 2 ? k + 2 : 0};
        long p = G.pad(q[0], q[1], q[2]);
        long cell = G.cell(i, j, k);
        S phic = S(st.phi[q[z]]);
        S rho = st.cons[0 * NP + p];
        S nr = rho;
        for (int d = 0; d < D; ++d) nr = nr - S(lam[d]) * (A.Gf[d][0 * NP + p] - A.Gf[d][0 * NP + p - stride[d]]);
        S nm[3];
        for (int kk = 0; kk < D; ++kk) {
          S v = st.cons[(1 + kk) * NP + p];
          for (int d = 0; d < D; ++d)
            v = v - S(lam[d]) * (A.Gf[d][(1 + kk) * NP + p] - A.Gf[d][(1 + kk) * NP + p - stride[d]]);
          if (kk == z) v = v + S(lam[z]) * Sbar[p];
          nm[kk] = v;
        }
        S calE = nc ? st.cons[(1 + D) * NP + p] : st.cons[(1 + D) * NP + p] + rho * phic;
        for (int d = 0; d < D; ++d)
          calE = calE - S(lam[d]) * (A.Gf[d][(1 + D) * NP + p] - A.Gf[d][(1 + D) * NP + p - stride[d]]);
        S nE;
        if (nc) {
          nE = calE + S(lam[z]) * uSbar[p];
        } else {
          nE = calE - nr * phic;
        }
        Uout[0 * G.ncell + cell] = nr;
        for (int kk = 0; kk < D; ++kk) Uout[(1 + kk) * G.ncell + cell] = nm[kk];
        Uout[(1 + D) * G.ncell + cell] = nE;
        // O9
        double vr = val(nr);
        double ir = 1.0 / vr;
        double kin = 0.0;
        for (int kk = 0; kk < D; ++kk) {
          double uk = val(nm[kk]) * ir;
          kin = (kk == 0) ? val(nm[kk]) * uk : kin + val(nm[kk]) * uk;
        }
        kin = 0.5 * kin;
        double np_ = gm1 * (val(nE) - kin);
        bool ok = (val(A.L[p]) > 0.0) && (vr > 0.0) && (np_ > 0.0) && std::isfinite(vr) &&
                  std::isfinite(np_) && std::isfinite(kin);
        if (!ok && cell < first_bad) first_bad = cell;
      }
  if (first_bad != std::numeric_limits<long>::max()) {
    if (fault_cell) *fault_cell = first_bad;
    return ORC_ENONPHYS;
  }
  return ORC_OK;
}


// ---------------------------------------------------------------- IMEX --
// Implicit acoustic step.  The paper names it as further work (Conclusion:
// solve the acoustic part implicitly to lift the acoustic CFL condition and
// keep the well-balanced gravity source) and prints no scheme; this is the
// reading taken here.  Sec. 2.1.2's acoustic step is solved with its
// interface values at the END of the step (backward Euler on the linear
// relaxation system at frozen a), everything else as in the explicit step.
// Unknowns per interior cell i: Pi_i and the normal velocities u_{d,i},
// x = [Pi | u_0 | ... | u_{D-1}], each block in interior cell order.  Frozen
// at t^n from O1-O4: a_j, S_j, theta_j of every face, rho_i, tau_i = 1/rho_i,
// p_i, c_i, and the hydrostatic offset p_g - p_i of every wall ghost.  With
// lambda_d = dt / dx_d:
//   u*_j  = (u_L + u_R)/2 - (Pi_R - Pi_L - S_j) / (2 a_j)       (0 at walls)
//   Pi*_j = (Pi_L + Pi_R)/2 - (a_j theta_j / 2)(u^n_R - u^n_L)
//   u_{d,i} = u^n_{d,i} - lambda_d tau_i ([Pi*]_{d,i} - S-bar_{d,i})
//   Pi_i    = p_i - rho_i c_i^2 sum_d lambda_d [u*]_{d,i}
// The acoustic dissipation of Pi* acts on the velocities of t^n (it is a
// diffusion of u with coefficient a theta / 2: with the low-Mach correction
// theta ~ |u*| / c its stability limit is a transport one, without it an
// acoustic one), so the velocity rows have the identity in u and u can be
// eliminated: the system for Pi alone is symmetric after scaling its rows
// by 1 / (rho c^2) (with periodic and wall boundaries).
// The last line is the Lagrangian pressure update linearised through the
// equation of state (dp = -rho c^2 dtau / tau, c^2 = gamma p / rho), the
// implicit counterpart of the relaxation Pi~ = p_EOS of Sec. 2.1.2.
// Parity unpinned for that coefficient: any positive one gives a
// consistent, well-balanced and stable step, so no property of the paper
// or of the mathematics tells rho c^2 apart (the rest of the system is
// pinned: tests/test_oracle_imex.py).  Ghost
// cells take the boundary rules of O1 applied to the unknowns: periodic
// images, outflow copies, and at walls Pi_g = Pi_i + (p_g - p_i)^n with the
// velocity of O1 (normal component reversed).  The implicit (u*, Pi*)
// replace the explicit ones in O5-O8.

// Padded extension of x (with_const: the wall ghosts' hydrostatic offset).
void imex_extend(const orc_config& c, const Grid& G, const State<double>& st, const double* x, bool with_const,
                 std::vector<double>& Pp, std::vector<double> up[3]) {
  const int D = G.D, z = G.zax;
  const long N = G.ncell;
  Pp.assign(G.npad, 0.0);
  for (int d = 0; d < D; ++d) up[d].assign(G.npad, 0.0);
  for (int q2 = 0; q2 < G.P[2]; ++q2)
    for (int q1 = 0; q1 < G.P[1]; ++q1)
      for (int q0 = 0; q0 < G.P[0]; ++q0) {
        int q[3] = {q0, q1, q2};
        int rq[3] = {q0, q1, q2};
        for (int a = 0; a < D; ++a)
          if (a != z) rq[a] = resolve_axis(c, G, a, q[a]);
        const long dst = G.pad(q0, q1, q2);
        const int qz = q[z], nz = G.n[z];
        bool wall_ghost = false;
        int side = (qz < 2) ? 0 : 1;
        if (qz < 2 || qz >= nz + 2) {
          if (c.bc[z][side] == BC_WALL) {
            wall_ghost = true;
            rq[z] = (side == 0) ? 2 : nz + 1;
          } else {
            rq[z] = resolve_axis(c, G, z, qz);
          }
        }
        const long cell = G.cell(rq[0] - 2, D > 1 ? rq[1] - 2 : 0, D > 2 ? rq[2] - 2 : 0);
        double Pi = x[cell];
        if (wall_ghost && with_const) {
          const long pi_ = G.pad(rq[0], rq[1], rq[2]);
          Pi = Pi + (st.prim[dst].p - st.prim[pi_].p);
        }
        Pp[dst] = Pi;
        for (int d = 0; d < D; ++d) {
          double u = x[(1 + d) * N + cell];
          if (wall_ghost && (c.wall_noslip || d == z)) u = -u;
          up[d][dst] = u;
        }
      }
}

// Implicit interface values of every padded face from the extension.
void imex_faces(const orc_config& c, const Grid& G, const State<double>& st, const StepArrays<double>& A,
                const std::vector<double>& Pp, const std::vector<double> up[3], bool with_const,
                std::vector<double> us[3], std::vector<double> pis[3]) {
  const int D = G.D;
  long stride[3] = {1, (long)G.P[0], (long)G.P[0] * G.P[1]};
  for (int d = 0; d < D; ++d) {
    us[d].assign(G.npad, 0.0);
    pis[d].assign(G.npad, 0.0);
    for (int q2 = 0; q2 < G.P[2]; ++q2)
      for (int q1 = 0; q1 < G.P[1]; ++q1)
        for (int q0 = 0; q0 < G.P[0]; ++q0) {
          int q[3] = {q0, q1, q2};
          if (q[d] + 1 >= G.P[d]) continue;
          const long p = G.pad(q0, q1, q2), pr = p + stride[d];
          const Face<double>& f = A.face[d][p];
          const double uL = up[d][p], uR = up[d][pr], PL = Pp[p], PR = Pp[pr];
          const double Sj = with_const ? f.S_ : 0.0;
          us[d][p] = A.wall[d][p] ? 0.0 : 0.5 * (uL + uR) - ((PR - PL) - Sj) / (2.0 * f.a);
          // the acoustic dissipation of Pi* acts on the velocities of t^n
          const double dun = st.prim[pr].u[d] - st.prim[p].u[d];
          pis[d][p] = 0.5 * (PL + PR) - (with_const ? ((0.5 * f.a) * f.theta) * dun : 0.0);
        }
  }
}

// Frozen data of the implicit system at t^n (O1, O2, O4).
struct ImexFrozen {
  Grid G;
  State<double> st;
  StepArrays<double> A;
  explicit ImexFrozen(const orc_config& c, const double* U) : G(c) {
    build_padded(c, G, U, st);
    long stride[3] = {1, (long)G.P[0], (long)G.P[0] * G.P[1]};
    for (int d = 0; d < G.D; ++d) {
      A.face[d].assign(G.npad, Face<double>());
      A.wall[d].assign(G.npad, 0);
      for (int q2 = 0; q2 < G.P[2]; ++q2)
        for (int q1 = 0; q1 < G.P[1]; ++q1)
          for (int q0 = 0; q0 < G.P[0]; ++q0) {
            int q[3] = {q0, q1, q2};
            if (q[d] + 1 >= G.P[d]) continue;
            long p = G.pad(q0, q1, q2);
            double phiL = st.phi[q[G.zax]], phiR = st.phi[q[G.zax] + (d == G.zax ? 1 : 0)];
            bool w = is_wall_face(c, G, d, q[d]);
            A.wall[d][p] = w;
            A.face[d][p] = acoustic_face(c, G, st.prim[p], st.prim[p + stride[d]], d, phiL, phiR, w);
          }
    }
  }
};

// Residual F(x) of the implicit system (with_const = false: its linear
// part), one row per unknown in the order of x.
void imex_residual(const orc_config& c, const ImexFrozen& F, double dt, const double* x, bool with_const,
                   double* r) {
  const Grid& G = F.G;
  const int D = G.D, z = G.zax;
  const long N = G.ncell;
  long stride[3] = {1, (long)G.P[0], (long)G.P[0] * G.P[1]};
  std::vector<double> Pp, up[3], us[3], pis[3];
  imex_extend(c, G, F.st, x, with_const, Pp, up);
  imex_faces(c, G, F.st, F.A, Pp, up, with_const, us, pis);
  for (int k = 0; k < G.n[2]; ++k)
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        const long cell = G.cell(i, j, k);
        const long p = G.pad(i + 2, D > 1 ? j + 2 : 0, D > 2 ? k + 2 : 0);
        const Prim<double>& q = F.st.prim[p];
        double div = 0.0;
        for (int d = 0; d < D; ++d) div = div + (dt / G.dx[d]) * (us[d][p] - us[d][p - stride[d]]);
        const double rc2 = q.rho * (q.c * q.c);
        r[cell] = (x[cell] - (with_const ? q.p : 0.0)) + rc2 * div;
        for (int d = 0; d < D; ++d) {
          double dpi = pis[d][p] - pis[d][p - stride[d]];
          if (d == z && with_const) dpi = dpi - 0.5 * (F.A.face[d][p].S_ + F.A.face[d][p - stride[d]].S_);
          const double un = with_const ? q.u[d] : 0.0;
          r[(1 + d) * N + cell] = (x[(1 + d) * N + cell] - un) + ((dt / G.dx[d]) * q.r) * dpi;
        }
      }
}

template <class S>
void imex_override(const orc_config& c, const Grid& G, const State<S>& st, StepArrays<S>& A, double dt,
                   const double* x) {
  if constexpr (std::is_same<S, double>::value) {
    std::vector<double> Pp, up[3], us[3], pis[3];
    imex_extend(c, G, st, x, true, Pp, up);
    imex_faces(c, G, st, A, Pp, up, true, us, pis);
    for (int d = 0; d < G.D; ++d)
      for (long p = 0; p < G.npad; ++p) {
        A.face[d][p].ustar = us[d][p];
        A.face[d][p].pistar = pis[d][p];
        A.face[d][p].P = pis[d][p] * us[d][p];
      }
  }
  (void)dt;
}

// O3: the largest local rate lambda_i over interior cells.
double max_rate(const orc_config& c, const double* U) {
  Grid G(c);
  const int D = G.D;
  double sumidx2 = 0.0;
  for (int d = 0; d < D; ++d) sumidx2 = (d == 0) ? G.idx[d] * G.idx[d] : sumidx2 + G.idx[d] * G.idx[d];
  const double dmax = std::max((4.0 * c.mu) / 3.0, c.kappa * G.gm1);
  double m = 0.0;
#pragma omp parallel for schedule(static) reduction(max : m)
  for (long cell = 0; cell < G.ncell; ++cell) {
    Prim<double> q = cons_to_prim(c, G, U, cell);
    // dt_mode 2 (IMEX step): the sound speed leaves the rate
    const double cs = (c.dt_mode == 2) ? 0.0 : q.c;
    double h = (std::fabs(q.u[0]) + cs) * G.idx[0];
    for (int d = 1; d < D; ++d) h = h + (std::fabs(q.u[d]) + cs) * G.idx[d];
    double l = h;
    if (c.dt_mode != 1) l = h + (2.0 * (dmax * q.r)) * sumidx2;
    if (!(l < std::numeric_limits<double>::infinity())) l = std::numeric_limits<double>::infinity();
    if (l > m) m = l;
  }
  return m;
}

inline uint64_t splitmix64_next(uint64_t& state) {
  // SplitMix64 (Steele, Lea and Flood, OOPSLA 2014; constants as published
  // in Vigna's reference implementation).
  state += 0x9E3779B97F4A7C15ULL;
  uint64_t zz = state;
  zz = (zz ^ (zz >> 30)) * 0xBF58476D1CE4E5B9ULL;
  zz = (zz ^ (zz >> 27)) * 0x94D049BB133111EBULL;
  return zz ^ (zz >> 31);
}

}  // namespace

// ================================================================ C API ====
extern "C" {

int orc_nvar(const orc_config* c) { return c->dim + 2; }

int orc_validate(const orc_config* c) {
  if (!c) return ORC_EINVAL;
  if (c->dim < 1 || c->dim > 3) return ORC_EINVAL;
  for (int a = 0; a < c->dim; ++a) {
    if (c->n[a] < 1 || !(c->L[a] > 0.0)) return ORC_EINVAL;
    for (int s = 0; s < 2; ++s) {
      int b = c->bc[a][s];
      if (b != BC_PERIODIC && b != BC_WALL && b != BC_OUTFLOW) return ORC_EINVAL;
      if (b == BC_WALL && a != c->dim - 1) return ORC_EINVAL;
    }
    if ((c->bc[a][0] == BC_PERIODIC) != (c->bc[a][1] == BC_PERIODIC)) return ORC_EINVAL;
  }
  const int z = c->dim - 1;
  if (c->g != 0.0 && (c->bc[z][0] != BC_WALL || c->bc[z][1] != BC_WALL)) return ORC_EINVAL;
  if (!(c->gamma > 1.0) || !(c->mu >= 0.0) || !(c->kappa >= 0.0) || !(c->K >= 1.0) || !(c->cfl > 0.0))
    return ORC_EINVAL;
  if (c->dt_mode != 0 && c->dt_mode != 1 && c->dt_mode != 2) return ORC_EINVAL;
  if (c->energy_form != 0 && c->energy_form != 1) return ORC_EINVAL;
  return ORC_OK;
}

double orc_max_rate(const orc_config* c, const double* U) { return max_rate(*c, U); }

double orc_dt(const orc_config* c, const double* U) { return c->cfl / max_rate(*c, U); }

// One step with a given dt; U is read, Uout written (may not alias).
int orc_step_dt(const orc_config* c, const double* U, double* Uout, double dt, int64_t* fault_cell) {
  return step_impl<double>(*c, U, Uout, dt, c->mu, c->kappa, fault_cell);
}

// n steps in place; dt of each step from O3 on its own input state unless
// dt_sched is given.  dt_log (optional) receives the dt used by each step;
// *t is advanced.  Returns the first failing status.
// Implicit acoustic step: the sparse matrix of the linear part of the
// system (probed column by column: exact coefficients) and its right-hand
// side -F(0); solve L x = rhs, then orc_step_imex_x.  cap: room for cap
// nonzeros; EINVAL if too small (*nnz then holds the count needed) or for
// the App. B energy form.
int orc_imex_system(const orc_config* c, const double* U, double dt, int64_t cap, int64_t* rows, int64_t* cols,
                    double* vals, double* rhs, int64_t* nnz) {
  if (orc_validate(c) != ORC_OK || c->energy_form != 0) return ORC_EINVAL;
  ImexFrozen F(*c, U);
  const long N = F.G.ncell;
  const long n = (long)(F.G.D + 1) * N;
  std::vector<double> e(n, 0.0), col(n);
  imex_residual(*c, F, dt, e.data(), true, rhs);
  for (long i = 0; i < n; ++i) rhs[i] = -rhs[i];
  int64_t k = 0;
  for (long j = 0; j < n; ++j) {
    e[j] = 1.0;
    imex_residual(*c, F, dt, e.data(), false, col.data());
    e[j] = 0.0;
    for (long i = 0; i < n; ++i)
      if (col[i] != 0.0) {
        if (k < cap) {
          rows[k] = i;
          cols[k] = j;
          vals[k] = col[i];
        }
        ++k;
      }
  }
  *nnz = k;
  return k <= cap ? ORC_OK : ORC_EINVAL;
}

// F(x) of the implicit system (test of a solution).
int orc_imex_residual(const orc_config* c, const double* U, double dt, const double* x, double* r) {
  if (orc_validate(c) != ORC_OK || c->energy_form != 0) return ORC_EINVAL;
  ImexFrozen F(*c, U);
  imex_residual(*c, F, dt, x, true, r);
  return ORC_OK;
}

// One step with the interface values of the solution x of the implicit
// system.
int orc_step_imex_x(const orc_config* c, const double* U, const double* x, double dt, double* Uout,
                    int64_t* fault_cell) {
  if (orc_validate(c) != ORC_OK || c->energy_form != 0) return ORC_EINVAL;
  return step_impl<double>(*c, U, Uout, dt, c->mu, c->kappa, fault_cell, x);
}
int orc_run(const orc_config* c, double* U, int nsteps, const double* dt_sched, double* dt_log, double* t,
            int64_t* fault_cell, int64_t* fault_step) {
  Grid G(*c);
  const size_t len = (size_t)(G.D + 2) * G.ncell;
  std::vector<double> tmp(len);
  for (int s = 0; s < nsteps; ++s) {
    double dt = dt_sched ? dt_sched[s] : (c->cfl / max_rate(*c, U));
    int rc = step_impl<double>(*c, U, tmp.data(), dt, c->mu, c->kappa, fault_cell);
    std::memcpy(U, tmp.data(), len * sizeof(double));
    if (dt_log) dt_log[s] = dt;
    if (t) *t += dt;
    if (rc != ORC_OK) {
      if (fault_step) *fault_step = s;
      return rc;
    }
  }
  return ORC_OK;
}

// Tangent-linear model of one step at fixed dt: given (U, dU, dmu, dkappa),
// returns Uout and dUout = J_U dU + J_mu dmu + J_kappa dkappa.
int orc_tlm(const orc_config* c, const double* U, const double* dU, double dmu, double dkappa, double dt,
            double* Uout, double* dUout) {
  Grid G(*c);
  const size_t len = (size_t)(G.D + 2) * G.ncell;
  std::vector<Dual> X(len), Y(len);
  for (size_t i = 0; i < len; ++i) X[i] = Dual(U[i], dU ? dU[i] : 0.0);
  int64_t fc = -1;
  int rc = step_impl<Dual>(*c, X.data(), Y.data(), dt, Dual(c->mu, dmu), Dual(c->kappa, dkappa), &fc);
  for (size_t i = 0; i < len; ++i) {
    if (Uout) Uout[i] = Y[i].v;
    dUout[i] = Y[i].d;
  }
  return rc;
}

// Reverse product of one step at fixed dt, by brute force: column j of the
// Jacobian is one tangent-linear pass seeded with e_j, so
//   lam_out[j] = < lam_in, J e_j >,  g_mu += < lam_in, J_mu >, g_kappa likewise.
// Slow (one full step per unknown); meant for small grids.
int orc_adjoint_dense(const orc_config* c, const double* U, const double* lam_in, double dt, double* lam_out,
                      double* g_mu, double* g_kappa) {
  Grid G(*c);
  const size_t len = (size_t)(G.D + 2) * G.ncell;
  std::vector<double> e(len, 0.0), col(len);
  int rc = ORC_OK;
  for (size_t j = 0; j < len; ++j) {
    e[j] = 1.0;
    rc = orc_tlm(c, U, e.data(), 0.0, 0.0, dt, nullptr, col.data());
    e[j] = 0.0;
    double s = 0.0;
    for (size_t i = 0; i < len; ++i) s += lam_in[i] * col[i];
    lam_out[j] = s;
  }
  for (int which = 0; which < 2; ++which) {
    orc_tlm(c, U, nullptr, which == 0 ? 1.0 : 0.0, which == 1 ? 1.0 : 0.0, dt, nullptr, col.data());
    double s = 0.0;
    for (size_t i = 0; i < len; ++i) s += lam_in[i] * col[i];
    if (which == 0 && g_mu) *g_mu += s;
    if (which == 1 && g_kappa) *g_kappa += s;
  }
  return rc;
}

// Initial states.  params meaning per problem (see oracle/__init__.py).
//  0 uniform    : rho, u0, u1, u2, p
//  1 RB linear-T: T_bottom, T_top, rho_bottom_cell (<=0: T of the bottom cell), amp
//  2 Gresho     : Ma
//  3 Sod        : (none)
//  4 isothermal : (none)  p = rho, T = 1, rho_0 = exp(-g z_0)
int orc_init(const orc_config* c, int problem, const double* prm, int nprm, uint64_t seed, double* U) {
  if (orc_validate(c) != ORC_OK) return ORC_EINVAL;
  Grid G(*c);
  const int D = G.D, z = G.zax;
  const long N = G.ncell;
  const double gm1 = G.gm1;
  auto P = [&](int i, double dflt) { return (i < nprm) ? prm[i] : dflt; };
  for (long i = 0; i < (long)(D + 2) * N; ++i) U[i] = 0.0;
  if (problem == 0) {
    double rho = P(0, 1.0), u[3] = {P(1, 0.0), P(2, 0.0), P(3, 0.0)}, p = P(4, 1.0);
    for (long cell = 0; cell < N; ++cell) {
      U[cell] = rho;
      double kin = 0.0;
      for (int k = 0; k < D; ++k) {
        U[(1 + k) * N + cell] = rho * u[k];
        kin = kin + u[k] * u[k];
      }
      U[(1 + D) * N + cell] = p / gm1 + 0.5 * rho * kin;
    }
    return ORC_OK;
  }
  if (problem == 1 || problem == 4) {
    const int nz = G.n[z];
    const double Lz = c->L[z];
    std::vector<double> T(nz), rho(nz);
    const bool iso = (problem == 4);
    const double Tb = iso ? 1.0 : P(0, 1.0), Tt = iso ? 1.0 : P(1, 0.5);
    for (int k = 0; k < nz; ++k) {
      double zk = ((double)k + 0.5) * G.dx[z];
      T[k] = Tb + (Tt - Tb) * (zk / Lz);
    }
    double r0 = iso ? std::exp(-(c->g * ((0.5) * G.dx[z]))) : P(2, -1.0);
    if (!(r0 > 0.0)) r0 = T[0];
    rho[0] = r0;
    for (int k = 0; k + 1 < nz; ++k) {
      double delta = G.phi(*c, k + 1) - G.phi(*c, k);
      rho[k + 1] = (rho[k] * (T[k] - 0.5 * delta)) / (T[k + 1] + 0.5 * delta);
    }
    const double amp = iso ? 0.0 : P(3, 0.0);
    uint64_t state = seed;
    for (long cell = 0; cell < N; ++cell) {
      long kz = (z == 0) ? cell % G.n[0] : (z == 1 ? (cell / G.n[0]) % G.n[1] : cell / ((long)G.n[0] * G.n[1]));
      double u01 = (double)(splitmix64_next(state) >> 11) * 0x1.0p-53;
      double dT = amp * (2.0 * u01 - 1.0);
      double p = rho[kz] * (T[kz] + dT);
      U[cell] = rho[kz];
      U[(1 + D) * N + cell] = p / gm1;
    }
    return ORC_OK;
  }
  if (problem == 2) {
    if (D != 2) return ORC_EINVAL;
    const double Ma = P(0, 1e-3);
    const double p0 = 1.0 / (c->gamma * Ma * Ma);
    const double xc = 0.5 * c->L[0], yc = 0.5 * c->L[1];
    for (int j = 0; j < G.n[1]; ++j)
      for (int i = 0; i < G.n[0]; ++i) {
        long cell = G.cell(i, j, 0);
        double x = ((double)i + 0.5) * G.dx[0] - xc;
        double y = ((double)j + 0.5) * G.dx[1] - yc;
        double r = std::sqrt(x * x + y * y);
        double ut, p;
        if (r < 0.2) {
          ut = 5.0 * r;
          p = p0 + 12.5 * r * r;
        } else if (r < 0.4) {
          ut = 2.0 - 5.0 * r;
          p = p0 + 12.5 * r * r + 4.0 - 20.0 * r + 4.0 * std::log(5.0 * r);
        } else {
          ut = 0.0;
          p = p0 - 2.0 + 4.0 * std::log(2.0);
        }
        // u_theta vanishes at the centre (u_theta = 5 r), so the Cartesian
        // components -u_theta y / r, u_theta x / r have the limit 0 there
        double ux = r > 0.0 ? -(ut * y) / r : 0.0, uy = r > 0.0 ? (ut * x) / r : 0.0;
        const double rho = 1.0;
        U[cell] = rho;
        U[N + cell] = rho * ux;
        U[2 * N + cell] = rho * uy;
        U[3 * N + cell] = p / gm1 + 0.5 * rho * (ux * ux + uy * uy);
      }
    return ORC_OK;
  }
  if (problem == 3) {
    for (long cell = 0; cell < N; ++cell) {
      long i = cell % G.n[0];
      double x = ((double)i + 0.5) * G.dx[0];
      bool left = x < 0.5 * c->L[0];
      double rho = left ? 1.0 : 0.125, p = left ? 1.0 : 0.1;
      U[cell] = rho;
      U[(1 + D) * N + cell] = p / gm1;
    }
    return ORC_OK;
  }
  return ORC_EINVAL;
}

// Unit access to the face solver (O4) for pins on a single interface.
// prim arrays: [rho, u_d, p]; c and rho c follow from the ideal gas.
void orc_face(const orc_config* c, int d, double rhoL, double uL, double pL, double rhoR, double uR,
              double pR, double phiL, double phiR, int wall, double* out /*a,S,ustar,theta,pistar,P*/) {
  Grid G(*c);
  Prim<double> L{}, R{};
  L.rho = rhoL; L.r = 1.0 / rhoL; L.u[d] = uL; L.p = pL;
  L.T = pL / rhoL; L.c = std::sqrt(c->gamma * L.T); L.rc = rhoL * L.c;
  R.rho = rhoR; R.r = 1.0 / rhoR; R.u[d] = uR; R.p = pR;
  R.T = pR / rhoR; R.c = std::sqrt(c->gamma * R.T); R.rc = rhoR * R.c;
  Face<double> f = acoustic_face(*c, G, L, R, d, phiL, phiR, wall != 0);
  out[0] = f.a; out[1] = f.S_; out[2] = f.ustar; out[3] = f.theta; out[4] = f.pistar; out[5] = f.P;
}

// Diagnostics of a state: out[0..] =
//  mass, mom0, mom1, mom2, e_total (sum of E + rho Phi), e_kin, e_int, e_grav,
//  max |u|, mean |u|, max Mach, Nu_bottom, Nu_top   (all volume-weighted sums)
void orc_diag(const orc_config* c, const double* U, double* out) {
  Grid G(*c);
  const int D = G.D, z = G.zax;
  const long N = G.ncell;
  double dV = 1.0;
  for (int d = 0; d < D; ++d) dV *= G.dx[d];
  double s[13] = {0};
  for (long cell = 0; cell < N; ++cell) {
    Prim<double> q = cons_to_prim(*c, G, U, cell);
    long kz = (z == 0) ? cell % G.n[0] : (z == 1 ? (cell / G.n[0]) % G.n[1] : cell / ((long)G.n[0] * G.n[1]));
    double phi = G.phi(*c, (int)kz);
    double rho = U[cell];
    double E = U[(1 + D) * N + cell];
    double kin = 0.0, uu = 0.0;
    for (int k = 0; k < D; ++k) {
      double m = U[(1 + k) * N + cell];
      s[1 + k] += m * dV;
      kin += 0.5 * m * q.u[k];
      uu += q.u[k] * q.u[k];
    }
    double um = std::sqrt(uu);
    s[0] += rho * dV;
    s[4] += (E + rho * phi) * dV;
    s[5] += kin * dV;
    s[6] += (E - kin) * dV;
    s[7] += rho * phi * dV;
    s[8] = std::max(s[8], um);
    s[9] += um;
    s[10] = std::max(s[10], um / q.c);
  }
  s[9] /= (double)N;
  // Nusselt numbers on fixed-temperature walls: horizontal mean of the wall
  // conductive flux over the conductive-profile flux dT/depth.
  if (c->bc[z][0] == BC_WALL && c->bc[z][1] == BC_WALL) {
    const double dT = c->T_wall[0] - c->T_wall[1];
    const double depth = c->L[z];
    long ncol = N / G.n[z];
    double nb = 0.0, nt = 0.0;
    for (long col = 0; col < ncol; ++col) {
      long i0, i1;
      if (z == 0) { i0 = 0; i1 = 0; }
      else if (z == 1) { i0 = col; i1 = 0; }
      else { i0 = col % G.n[0]; i1 = col / G.n[0]; }
      long cb = (z == 0) ? 0 : (z == 1 ? G.cell((int)i0, 0, 0) : G.cell((int)i0, (int)i1, 0));
      long ct = (z == 0) ? G.n[0] - 1
                         : (z == 1 ? G.cell((int)i0, G.n[1] - 1, 0) : G.cell((int)i0, (int)i1, G.n[2] - 1));
      double Tb = cons_to_prim(*c, G, U, cb).T, Tt = cons_to_prim(*c, G, U, ct).T;
      nb += 2.0 * (c->T_wall[0] - Tb) / G.dx[z];
      nt += 2.0 * (Tt - c->T_wall[1]) / G.dx[z];
    }
    if (dT != 0.0) {
      s[11] = (nb / (double)ncol) * depth / dT;
      s[12] = (nt / (double)ncol) * depth / dT;
    }
  }
  for (int i = 0; i < 13; ++i) out[i] = s[i];
}

// i-th output of SplitMix64 seeded with `seed`, for cross-checks.
void orc_splitmix64(uint64_t seed, long n, uint64_t* out) {
  uint64_t s = seed;
  for (long i = 0; i < n; ++i) out[i] = splitmix64_next(s);
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
