// Host driver that exercises the oracle under AddressSanitizer and
// UndefinedBehaviorSanitizer (built and run by tests/test_sanitizers.py
// with g++; CPU only).  Every exported routine runs on small problems of
// each kind; any out-of-bounds access, use of uninitialised heap memory
// detected by the sanitizers, signed overflow or similar aborts the run.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

extern "C" {
typedef struct cfg_t {
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
  int32_t energy_form;
  int32_t pad_;
} cfg_t;
int orc_validate(const cfg_t* c);
int orc_init(const cfg_t* c, int problem, const double* prm, int nprm, uint64_t seed, double* U);
double orc_dt(const cfg_t* c, const double* U);
int orc_run(const cfg_t* c, double* U, int nsteps, const double* dt_sched, double* dt_log, double* t,
            int64_t* fault_cell, int64_t* fault_step);
int orc_tlm(const cfg_t* c, const double* U, const double* dU, double dmu, double dkappa, double dt, double* Uout,
            double* dUout);
int orc_adjoint_dense(const cfg_t* c, const double* U, const double* lam_in, double dt, double* lam_out,
                      double* gmu, double* gkappa);
void orc_diag(const cfg_t* c, const double* U, double* out);
}

static cfg_t base(int dim, int nx, int ny, int nz, double g, double mu, double kappa) {
  cfg_t c{};
  c.dim = dim;
  c.n[0] = nx;
  c.n[1] = dim == 3 ? ny : nz;
  c.n[2] = dim == 3 ? nz : 1;
  c.L[0] = c.L[1] = c.L[2] = 1.0;
  c.gamma = 5.0 / 3.0;
  c.g = g;
  c.mu = mu;
  c.kappa = kappa;
  c.K = 1.1;
  c.cfl = 0.4;
  c.low_mach = 1;
  c.dt_mode = 0;
  for (int a = 0; a < 3; ++a) c.bc[a][0] = c.bc[a][1] = 0;
  if (g != 0.0) c.bc[dim - 1][0] = c.bc[dim - 1][1] = 1;
  c.wall_noslip = 1;
  c.thermal[0] = c.thermal[1] = 1;
  c.T_wall[0] = 1.0;
  c.T_wall[1] = 0.5;
  return c;
}

static long cells(const cfg_t& c) {
  long n = 1;
  for (int a = 0; a < c.dim; ++a) n *= c.n[a];
  return n;
}

static int run_case(const char* name, cfg_t c, int problem, std::vector<double> prm, int steps, bool adjoint) {
  const long N = cells(c) * (c.dim + 2);
  std::vector<double> U(N), U0, log(steps > 0 ? steps : 1), out(16);
  if (orc_validate(&c) != 0) {
    std::printf("%s: invalid config\n", name);
    return 1;
  }
  if (orc_init(&c, problem, prm.data(), (int)prm.size(), 7, U.data()) != 0) {
    std::printf("%s: init failed\n", name);
    return 1;
  }
  U0 = U;
  double t = 0.0;
  int64_t fc = -1;
  int64_t fs = -1;
  const int rc = orc_run(&c, U.data(), steps, nullptr, log.data(), &t, &fc, &fs);
  orc_diag(&c, U.data(), out.data());
  double s = 0.0;
  for (double v : U) s += v;
  std::printf("%s: rc %d t %.6g sum %.12g\n", name, rc, t, s);
  if (adjoint) {
    const double dt = orc_dt(&c, U0.data());
    std::vector<double> d(N), o(N), lam(N), lo(N);
    for (long i = 0; i < N; ++i) {
      d[i] = std::sin(0.37 * (double)i);
      lam[i] = std::cos(0.91 * (double)i);
    }
    double gm = 0.0, gk = 0.0;
    if (orc_tlm(&c, U0.data(), d.data(), 0.0, 0.0, dt, nullptr, o.data()) != 0) return 1;
    if (orc_adjoint_dense(&c, U0.data(), lam.data(), dt, lo.data(), &gm, &gk) != 0) return 1;
    double a = 0.0, b = 0.0;
    for (long i = 0; i < N; ++i) {
      a += o[i] * lam[i];
      b += d[i] * lo[i];
    }
    std::printf("%s: <J d, l> %.15g <d, J^T l> %.15g\n", name, a, b);
    if (!(std::fabs(a - b) <= 1e-10 * (std::fabs(a) + 1e-300))) return 1;
  }
  return rc == 0 ? 0 : 1;
}

int main() {
  int bad = 0;
  bad += run_case("rb2d", base(2, 12, 1, 8, 1.0, 2e-3, 3e-3), 1, {1.0, 0.5, -1.0, 1e-2}, 20, true);
  bad += run_case("rb3d", base(3, 6, 5, 4, 1.0, 2e-3, 3e-3), 1, {1.0, 0.5, -1.0, 1e-2}, 8, true);
  bad += run_case("rb3d_column", base(3, 1, 1, 6, 1.0, 2e-3, 3e-3), 1, {1.0, 0.5, -1.0, 1e-2}, 8, false);
  bad += run_case("gresho_odd", base(2, 9, 1, 9, 0.0, 0.0, 0.0), 2, {0.1}, 10, true);
  cfg_t sod = base(2, 40, 1, 2, 0.0, 0.0, 0.0);
  sod.gamma = 1.4;
  sod.bc[0][0] = sod.bc[0][1] = 2;
  bad += run_case("sod", sod, 3, {}, 30, false);
  cfg_t iso = base(2, 2, 1, 16, 1.0, 0.0, 0.0);
  iso.thermal[0] = iso.thermal[1] = 0;  // adiabatic walls keep the isothermal column at rest
  bad += run_case("iso", iso, 4, {}, 30, false);
  std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
  return bad ? 1 : 0;
}
