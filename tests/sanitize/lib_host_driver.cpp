// Host driver that exercises the library's host-only entry points (no GPU
// call) under AddressSanitizer and UndefinedBehaviorSanitizer: configuration
// checks, host-side initial states of every problem, revolve plans and the
// batch set-up.  Built with the sanitizers on the host pass only and run by
// tests/test_sanitizers.py.
#include <cstdio>
#include <vector>

#include "../../include/ars.h"

static ars_config rb(int dim, int nx, int ny, int nz) {
  ars_config c{};
  c.dim = dim;
  c.n[0] = nx;
  c.n[1] = dim == 3 ? ny : nz;
  c.n[2] = dim == 3 ? nz : 1;
  c.L[0] = 2.0;
  c.L[1] = 1.0;
  c.L[2] = 1.0;
  c.gamma = 5.0 / 3.0;
  c.g = 1.0;
  c.mu = 2e-3;
  c.kappa = 3e-3;
  c.K = 1.1;
  c.cfl = 0.4;
  c.low_mach = 1;
  c.bc[dim - 1][0] = c.bc[dim - 1][1] = ARS_BC_WALL;
  c.wall_noslip = 1;
  c.thermal[0] = c.thermal[1] = ARS_T_FIXED;
  c.T_wall[0] = 1.0;
  c.T_wall[1] = 0.5;
  return c;
}

int main() {
  int bad = 0;
  const int shapes[][4] = {{2, 64, 1, 32}, {2, 1, 1, 7}, {2, 7, 1, 5}, {3, 6, 5, 4}, {3, 1, 1, 9}, {3, 2, 3, 1}};
  for (const auto& sh : shapes) {
    ars_config c = rb(sh[0], sh[1], sh[2], sh[3]);
    if (ars_validate(&c) != ARS_OK) ++bad;
    ars_ctx* x = nullptr;
    if (ars_create(&c, &x) != ARS_OK) {
      ++bad;
      continue;
    }
    std::vector<double> h(ars_state_len(x));
    const double prm_rb[4] = {1.0, 0.5, -1.0, 1e-2};
    const double prm_u[5] = {1.0, 0.1, 0.2, 0.3, 2.0};
    if (ars_init_state_host(x, ARS_PROB_RB, prm_rb, 4, 11, h.data()) != ARS_OK) ++bad;
    if (ars_init_state_host(x, ARS_PROB_UNIFORM, prm_u, 5, 0, h.data()) != ARS_OK) ++bad;
    if (ars_init_state_host(x, ARS_PROB_ISOTHERMAL, nullptr, 0, 0, h.data()) != ARS_OK) ++bad;
    if (ars_init_state_host(x, ARS_PROB_SOD, nullptr, 0, 0, h.data()) != ARS_OK) ++bad;
    const double prm_g[1] = {0.1};
    const int rg = ars_init_state_host(x, ARS_PROB_GRESHO, prm_g, 1, 0, h.data());
    if (rg != (sh[0] == 2 ? ARS_OK : ARS_EINVAL)) ++bad;
    if (ars_init_state_host(x, 99, nullptr, 0, 0, h.data()) != ARS_EINVAL) ++bad;
    if (ars_set_tiling(x, 0, 0) != ARS_EINVAL || ars_set_tiling(x, 3, 2) != ARS_OK) ++bad;
    ars_destroy(x);
  }
  // invalid configurations
  ars_config c = rb(2, 8, 1, 8);
  c.gamma = 1.0;
  if (ars_validate(&c) != ARS_EINVAL) ++bad;
  c = rb(2, 8, 1, 8);
  c.bc[1][0] = ARS_BC_PERIODIC;
  if (ars_validate(&c) != ARS_EINVAL) ++bad;
  // revolve plans
  for (int n : {1, 2, 7, 50, 200}) {
    for (int s : {1, 2, 3, 16}) {
      int64_t fw = 0;
      const int na = ars_revolve_plan(n, s, nullptr, 0, &fw);
      if (na <= 0) {
        ++bad;
        continue;
      }
      std::vector<int32_t> a(4 * (size_t)na);
      if (ars_revolve_plan(n, s, a.data(), na, &fw) != na || fw != ars_revolve_cost(n, s)) ++bad;
    }
  }
  // batch set-up (host only)
  std::vector<ars_config> cs = {rb(2, 64, 1, 32), rb(2, 1, 1, 7), rb(2, 256, 1, 128), rb(2, 7, 1, 5)};
  ars_batch* b = nullptr;
  if (ars_batch_create((int)cs.size(), cs.data(), &b) != ARS_OK) {
    ++bad;
  } else {
    std::vector<int> zc(cs.size());
    int rows = 0;
    if (ars_batch_get_tiling(b, &rows, zc.data()) != ARS_OK) ++bad;
    if (ars_batch_set_tiling(b, 8, nullptr) != ARS_OK) ++bad;
    if (ars_batch_state_len(b) == 0 || ars_batch_table_bytes(b) == 0) ++bad;
    ars_batch_destroy(b);
  }
  std::printf(bad ? "FAILED %d\n" : "ok\n", bad);
  return bad ? 1 : 0;
}
