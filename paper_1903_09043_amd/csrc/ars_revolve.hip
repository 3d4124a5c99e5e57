// ars_revolve.hip -- binomial checkpointing plan for reversing n explicit
// steps with s snapshot slots (slot 0 holds U^0), host code.
//
// T(n, s) = minimal number of forward steps to run the adjoints of steps
// n-1, ..., 0 when the state at the start of the range is in a slot and s
// slots (that one included) are available:
//   T(1, s) = 0,   T(n, 1) = n (n - 1) / 2,
//   T(n, s) = min_{1 <= m < n} [ m + T(n - m, s - 1) + T(m, s) ]
// (advance m steps and store U^m, reverse the right part with one slot
// fewer, then the left part).  Its value equals Griewank's closed form
// r n - C(s + r, s + 1) with r the smallest integer such that
// C(s + r, s) >= n; tests check both against brute force.
#include <cstdint>
#include <vector>

#include "../../include/ars.h"

namespace {

struct Plan {
  int N, S;
  std::vector<int64_t> T;  // (N+1) x (S+1)
  std::vector<int> split;
  int64_t& t(int n, int s) { return T[(size_t)n * (S + 1) + s]; }
  int& m(int n, int s) { return split[(size_t)n * (S + 1) + s]; }
  Plan(int n, int s) : N(n), S(s), T((size_t)(n + 1) * (s + 1), 0), split((size_t)(n + 1) * (s + 1), 0) {
    for (int nn = 1; nn <= N; ++nn)
      for (int ss = 1; ss <= S; ++ss) {
        if (nn == 1) {
          t(nn, ss) = 0;
          continue;
        }
        if (ss == 1) {
          t(nn, ss) = (int64_t)nn * (nn - 1) / 2;
          continue;
        }
        int64_t best = -1;
        int bm = 1;
        for (int mm = 1; mm < nn; ++mm) {
          const int64_t c = mm + t(nn - mm, ss - 1) + t(mm, ss);
          if (best < 0 || c < best) {
            best = c;
            bm = mm;
          }
        }
        t(nn, ss) = best;
        m(nn, ss) = bm;
      }
  }
};

struct Emitter {
  int32_t* out;
  int cap, count;
  int64_t fwd;
  void emit(int op, int step, int arg) {
    if (out && count < cap) {
      out[4 * count + 0] = op;
      out[4 * count + 1] = step;
      out[4 * count + 2] = arg;
      out[4 * count + 3] = 0;
    }
    ++count;
  }
};

enum { OP_ADVANCE = 0, OP_STORE = 1, OP_RESTORE = 2, OP_ADJOINT = 3 };

void reverse_range(Plan& P, Emitter& E, int lo, int hi, int slot, int s) {
  const int n = hi - lo;
  if (n == 1) {
    E.emit(OP_RESTORE, lo, slot);
    E.emit(OP_ADJOINT, lo, 0);
    return;
  }
  if (s == 1) {
    for (int k = hi - 1; k >= lo; --k) {
      E.emit(OP_RESTORE, lo, slot);
      if (k > lo) {
        E.emit(OP_ADVANCE, lo, k);
        E.fwd += k - lo;
      }
      E.emit(OP_ADJOINT, k, 0);
    }
    return;
  }
  const int mm = P.m(n, s);
  E.emit(OP_RESTORE, lo, slot);
  E.emit(OP_ADVANCE, lo, lo + mm);
  E.fwd += mm;
  const int slot2 = slot + 1;  // slots are used as a stack
  E.emit(OP_STORE, lo + mm, slot2);
  reverse_range(P, E, lo + mm, hi, slot2, s - 1);
  reverse_range(P, E, lo, lo + mm, slot, s);
}

}  // namespace

extern "C" {

int64_t ars_revolve_cost(int n, int s) {
  if (n < 1 || s < 1) return -1;
  Plan P(n, s);
  return P.t(n, s);
}

int ars_revolve_plan(int n, int s, int32_t* actions, int cap, int64_t* forward_steps) {
  if (n < 1 || s < 1 || cap < 0) return ARS_EINVAL;
  Plan P(n, s);
  Emitter E{actions, cap, 0, 0};
  reverse_range(P, E, 0, n, 0, s);
  if (forward_steps) *forward_steps = E.fwd;
  return E.count;
}

}  // extern "C"
