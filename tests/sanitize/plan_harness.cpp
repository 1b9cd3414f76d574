// Host-only driver of the planner, the reordering planner and the pass-kernel
// generator over many random gate lists, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_cpu.py.  No GPU call is
// made; the few device entry points qs_reorder.cpp refers to are stubs here.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "qs_internal.h"

namespace qs {
// run_reordered (not exercised here) refers to these.
Status run_gates(StateImpl*, const std::vector<XGate>&, int) { return Status::ok(); }
Status launch_permute(StateImpl*, const int32_t*) { return Status::ok(); }
Status hip_status(hipError_t e, const char*) {
  Status s;
  if (e != hipSuccess) s.code = QS_EHIP;
  return s;
}
}  // namespace qs

using namespace qs;

static XGate random_gate(std::mt19937_64& rng, int n, int nparams) {
  XGate g{};
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  const int kind = (int)(rng() % 7);
  g.target = (int)(rng() % n);
  g.control = -1;
  g.param = -1;
  for (double& m : g.m) m = u(rng);
  if (kind <= 1) {
    g.kind = QS_OP_U;
  } else if (kind == 2) {  // controlled U
    g.kind = QS_OP_CU;
    do g.control = (int)(rng() % n); while (g.control == g.target);
  } else if (kind == 3) {  // controlled phase (diagonal, d0 = 1)
    g.kind = QS_OP_CU;
    do g.control = (int)(rng() % n); while (g.control == g.target);
    g.m[0] = 1.0; g.m[1] = 0.0; g.m[2] = g.m[3] = g.m[4] = g.m[5] = 0.0;
  } else if (kind == 4) {  // diagonal
    g.kind = QS_OP_U;
    g.m[2] = g.m[3] = g.m[4] = g.m[5] = 0.0;
  } else {  // rotation
    g.kind = QS_OP_RX + (int)(rng() % 3);
    g.param = (int)(rng() % nparams);
    if (g.kind == QS_OP_RZ) g.m[2] = g.m[3] = g.m[4] = g.m[5] = 0.0;
  }
  return g;
}

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? atoi(argv[1]) : 60;
  std::mt19937_64 rng(1601);
  long long passes = 0, kernels = 0, reorders = 0;
  for (int r = 0; r < rounds; ++r) {
    const int dtype = (r & 1) ? QS_C64 : QS_C128;
    const int n = 13 + (int)(rng() % 22);  // 13 .. 34
    if (dtype == QS_C128 && n > 33) continue;
    const int ngates = 1 + (int)(rng() % 400);
    std::vector<XGate> gates;
    for (int i = 0; i < ngates; ++i) gates.push_back(random_gate(rng, n, 16));
    for (int wide = 0; wide < 2; ++wide) {
      Plan plan;
      plan_gates(n, dtype, gates, true, &plan, true, 1 << 30, false, wide != 0);
      passes += (long long)plan.passes.size();
      for (const Pass& p : plan.passes)
        if (p.kind == kPassFused) kernels += !jit_pass_text(plan, p, n, dtype, false).empty();
    }
    // the adjoint's planning: gradient slots, no single-gate passes
    Plan ap;
    plan_gates(n, dtype, gates, true, &ap, false, kAdjMaxSlots, true);
    for (const Pass& p : ap.passes)
      if (p.kind == kPassFused) kernels += !jit_pass_text(ap, p, n, dtype, true).empty();
    ReorderPlan rp;
    const int nlocal = n - 1 - (int)(rng() % 3);
    if (plan_reorder(n, nlocal, gates, &rp).good()) reorders += (long long)rp.remap_at.size();
  }
  printf("rounds %d passes %lld kernels %lld reorderings %lld\n", rounds, passes, kernels, reorders);
  return 0;
}
