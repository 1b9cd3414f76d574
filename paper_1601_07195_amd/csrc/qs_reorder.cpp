// qs_reorder.cpp -- qubit-reordering planner (host) and its one-GPU runner.
//
// Communication avoidance by state reordering (Sec. 6): when the state is
// split over 2^(n - m) shards by its top n - m qubits (Sec. 3.2), a gate
// whose target is one of those qubits pairs amplitudes held by different
// shards.  Sec. 3.2's scheme pays two pairwise half-state exchanges for every
// such gate (Table 2, cases 2, 5, 6).  Reordering instead relabels qubits so
// that the target becomes a local qubit: one all-to-all swaps k upper qubits
// with k local ones, after which every gate on them is local until they are
// swapped out again.
//
// The planner walks the gate list keeping the position of every qubit.
// Diagonal gates never need one (on an upper qubit they are a per-shard
// scalar), and neither do controls (a per-shard predicate).  When a
// non-diagonal gate finds its target at an upper position, one reordering
// brings it in together with every other upper qubit that is needed before
// the local qubit it would displace (furthest next use first, Belady's
// rule); local qubits of the 1 KiB block bits are displaced last, so that
// the swaps move whole blocks.  After the last gate one more reordering
// restores the caller's qubit order.
//
// On one GPU the shards are the top n - m bits of the index: the runner
// applies the reorderings with the in-place permutation kernels and the
// gates between them with the fusion planner, and the result equals the
// plain gate list applied in order.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "qs_internal.h"

namespace qs {

namespace {
constexpr int kBlockBits = 7;  // amplitude bits of 1 KiB at complex64 (6 at complex128)
}

Status plan_reorder(int n, int nlocal, const std::vector<XGate>& gates, ReorderPlan* out) {
  if (nlocal < 1 || nlocal > n) return Status{QS_EINVAL, "reorder: nlocal out of range"};
  const int N = (int)gates.size();
  const int m = nlocal;
  out->tgt.assign(N, -1);
  out->ctl.assign(N, -1);
  out->remap_at.clear();
  out->remap_perm.clear();
  out->final_perm.assign(n, 0);
  memset(&out->info, 0, sizeof(out->info));

  std::vector<char> diag(N);
  std::vector<std::vector<int>> uses(n);  // gates with a non-diagonal action on each qubit, in order
  for (int g = 0; g < N; ++g) {
    diag[g] = gate_is_diagonal(gates[g]);
    if (!diag[g]) uses[gates[g].target].push_back(g);
  }
  std::vector<size_t> cur(n, 0);
  auto next_use = [&](int q, int g) {
    while (cur[q] < uses[q].size() && uses[q][cur[q]] < g) ++cur[q];
    return cur[q] < uses[q].size() ? uses[q][cur[q]] : INT_MAX;
  };

  std::vector<int> pos(n), at(n);  // qubit -> position, position -> qubit
  for (int q = 0; q < n; ++q) pos[q] = at[q] = q;

  for (int g = 0; g < N; ++g) {
    const XGate& x = gates[g];
    if (!diag[g] && x.target >= m) {  // Sec. 3.2's scheme, caller's order
      ++out->info.global_gates;
      out->info.traffic_pairwise += (x.control >= 0 && x.control < m) ? 1.0 : 2.0;
    }
    if (!diag[g] && pos[x.target] >= m) {
      std::vector<int> in;  // qubits at upper positions, soonest needed first
      for (int p = m; p < n; ++p) in.push_back(at[p]);
      std::stable_sort(in.begin(), in.end(),
                       [&](int a, int b) { return next_use(a, g) < next_use(b, g); });
      std::vector<int> perm(n);
      for (int p = 0; p < n; ++p) perm[p] = p;
      std::vector<char> used(n, 0);
      int k = 0;
      for (size_t i = 0; i < in.size(); ++i) {
        const int qi = in[i], pi = pos[qi];
        // the local position to give up: block-aligned before the block
        // bits, then the latest next use, then (ties) one whose qubit this
        // sends home, then one that is the incoming qubit's home
        int best = -1;
        auto better = [&](int a, int b) {
          const bool la = a >= kBlockBits, lb = b >= kBlockBits;
          if (la != lb) return la;
          const int na = next_use(at[a], g), nb = next_use(at[b], g);
          if (na != nb) return na > nb;
          const bool ha = at[a] == pi, hb = at[b] == pi;
          if (ha != hb) return ha;
          return a == qi && b != qi;
        };
        for (int p = 0; p < m; ++p)
          if (!used[p] && (best < 0 || better(p, best))) best = p;
        if (best < 0) break;
        const int qv = at[best];
        if (i > 0 && next_use(qi, g) >= next_use(qv, g)) break;
        used[best] = 1;
        perm[pi] = best;
        perm[best] = pi;
        pos[qi] = best;
        pos[qv] = pi;
        at[best] = qi;
        at[pi] = qv;
        ++k;
      }
      out->remap_at.push_back(g);
      out->remap_perm.insert(out->remap_perm.end(), perm.begin(), perm.end());
      ++out->info.remaps;
      out->info.swaps += k;
      out->info.traffic_reordered += 2.0 * (1.0 - std::ldexp(1.0, -k));
    }
    out->tgt[g] = pos[x.target];
    out->ctl[g] = x.control >= 0 ? pos[x.control] : -1;
  }
  // back to the caller's order: the qubit at position p returns to position at[p]
  int k = 0;
  for (int p = 0; p < n; ++p) {
    out->final_perm[p] = at[p];
    k += p >= m && at[p] != p;
  }
  out->info.restore_swaps = k;
  if (k > 0) out->info.traffic_reordered += 2.0 * (1.0 - std::ldexp(1.0, -k));
  return Status::ok();
}

Status run_reordered(StateImpl* s, int nlocal, const std::vector<XGate>& gates, int flags,
                     qs_reorder_info* info) {
  ReorderPlan plan;
  Status st = plan_reorder(s->n, nlocal, gates, &plan);
  if (!st.good()) return st;
  const int n = s->n;
  std::vector<XGate> seg;
  size_t r = 0;
  for (size_t g = 0; g <= gates.size(); ++g) {
    const bool remap_here = r < plan.remap_at.size() && (size_t)plan.remap_at[r] == g;
    if (remap_here || g == gates.size()) {
      if (!seg.empty()) {
        st = run_gates(s, seg, flags);
        if (!st.good()) return st;
        seg.clear();
      }
      if (remap_here) {
        st = launch_permute(s, plan.remap_perm.data() + r * n);
        if (!st.good()) return st;
        ++r;
      }
    }
    if (g < gates.size()) {
      XGate x = gates[g];
      x.target = plan.tgt[g];
      x.control = plan.ctl[g];
      seg.push_back(x);
    }
  }
  bool identity = true;
  for (int p = 0; p < n; ++p) identity &= plan.final_perm[p] == p;
  if (!identity) {
    st = launch_permute(s, plan.final_perm.data());
    if (!st.good()) return st;
  }
  if (info) *info = plan.info;
  return Status::ok();
}

}  // namespace qs
