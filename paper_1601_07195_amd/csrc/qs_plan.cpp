// qs_plan.cpp -- the fusion planner (host only).
//
// Cache blocking by gate fusion (qHiPSTER Sec. 4.4, Fig. 4) re-planned for a
// GPU: instead of one last-level-cache block of the low qubits, every pass
// picks its own tile -- the low qubits (for coalesced HBM access) plus up to
// five high qubits -- and takes as many gates as fit, so that the state makes
// one HBM round trip per pass instead of one per gate.
//
// Which gates a pass can take:
//   * a non-diagonal gate needs its target in the tile (its control may be
//     anywhere: outside the tile it is a per-tile predicate);
//   * a diagonal gate (controlled phases, RZ, ...) fits any pass: on a
//     qubit outside the tile it is a per-tile scalar.
// Gates are taken in order, and a later gate may move ahead of gates left
// for a later pass only if it commutes with each of them.  Two gates commute
// here when every qubit they share is acted on diagonally by both (a control
// acts diagonally; so does the target of a diagonal gate) -- a sufficient
// condition, exact in arithmetic.
//
// Inside a pass, non-diagonal gates act on register bits; the planner tracks
// which tile bits sit in registers and inserts an on-chip remap (through LDS)
// when a gate's target is not one of them, choosing the next register set as
// the targets needed soonest.
#include <algorithm>
#include <cstring>

#include "qs_internal.h"

namespace qs {

FuseGeom fuse_geom(int dtype, bool wide) {
  FuseGeom g;
  // 8 (complex128) or 16 (complex64) amplitudes per thread: more register
  // bits raise register pressure past two waves per SIMD on gfx950.
  if (dtype == QS_C128) {
    g.nreg = 3;
    g.L = wide ? 4 : 6;
    g.lane0 = 0;
  } else {
    g.nreg = 4;
    g.L = wide ? 5 : 7;
    g.lane0 = 1;
  }
  g.T = g.nreg + kFuseThreadBits;
  return g;
}

bool gate_is_diagonal(const XGate& g) {
  // A rotation keeps the form of its generator (its gradient term depends
  // on it): only RZ counts as diagonal, whatever the angle.
  if (g.kind == QS_OP_RX || g.kind == QS_OP_RY) return false;
  if (g.kind == QS_OP_RZ) return true;
  return g.m[2] == 0.0 && g.m[3] == 0.0 && g.m[4] == 0.0 && g.m[5] == 0.0;
}

namespace {

constexpr int kWindow = 512;     // gates scanned ahead for one pass
constexpr int kMaxSkipped = 96;  // stop scanning once this many gates wait

// Per-qubit action of a gate: 0 = none, 1 = diagonal, 2 = non-diagonal.
struct Footprint {
  int q[2];
  int act[2];
  int nq;
};

Footprint footprint(const XGate& g) {
  Footprint f;
  f.nq = 0;
  const bool diag = gate_is_diagonal(g);
  f.q[f.nq] = g.target;
  f.act[f.nq++] = diag ? 1 : 2;
  if (g.control >= 0) {
    f.q[f.nq] = g.control;
    f.act[f.nq++] = 1;
  }
  return f;
}

bool commute(const Footprint& a, const Footprint& b) {
  for (int i = 0; i < a.nq; ++i)
    for (int j = 0; j < b.nq; ++j)
      if (a.q[i] == b.q[j] && (a.act[i] == 2 || b.act[j] == 2)) return false;
  return true;
}

// c = a * b for 2x2 complex matrices in the 8-double layout.
void mul2(const double* a, const double* b, double* c) {
  double t[8];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      double re = 0.0, im = 0.0;
      for (int k = 0; k < 2; ++k) {
        const double ar = a[4 * i + 2 * k], ai = a[4 * i + 2 * k + 1];
        const double br = b[4 * k + 2 * j], bi = b[4 * k + 2 * j + 1];
        re += ar * br - ai * bi;
        im += ar * bi + ai * br;
      }
      t[4 * i + 2 * j] = re;
      t[4 * i + 2 * j + 1] = im;
    }
  std::memcpy(c, t, sizeof(t));
}

// What the planner remembers about an emitted fused op.
struct OpMeta {
  bool remap;
  bool mergeable;  // no gradient slot
  int target, control;
  Footprint fp;
};

struct Mapping {
  int thr[8];
  int reg[5];
};

bool same_lanes(const Mapping& a, const Mapping& b) {
  for (int i = 0; i < 6; ++i)
    if (a.thr[i] != b.thr[i]) return false;
  return true;
}

FMap to_fmap(const Mapping& m) {
  FMap f;
  std::memset(&f, 0, sizeof(f));
  for (int i = 0; i < 8; ++i) f.thr[i] = (int8_t)m.thr[i];
  for (int k = 0; k < 5; ++k) f.reg[k] = (int8_t)m.reg[k];
  return f;
}

}  // namespace

void plan_gates(int n, int dtype, const std::vector<XGate>& gates, bool fuse, Plan* out,
                bool allow_single, int max_grad, bool grad, bool wide) {
  out->passes.clear();
  out->ops.clear();
  out->maps.clear();
  out->order.clear();
  out->grad_rows.clear();
  out->run_tab.clear();
  const int N = (int)gates.size();
  out->pass_of.assign(N, -1);
  const FuseGeom G = fuse_geom(dtype, wide);
  out->geom = G;

  auto stream_pass = [&](int g) {
    Pass p;
    std::memset(&p, 0, sizeof(p));
    p.kind = gates[g].control >= 0 ? kPassCU : kPass1q;
    p.gate = g;
    out->pass_of[g] = (int)out->passes.size();
    out->order.push_back(g);
    out->passes.push_back(p);
  };

  if (!fuse || n < G.T) {
    for (int g = 0; g < N; ++g) stream_pass(g);
    return;
  }

  std::vector<Footprint> fp(N);
  std::vector<char> diag(N);
  for (int g = 0; g < N; ++g) {
    fp[g] = footprint(gates[g]);
    diag[g] = gate_is_diagonal(gates[g]);
  }
  std::vector<char> done(N, 0);
  std::vector<OpMeta> meta;  // aligned with out->ops
  const int slots = G.T - G.L;
  int start = 0;
  while (start < N) {
    // ---- choose the gates of this pass
    std::vector<int> take;
    std::vector<int> skipped;
    std::vector<int> high;  // high tile qubits (unsorted while collecting)
    auto in_tile = [&](int q) {
      return q < G.L || std::find(high.begin(), high.end(), q) != high.end();
    };
    int ngrad = 0;
    for (int g = start; g < N && g < start + kWindow; ++g) {
      if (done[g]) continue;
      if (grad && gates[g].param >= 0 && ngrad >= max_grad) break;
      bool blocked = false;
      for (int s : skipped)
        if (!commute(fp[g], fp[s])) {
          blocked = true;
          break;
        }
      if (!blocked) {
        const int t = gates[g].target;
        if (diag[g] || in_tile(t)) {
          take.push_back(g);
          ngrad += grad && gates[g].param >= 0;
          continue;
        }
        if ((int)high.size() < slots) {
          high.push_back(t);
          take.push_back(g);
          ngrad += grad && gates[g].param >= 0;
          continue;
        }
      }
      skipped.push_back(g);
      if ((int)skipped.size() >= kMaxSkipped) break;
    }
    for (int g : take) done[g] = 1;
    while (start < N && done[start]) ++start;

    if (take.size() == 1 && allow_single) {  // one gate: the streaming kernels are as cheap or cheaper
      stream_pass(take[0]);
      continue;
    }

    // ---- tile: fill the free high slots with the lowest unused qubits
    for (int q = G.L; q < n && (int)high.size() < slots; ++q)
      if (!in_tile(q)) high.push_back(q);
    std::sort(high.begin(), high.end());
    int tile_bit_of[64];
    for (int q = 0; q < 64; ++q) tile_bit_of[q] = -1;
    for (int q = 0; q < G.L; ++q) tile_bit_of[q] = q;
    for (int h = 0; h < slots; ++h) tile_bit_of[high[h]] = G.L + h;

    // ---- register allocation
    // Lanes (thread bits 0..5) always start and end on tile bits lane0 ..
    // lane0 + 5 (coalesced); complex64 keeps tile bit 0 in register bit 0 at
    // load and store (it lives inside the 16-byte unit).
    const int free0 = G.lane0 + 6;  // first tile bit that is neither lane nor in-unit
    std::vector<int> targets;        // tile bit of each non-diagonal gate, in order
    for (int g : take)
      if (!diag[g]) targets.push_back(tile_bit_of[gates[g].target]);

    Mapping cur;
    for (int i = 0; i < 6; ++i) cur.thr[i] = G.lane0 + i;
    {
      // registers (beyond the in-unit bit) and wave bits from the free bits,
      // preferring the first free-bit targets of the pass
      std::vector<int> pick;
      for (int tb : targets)
        if (tb >= free0 && std::find(pick.begin(), pick.end(), tb) == pick.end() &&
            (int)pick.size() < G.nreg - G.lane0)
          pick.push_back(tb);
      for (int tb = free0; tb < G.T && (int)pick.size() < G.nreg - G.lane0; ++tb)
        if (std::find(pick.begin(), pick.end(), tb) == pick.end()) pick.push_back(tb);
      int k = 0;
      if (G.lane0 == 1) cur.reg[k++] = 0;
      for (int tb : pick) cur.reg[k++] = tb;
      for (; k < 5; ++k) cur.reg[k] = -1;
      int w = 6;
      for (int tb = free0; tb < G.T; ++tb)
        if (std::find(pick.begin(), pick.end(), tb) == pick.end()) cur.thr[w++] = tb;
    }
    const Mapping load = cur;

    Pass p;
    std::memset(&p, 0, sizeof(p));
    p.kind = kPassFused;
    p.op_first = (int)out->ops.size();
    p.map_load = (int)out->maps.size();
    out->maps.push_back(to_fmap(load));
    p.nh = slots;
    for (int h = 0; h < slots; ++h) p.hpos[h] = (int8_t)high[h];
    p.grad_first = (int)out->grad_rows.size();
    p.ngrad = 0;

    auto where = [&](const Mapping& m, int q) -> int32_t {
      const int tb = tile_bit_of[q];
      if (tb < 0) return make_spec(kOutside, q);
      for (int k = 0; k < G.nreg; ++k)
        if (m.reg[k] == tb) return make_spec(kInReg, k);
      for (int i = 0; i < 8; ++i)
        if (m.thr[i] == tb) return make_spec(kInThread, i);
      return make_spec(kOutside, q);  // unreachable: every tile bit is mapped
    };
    auto emit_remap = [&](const Mapping& to) {
      FOp op;
      std::memset(&op, 0, sizeof(op));
      op.kind = kOpRemap;
      op.aux = (int)out->maps.size() - 1;  // the current mapping is the last pushed
      out->maps.push_back(to_fmap(to));
      op.tgt = (int)out->maps.size() - 1;
      op.ctl = make_spec(kNoBit, 0);
      out->ops.push_back(op);
      OpMeta mt;
      mt.remap = true;
      mt.mergeable = false;
      mt.target = mt.control = -1;
      mt.fp.nq = 0;
      meta.push_back(mt);
      ++p.remaps;
    };

    // Fold gate g into the latest earlier op of this pass that it does not
    // commute with, when both act on the same target and control (the gate
    // moves back past ops it commutes with, which is exact): U then U, diag
    // then diag, a diag after a register U, or a U after a diag whose target
    // sat in a register.  The merged op stays where the earlier one was, with
    // that op's bit locations.
    auto try_merge = [&](int g) -> bool {
      const XGate& x = gates[g];
      for (int j = (int)out->ops.size() - 1; j >= p.op_first; --j) {
        OpMeta& m = meta[j];
        if (m.remap) continue;
        if (commute(fp[g], m.fp)) continue;
        if (!m.mergeable || m.target != x.target || m.control != x.control) return false;
        FOp& y = out->ops[j];
        const int ykind = y.kind & 255;
        if (diag[g]) {
          if (ykind == kOpDiag) {  // elementwise product of diagonals
            double d0[8] = {x.m[0], x.m[1], 0, 0, 0, 0, 0, 0}, e0[8] = {y.m[0], y.m[1], 0, 0, 0, 0, 0, 0};
            double d1[8] = {x.m[6], x.m[7], 0, 0, 0, 0, 0, 0}, e1[8] = {y.m[6], y.m[7], 0, 0, 0, 0, 0, 0};
            double r0[8], r1[8];
            mul2(d0, e0, r0);
            mul2(d1, e1, r1);
            y.m[0] = r0[0]; y.m[1] = r0[1]; y.m[6] = r1[0]; y.m[7] = r1[1];
          } else {  // diag(x) * U
            mul2(x.m, y.m, y.m);
          }
        } else {
          if (ykind == kOpU) {
            mul2(x.m, y.m, y.m);
          } else {  // U * diag(y): only if y's target was a register bit
            if ((y.tgt >> 8) != kInReg) return false;
            double dm[8] = {y.m[0], y.m[1], 0, 0, 0, 0, y.m[6], y.m[7]};
            mul2(x.m, dm, y.m);
            y.kind = kOpU;
            y.tgt = y.tgt & 255;
          }
          m.fp.act[0] = 2;  // the merged op is no longer diagonal on its target
        }
        return true;
      }
      return false;
    };

    int ti = 0;  // index into targets
    for (int g : take) {
      const XGate& x = gates[g];
      const bool gradop = grad && x.param >= 0;
      if (!gradop && try_merge(g)) {
        ti += !diag[g];
        out->pass_of[g] = (int)out->passes.size();
        out->order.push_back(g);
        continue;
      }
      FOp op;
      std::memset(&op, 0, sizeof(op));
      std::memcpy(op.m, x.m, sizeof(op.m));
      op.aux = -1;
      if (gradop) {  // gradient slot; the Pauli generator rides in bits 8.. of kind
        op.aux = p.ngrad++;
        out->grad_rows.push_back(x.param);
      }
      if (diag[g]) {
        op.kind = kOpDiag | (op.aux >= 0 ? (x.kind - QS_OP_RX + 1) << 8 : 0);
        op.tgt = where(cur, x.target);
      } else {
        const int tb = targets[ti];
        int rk = -1;
        for (int k = 0; k < G.nreg; ++k)
          if (cur.reg[k] == tb) rk = k;
        if (rk < 0) {
          // New register set: the distinct targets needed soonest, then the
          // current registers, in that order of preference.
          std::vector<int> want;
          for (int j = ti; j < (int)targets.size() && (int)want.size() < G.nreg; ++j)
            if (std::find(want.begin(), want.end(), targets[j]) == want.end())
              want.push_back(targets[j]);
          for (int k = 0; k < G.nreg && (int)want.size() < G.nreg; ++k)
            if (std::find(want.begin(), want.end(), cur.reg[k]) == want.end())
              want.push_back(cur.reg[k]);
          Mapping nm = cur;
          // registers keep their slot when they stay; newcomers take the
          // slots of leavers, and leavers take the thread slots of newcomers
          std::vector<int> leave, enter;
          for (int k = 0; k < G.nreg; ++k)
            if (std::find(want.begin(), want.end(), cur.reg[k]) == want.end()) leave.push_back(k);
          for (int tbw : want) {
            bool isreg = false;
            for (int k = 0; k < G.nreg; ++k) isreg |= cur.reg[k] == tbw;
            if (!isreg) enter.push_back(tbw);
          }
          for (size_t e = 0; e < enter.size(); ++e) {
            const int k = leave[e];
            const int old_tb = cur.reg[k];
            int ti_slot = -1;
            for (int i = 0; i < 8; ++i)
              if (cur.thr[i] == enter[e]) ti_slot = i;
            nm.reg[k] = enter[e];
            nm.thr[ti_slot] = old_tb;
          }
          emit_remap(nm);
          cur = nm;
          for (int k = 0; k < G.nreg; ++k)
            if (cur.reg[k] == tb) rk = k;
        }
        op.kind = kOpU | (op.aux >= 0 ? (x.kind - QS_OP_RX + 1) << 8 : 0);
        op.tgt = rk;
        ++ti;
      }
      op.ctl = x.control >= 0 ? where(cur, x.control) : make_spec(kNoBit, 0);
      out->pass_of[g] = (int)out->passes.size();
      out->order.push_back(g);
      out->ops.push_back(op);
      OpMeta mt;
      mt.remap = false;
      mt.mergeable = !gradop;
      mt.target = x.target;
      mt.control = x.control;
      mt.fp = fp[g];
      meta.push_back(mt);
    }
    // ---- store mapping: coalesced lanes, and (complex64) tile bit 0 in
    // register bit 0; otherwise remap back to the load mapping
    bool ok = same_lanes(cur, load) && (G.lane0 == 0 || cur.reg[0] == 0);
    if (!ok) {
      emit_remap(load);
      cur = load;
    }
    p.map_store = (int)out->maps.size() - 1;
    // ---- phase runs.  Phase ops (diagonal, d0 = 1, no gradient slot)
    // commute with each other, so a block of consecutive ones may be
    // reordered freely.  A controlled phase is symmetric in its two qubits,
    // so each takes as target the qubit held closest (register, then thread
    // bit, then outside the tile) and as control the other.  The block is
    // then sorted by target, and the ops on one target whose control is not
    // a register bit become one run header followed by their entries: the
    // kernel multiplies their phases per lane and scales the tile once.
    // Forward passes only: the adjoint kernels have no registers to spare
    // for it.
    if (!grad) {
      auto is_phase = [&](const FOp& o) {
        return (o.kind & 255) == kOpDiag && o.aux < 0 && o.m[0] == 1.0 && o.m[1] == 0.0;
      };
      auto rank = [](int32_t spec) { return spec >> 8; };  // kInReg < kInThread < kOutside
      std::vector<FOp> nops;
      std::vector<OpMeta> nmeta;
      size_t i = (size_t)p.op_first;
      while (i < out->ops.size()) {
        if (!is_phase(out->ops[i])) {
          nops.push_back(out->ops[i]);
          nmeta.push_back(meta[i]);
          ++i;
          continue;
        }
        size_t j = i;
        while (j < out->ops.size() && is_phase(out->ops[j])) ++j;
        std::vector<FOp> blk(out->ops.begin() + i, out->ops.begin() + j);
        for (FOp& o : blk)
          if (rank(o.ctl) != kNoBit && rank(o.ctl) < rank(o.tgt)) std::swap(o.tgt, o.ctl);
        std::stable_sort(blk.begin(), blk.end(), [](const FOp& a, const FOp& b) { return a.tgt < b.tgt; });
        auto member = [&](const FOp& o) { return rank(o.ctl) != kInReg; };
        size_t a = 0;
        while (a < blk.size()) {
          size_t b = a;
          if (member(blk[a]))
            while (b + 1 < blk.size() && member(blk[b + 1]) && blk[b + 1].tgt == blk[a].tgt) ++b;
          OpMeta om;
          om.remap = true;  // never a merge target
          om.mergeable = false;
          om.target = om.control = -1;
          om.fp.nq = 0;
          if (b > a) {
            FOp h;
            std::memset(&h, 0, sizeof(h));
            h.kind = kOpPhaseRun;
            h.tgt = blk[a].tgt;
            h.ctl = make_spec(kNoBit, 0);
            // entries controlled by a qubit outside the tile: their product
            // depends only on the tile index, so it goes into two tables
            // (low and high bits of the tile index) built here; the other
            // entries stay explicit.  m[0]: the tables' offset in run_tab
            // (made a byte offset at upload), m[1]: low-table bits, m[2]: 1
            // when the run has tables.
            std::vector<const FOp*> lane, outside;
            for (size_t k = a; k <= b; ++k)
              ((blk[k].ctl >> 8) == kOutside ? outside : lane).push_back(&blk[k]);
            if (!outside.empty()) {
              const int nb = n - G.T;  // tile-index bits
              const int lb = (nb + 1) / 2, hb = nb - lb;
              auto tile_bit = [&](int q) {  // tile-index bit of an outside qubit
                int below = 0;
                for (int t = 0; t < n && t < q; ++t) below += in_tile(t);
                return q - below;
              };
              const size_t off = out->run_tab.size();
              out->run_tab.resize(off + 2 * ((size_t)1 << lb) + 2 * ((size_t)1 << hb), 0.0);
              double* tlo = out->run_tab.data() + off;
              double* thi = tlo + 2 * ((size_t)1 << lb);
              for (size_t x = 0; x < ((size_t)1 << lb); ++x) { tlo[2 * x] = 1.0; }
              for (size_t x = 0; x < ((size_t)1 << hb); ++x) { thi[2 * x] = 1.0; }
              for (const FOp* e : outside) {
                const int j = tile_bit(e->ctl & 255);
                const bool low = j < lb;
                double* t = low ? tlo : thi;
                const int bit = low ? j : j - lb;
                const size_t size = (size_t)1 << (low ? lb : hb);
                for (size_t x = 0; x < size; ++x) {
                  if (!((x >> bit) & 1)) continue;
                  const double r = t[2 * x], i = t[2 * x + 1];
                  t[2 * x] = r * e->m[6] - i * e->m[7];
                  t[2 * x + 1] = r * e->m[7] + i * e->m[6];
                }
              }
              h.m[0] = (double)off;
              h.m[1] = (double)lb;
              h.m[2] = 1.0;
            }
            // two or more entries with no control or a thread-bit control:
            // their product by the thread index goes into one more table of
            // one value per thread (m[3]: its offset in run_tab, made a byte
            // offset at upload; m[4]: 1 when present), and no entries follow
            if (lane.size() >= 2) {
              constexpr size_t nt = (size_t)1 << kFuseThreadBits;
              const size_t off = out->run_tab.size();
              out->run_tab.resize(off + 2 * nt, 0.0);
              double* t = out->run_tab.data() + off;
              for (size_t x = 0; x < nt; ++x) t[2 * x] = 1.0;
              for (const FOp* e : lane) {
                const bool thr = (e->ctl >> 8) == kInThread;
                const int bit = e->ctl & 255;
                for (size_t x = 0; x < nt; ++x) {
                  if (thr && !((x >> bit) & 1)) continue;
                  const double r = t[2 * x], i = t[2 * x + 1];
                  t[2 * x] = r * e->m[6] - i * e->m[7];
                  t[2 * x + 1] = r * e->m[7] + i * e->m[6];
                }
              }
              h.m[3] = (double)off;
              h.m[4] = 1.0;
              lane.clear();
            }
            h.aux = (int)lane.size();
            nops.push_back(h);
            nmeta.push_back(om);
            for (const FOp* le : lane) {
              FOp e = *le;
              e.kind = kOpPhaseEntry;
              nops.push_back(e);
              nmeta.push_back(om);
            }
          } else {
            nops.push_back(blk[a]);
            nmeta.push_back(om);
          }
          a = b + 1;
        }
        i = j;
      }
      out->ops.resize((size_t)p.op_first);
      meta.resize((size_t)p.op_first);
      out->ops.insert(out->ops.end(), nops.begin(), nops.end());
      meta.insert(meta.end(), nmeta.begin(), nmeta.end());
    }
    p.nops = (int)out->ops.size() - p.op_first;
    out->passes.push_back(p);
  }
}

}  // namespace qs
