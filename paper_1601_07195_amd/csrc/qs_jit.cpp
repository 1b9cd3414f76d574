// qs_jit.cpp -- fused passes compiled per pass shape at run time (ROCm
// clang in child processes, or hipRTC).
//
// The planner (qs_plan.cpp) turns a block of gates into a list of fused ops
// over a register tile (qHiPSTER Sec. 4.4, Fig. 4: one memory round trip per
// block).  The interpreter kernels in qs_fused.hip decode that list at run
// time; this file instead writes one straight-line kernel per pass, with
// every structural field of every op (kind, target register bit, where the
// control lives, which tile bits the lanes and registers hold before and
// after each LDS remap, the gradient slot) fixed in the source.  Only the
// numbers stay data: gate matrices, phases and the phase-run tables are read
// from the same uploaded op records the interpreter uses.  With nothing to
// decode and no branch merges inside the tile's register arrays, the pass
// issues little beyond the gate arithmetic itself, its remaps and its
// loads and stores.
//
// Kernels are cached by their source text (which is the pass's shape), so a
// circuit of the same form with new parameters -- the next step of a
// variational loop -- or the same circuit run again launches without
// compiling.  Missing kernels of one call are compiled together, spread over
// host threads, before the call's first launch.
#include <fcntl.h>
#include <hip/hiprtc.h>
#include <signal.h>
#include <spawn.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/wait.h>
#include <unistd.h>

#include <algorithm>
#include <chrono>
#include <fstream>
#include <cstdio>
#include <functional>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "qs_internal.h"

extern char** environ;

namespace qs {

namespace {

// ------------------------------------------------------------ emitter

struct Src {
  std::string s;
  void operator()(const char* fmt, ...) __attribute__((format(printf, 2, 3))) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    const int n = vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (n >= (int)sizeof buf) {
      std::string big((size_t)n + 1, '\0');
      va_start(ap, fmt);
      vsnprintf(&big[0], big.size(), fmt, ap);
      va_end(ap);
      big.resize((size_t)n);
      s += big;
    } else {
      s.append(buf, (size_t)n);
    }
    s += '\n';
  }
};

// Stands for the kernel's name in its text (the name is a hash of the text).
const char* const kNamePlaceholder = "QS_PASS_NAME";

// Device helpers shared by every generated kernel of a program.
const char* kPrelude = R"(
typedef double qs_d2 __attribute__((ext_vector_type(2)));
typedef float qs_f2 __attribute__((ext_vector_type(2)));
typedef float qs_f4 __attribute__((ext_vector_type(4)));
struct QsOp { int kind, tgt, ctl, aux; double m[8]; };
__device__ __forceinline__ int qs_swz128(int j) { return j ^ (((j >> 3) ^ (j >> 6) ^ (j >> 9)) & 7); }
__device__ __forceinline__ int qs_swz64(int j) { return j ^ (((j >> 4) ^ (j >> 8) ^ (j >> 12)) & 15); }
template <int CTRL>
__device__ __forceinline__ double qs_dpp(double v) {
  const unsigned long long b = (unsigned long long)__builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
// sum over a 16-lane row, every lane receives it (fixed order)
__device__ __forceinline__ double qs_row_sum16(double v) {
  v += qs_dpp<0x140>(v);
  v += qs_dpp<0x141>(v);
  v += qs_dpp<0x1B>(v);
  v += qs_dpp<0xB1>(v);
  return v;
}
// (X[A], X[B]) <- Q (X[A], X[B]) with coefficients c0..c3 in scope
#define QS_U(XR, XI, A, B) { const R ar_ = XR[A], ai_ = XI[A], br_ = XR[B], bi_ = XI[B]; \
  XR[A] = c0r * ar_ - c0i * ai_ + c1r * br_ - c1i * bi_; \
  XI[A] = c0r * ai_ + c0i * ar_ + c1r * bi_ + c1i * br_; \
  XR[B] = c2r * ar_ - c2i * ai_ + c3r * br_ - c3i * bi_; \
  XI[B] = c2r * ai_ + c2i * ar_ + c3r * bi_ + c3i * br_; }
// the same for a real matrix
#define QS_UR(XR, XI, A, B) { const R ar_ = XR[A], ai_ = XI[A], br_ = XR[B], bi_ = XI[B]; \
  XR[A] = c0r * ar_ + c1r * br_; XI[A] = c0r * ai_ + c1r * bi_; \
  XR[B] = c2r * ar_ + c3r * br_; XI[B] = c2r * ai_ + c3r * bi_; }
// X[A] *= (FR + i FI)
#define QS_SC(XR, XI, A, FR, FI) { const R t_ = XR[A]; \
  XR[A] = (FR) * t_ - (FI) * XI[A]; XI[A] = (FR) * XI[A] + (FI) * t_; }
// (PR, PI) *= (DR + i DI)
#define QS_CMUL(PR, PI, DR, DI) { const R t_ = PR * (DR) - PI * (DI); PI = PR * (DI) + PI * (DR); PR = t_; }
// Im(conj(l) w)
#define QS_IMC(LR, LI, WR, WI) ((double)(LR) * (double)(WI) - (double)(LI) * (double)(WR))
// Tile of workgroup b in a grid of one workgroup per tile: with order k,
// the tiles form 2^k contiguous regions and dispatch slot b takes tile
// b >> k of region b mod 2^k, so consecutive slots (which the dispatcher
// deals round-robin to the 8 XCDs) walk 2^k regions side by side; k = 0
// is the plain order, k = 3 gives each XCD its own eighth.  Tile counts are
// powers of two; any other grid walks the tiles in order.
__device__ __forceinline__ unsigned long long qs_tile_of(unsigned long long b, unsigned long long ntiles,
                                                         unsigned order) {
  if (order > 0 && order < 32 && (unsigned long long)gridDim.x == ntiles && (ntiles >> order) > 0 &&
      (ntiles & ((1ull << order) - 1ull)) == 0) {
    const unsigned long long per = ntiles >> order;
    return (b & ((1ull << order) - 1ull)) * per + (b >> order);
  }
  return b;
}
)";

// Tile-bit layout of one pass (the same values the interpreter receives in
// FusedArgs and FMapDev).
struct Geo {
  int dtype, nreg, RA, T, L, lane0, es;
  bool c64;
};

inline int swz(const Geo& g, int j) {
  return g.c64 ? (j ^ (((j >> 4) ^ (j >> 8) ^ (j >> 12)) & 15))
               : (j ^ (((j >> 3) ^ (j >> 6) ^ (j >> 9)) & 7));
}

// Byte offset in the remap buffer of register r's part of a tile position.
int regoff(const Geo& g, const FMap& m, int r) {
  int o = 0;
  for (int k = 0; k < g.nreg; ++k)
    if ((r >> k) & 1) o |= 1 << m.reg[k];
  return swz(g, o) * g.es;
}

class PassEmitter {
 public:
  PassEmitter(const Plan& plan, const Pass& p, int n, int dtype, bool adj)
      : plan_(plan), p_(p), n_(n), adj_(adj) {
    const FuseGeom G = plan.geom;
    g_.dtype = dtype;
    g_.nreg = G.nreg;
    g_.RA = 1 << G.nreg;
    g_.T = G.T;
    g_.L = G.L;
    g_.lane0 = G.lane0;
    g_.c64 = dtype == QS_C64;
    g_.es = g_.c64 ? 8 : 16;
  }

  // The kernel's definition, with kNamePlaceholder for its name; empty when
  // the pass has a shape this generator does not take (the interpreter runs
  // it then).
  std::string body() {
    if (!check()) return std::string();
    emit();
    return src_.s;
  }

 private:
  const Plan& plan_;
  const Pass& p_;
  int n_;
  bool adj_;
  Geo g_;
  Src src_;
  std::vector<int> thr_off_emitted_;

  int gq(int tb) const { return tb < g_.L ? tb : (int)p_.hpos[tb - g_.L]; }

  bool check() const {
    const FMap& ml = plan_.maps[p_.map_load];
    const FMap& ms = plan_.maps[p_.map_store];
    for (int i = 0; i < 6; ++i)
      if (ml.thr[i] != g_.lane0 + i || ms.thr[i] != g_.lane0 + i) return false;
    if (g_.c64 && (ml.reg[0] != 0 || ms.reg[0] != 0)) return false;
    if (p_.nh > 8 || p_.ngrad > kAdjMaxSlots) return false;
    for (int i = p_.op_first; i < p_.op_first + p_.nops; ++i) {
      const int k = plan_.ops[i].kind & 255;
      if (k != kOpRemap && k != kOpU && k != kOpDiag && k != kOpPhaseRun && k != kOpPhaseEntry)
        return false;
      if (adj_ && (k == kOpPhaseRun || k == kOpPhaseEntry)) return false;
    }
    return true;
  }

  // `var` = the global index base of tile `tilev`: the tile index with a 0
  // bit inserted at every high tile qubit, above the low qubits.
  void emit_base(const char* var, const char* tilev) {
    src_("    unsigned long long %s = %s << %d;", var, tilev, g_.L);
    for (int h = 0; h < p_.nh; ++h) {
      const int P = p_.hpos[h];
      src_("    %s = ((%s >> %d) << %d) | (%s & %lluull);", var, var, P, P + 1, var, (1ull << P) - 1ull);
    }
  }

  bool has_remap() const {
    for (int i = p_.op_first; i < p_.op_first + p_.nops; ++i)
      if ((plan_.ops[i].kind & 255) == kOpRemap) return true;
    return false;
  }

  // Uniform 64-bit offset (in amplitudes) of the wave bits of a mapping.
  std::string wave_part(const FMap& m) const {
    char b[160];
    snprintf(b, sizeof b, "(((unsigned long long)(wv & 1)) << %d) | (((unsigned long long)(wv >> 1)) << %d)",
             gq(m.thr[6]), gq(m.thr[7]));
    return b;
  }
  unsigned long long reg_part(const FMap& m, int r) const {
    unsigned long long o = 0;
    for (int k = 0; k < g_.nreg; ++k)
      if ((r >> k) & 1) o |= 1ull << gq(m.reg[k]);
    return o;
  }

  // Condition text for a thread-bit spec: lane bits per lane, wave bits
  // uniform.
  static std::string thread_bit(int i) {
    char b[64];
    if (i < 6)
      snprintf(b, sizeof b, "((lane >> %d) & 1)", i);
    else
      snprintf(b, sizeof b, "((wv >> %d) & 1)", i - 6);
    return b;
  }
  static std::string outside_bit(int q) {
    char b[64];
    snprintf(b, sizeof b, "((int)(base >> %d) & 1)", q);
    return b;
  }

  // Variable holding map m's swizzled byte offset of this thread's bits.
  std::string thr_off(int mi) {
    char name[32];
    snprintf(name, sizeof name, "to%d", mi);
    if (std::find(thr_off_emitted_.begin(), thr_off_emitted_.end(), mi) == thr_off_emitted_.end()) {
      thr_off_emitted_.push_back(mi);
      const FMap& m = plan_.maps[mi];
      std::string e = "0";
      for (int i = 0; i < 8; ++i) {
        char b[64];
        snprintf(b, sizeof b, " | (((tid >> %d) & 1) << %d)", i, (int)m.thr[i]);
        e += b;
      }
      src_("    const int %s = %s(%s) * %d;", name, g_.c64 ? "qs_swz64" : "qs_swz128", e.c_str(), g_.es);
    }
    return name;
  }

  // Offset, in 16-byte units, of this lane's bits under mapping m: the lane
  // index itself when the lanes hold the lowest unit bits (contiguous
  // 1 KiB per access), else each lane bit placed at its qubit.
  std::string lane_part(const FMap& m) const {
    const int sh = g_.c64 ? 1 : 0;  // unit bit = qubit - 1 at complex64
    bool plain = true;
    for (int i = 0; i < 6; ++i) plain &= gq(m.thr[i]) - sh == i;
    if (plain) return "(unsigned long long)lane";
    std::string e = "(0ull";
    for (int i = 0; i < 6; ++i) {
      char b[96];
      snprintf(b, sizeof b, " | ((unsigned long long)((lane >> %d) & 1) << %d)", i, gq(m.thr[i]) - sh);
      e += b;
    }
    return e + ")";
  }

  void emit_load(const char* XR, const char* XI, const char* ptr) {
    const FMap& m = plan_.maps[p_.map_load];
    src_("    {");
    src_("      const unsigned long long ub = base | %s;", wave_part(m).c_str());
    src_("      const unsigned long long lo_ = %s;", lane_part(m).c_str());
    if (!g_.c64) {
      src_("      const qs_d2* pa = %s + ub;", ptr);
      for (int r = 0; r < g_.RA; ++r) {
        src_("      { const qs_d2 v = __builtin_nontemporal_load(pa + %lluull + lo_); %s[%d] = v.x; %s[%d] = v.y; }",
             reg_part(m, r), XR, r, XI, r);
      }
    } else {
      src_("      const qs_f4* pa = %s + (ub >> 1);", ptr);
      for (int r = 0; r < g_.RA; r += 2) {
        src_("      { const qs_f4 v = __builtin_nontemporal_load(pa + %lluull + lo_); %s[%d] = v.x; %s[%d] = v.y; "
             "%s[%d] = v.z; %s[%d] = v.w; }",
             reg_part(m, r) >> 1, XR, r, XI, r, XR, r + 1, XI, r + 1);
      }
    }
    src_("    }");
  }

  void emit_store(const char* XR, const char* XI, const char* ptr) {
    const FMap& m = plan_.maps[p_.map_store];
    src_("    {");
    src_("      const unsigned long long ub = base | %s;", wave_part(m).c_str());
    src_("      const unsigned long long lo_ = %s;", lane_part(m).c_str());
    if (!g_.c64) {
      src_("      qs_d2* pa = %s + ub;", ptr);
      for (int r = 0; r < g_.RA; ++r)
        src_("      __builtin_nontemporal_store(qs_d2{%s[%d], %s[%d]}, pa + %lluull + lo_);", XR, r, XI, r,
             reg_part(m, r));
    } else {
      src_("      qs_f4* pa = %s + (ub >> 1);", ptr);
      for (int r = 0; r < g_.RA; r += 2)
        src_("      __builtin_nontemporal_store(qs_f4{%s[%d], %s[%d], %s[%d], %s[%d]}, pa + %lluull + lo_);", XR,
             r, XI, r, XR, r + 1, XI, r + 1, reg_part(m, r) >> 1);
    }
    src_("    }");
  }

  void emit_remap_tile(const char* XR, const char* XI, int mo, int mn) {
    const std::string to = thr_off(mo), tn = thr_off(mn);
    const char* VE = g_.c64 ? "qs_f2" : "qs_d2";
    src_("    {");
    for (int r = 0; r < g_.RA; ++r)
      src_("      *(%s*)(lb + (%s ^ %d)) = %s{%s[%d], %s[%d]};", VE, to.c_str(), regoff(g_, plan_.maps[mo], r), VE,
           XR, r, XI, r);
    src_("      __syncthreads();");
    for (int r = 0; r < g_.RA; ++r)
      src_("      { const %s v = *(const %s*)(lb + (%s ^ %d)); %s[%d] = v.x; %s[%d] = v.y; }", VE, VE, tn.c_str(),
           regoff(g_, plan_.maps[mn], r), XR, r, XI, r);
    src_("      __syncthreads();");
    src_("    }");
  }

  // Pairs (r, r | 2^k) whose register control bit (creg >= 0) is 1.
  void pairs(int k, int creg, std::vector<std::pair<int, int>>* out) const {
    for (int r = 0; r < g_.RA; ++r) {
      if (r & (1 << k)) continue;
      if (creg >= 0 && !((r >> creg) & 1)) continue;
      out->push_back({r, r | (1 << k)});
    }
  }

  // Coefficients c0..c3 of op i's matrix; `sel` (a lane condition) or
  // empty: lanes where it is 0 take the identity.
  void emit_coeffs(int i, bool real, const std::string& sel) {
    src_("      const double* m_ = %s->m;", opref(i).c_str());
    static const char* nm[8] = {"c0r", "c0i", "c1r", "c1i", "c2r", "c2i", "c3r", "c3i"};
    if (!sel.empty()) src_("      const bool on_ = %s;", sel.c_str());
    for (int e = 0; e < 8; ++e) {
      if (real && (e & 1)) continue;
      const char* id = (e == 0 || e == 6) ? "(R)1" : "(R)0";
      if (sel.empty()) {
        src_("      const R %s = (R)m_[%d];", nm[e], e);
      } else {
        // loaded first, then selected: a select around the load itself
        // becomes a branch per coefficient
        src_("      const R %s_ld = (R)m_[%d];", nm[e], e);
        src_("      const R %s = on_ ? %s_ld : %s;", nm[e], nm[e], id);
      }
    }
  }

  // The op record of op i as an SGPR pointer released one op ahead: the
  // empty asm keeps the compiler from hoisting every op's coefficient loads
  // to the top of the kernel (which runs out of scalar registers and spills
  // them into vector-register lanes), while still letting the next op's
  // loads overlap the current op's arithmetic.
  std::string opref(int i) const {
    char b[32];
    snprintf(b, sizeof b, "op%d_", i - p_.op_first);
    return b;
  }
  // Only the offset goes through the asm: the pointer stays derived from
  // the kernel's restrict, read-only `ops`, so its records are still read
  // with scalar loads (an opaque pointer would be read with vector loads
  // that queue behind the tile's).
  void release_op(int i) {
    if (i >= p_.op_first + p_.nops) return;
    const std::string r = opref(i);
    src_("    int %so = %d;", r.c_str(), i - p_.op_first);
    src_("    asm volatile(\"\" : \"+s\"(%so));", r.c_str());
    src_("    const QsOp* %s = ops + %so;", r.c_str(), r.c_str());
  }

  void emit_u(int i) {
    const FOp& op = plan_.ops[i];
    const int k = op.tgt;
    const int cw = op.ctl >> 8, ci = op.ctl & 255;
    const bool real = op.m[1] == 0.0 && op.m[3] == 0.0 && op.m[5] == 0.0 && op.m[7] == 0.0;
    const int pauli = (op.kind >> 8) & 255;
    src_("    {  // op %d: U on register bit %d, control %d/%d%s", i - p_.op_first, k, cw, ci, real ? ", real" : "");
    std::string cond, sel;
    if (cw == kInThread) (ci < 6 ? sel : cond) = thread_bit(ci);
    if (cw == kOutside) cond = outside_bit(ci);
    if (adj_ && op.aux >= 0) {
      // rotation (never controlled): Im<lambda|P|psi> before U^dagger
      std::vector<std::pair<int, int>> pr;
      pairs(k, -1, &pr);
      src_("      double g_ = 0.0;");
      for (auto& q : pr) {
        const int a = q.first, b = q.second;
        if (pauli == 1)  // X psi = (a1, a0)
          src_("      g_ += QS_IMC(yr[%d], yi[%d], xr[%d], xi[%d]) + QS_IMC(yr[%d], yi[%d], xr[%d], xi[%d]);", a, a, b,
               b, b, b, a, a);
        else  // Y psi = (-i a1, i a0)
          src_("      g_ += QS_IMC(yr[%d], yi[%d], xi[%d], -xr[%d]) + QS_IMC(yr[%d], yi[%d], -xi[%d], xr[%d]);", a,
               a, b, b, b, b, a, a);
      }
      emit_grad_store(op.aux);
    }
    if (!cond.empty()) src_("      if (%s) {", cond.c_str());
    emit_coeffs(i, real, sel);
    std::vector<std::pair<int, int>> pr;
    pairs(k, cw == kInReg ? ci : -1, &pr);
    for (auto& q : pr) {
      src_("      %s(xr, xi, %d, %d)", real ? "QS_UR" : "QS_U", q.first, q.second);
      if (adj_) src_("      %s(yr, yi, %d, %d)", real ? "QS_UR" : "QS_U", q.first, q.second);
    }
    if (!cond.empty()) src_("      }");
    src_("    }");
  }

  void emit_grad_store(int slot) {
    src_("      g_ = qs_row_sum16(g_);");
    src_("      if ((tid & 15) == 0) acc[%d + (tid >> 4)] += g_;", slot * 16);
  }

  // Registers r whose target / control conditions hold get factor (fr, fi);
  // which registers take d1 and which d0 follows the target spec.
  void emit_diag(int i) {
    const FOp& op = plan_.ops[i];
    const int tw = op.tgt >> 8, tix = op.tgt & 255;
    const int cw = op.ctl >> 8, ci = op.ctl & 255;
    const bool phase = op.m[0] == 1.0 && op.m[1] == 0.0;
    src_("    {  // op %d: diagonal, target %d/%d, control %d/%d%s", i - p_.op_first, tw, tix, cw, ci,
         phase ? ", phase" : "");
    src_("      const double* m_ = %s->m;", opref(i).c_str());
    if (adj_ && op.aux >= 0) {
      // RZ: Im<lambda|Z|psi>, sign by the target bit
      src_("      double g_ = 0.0;");
      if (tw == kInReg) {
        for (int r = 0; r < g_.RA; ++r)
          src_("      g_ %s= QS_IMC(yr[%d], yi[%d], xr[%d], xi[%d]);", ((r >> tix) & 1) ? "-" : "+", r, r, r, r);
      } else {
        src_("      {");
        src_("        double s_ = 0.0;");
        for (int r = 0; r < g_.RA; ++r) src_("        s_ += QS_IMC(yr[%d], yi[%d], xr[%d], xi[%d]);", r, r, r, r);
        src_("        g_ = %s ? -s_ : s_;", tw == kInThread ? thread_bit(tix).c_str() : outside_bit(tix).c_str());
        src_("      }");
      }
      emit_grad_store(op.aux);
    }
    std::string cond, csel;
    if (cw == kInThread) (ci < 6 ? csel : cond) = thread_bit(ci);
    if (cw == kOutside) cond = outside_bit(ci);
    const int creg = cw == kInReg ? ci : -1;
    if (tw == kOutside && phase) cond = cond.empty() ? outside_bit(tix) : cond + " && " + outside_bit(tix);
    if (!cond.empty()) src_("      if (%s) {", cond.c_str());
    src_("      const R d0r = (R)m_[0], d0i = (R)m_[1], d1r = (R)m_[6], d1i = (R)m_[7];");
    auto scale_regs = [&](const char* fr, const char* fi, int want_bit /* -1 any */) {
      for (int r = 0; r < g_.RA; ++r) {
        if (creg >= 0 && !((r >> creg) & 1)) continue;
        if (want_bit >= 0 && ((r >> tix) & 1) != want_bit) continue;
        src_("      QS_SC(xr, xi, %d, %s, %s)", r, fr, fi);
        if (adj_) src_("      QS_SC(yr, yi, %d, %s, %s)", r, fr, fi);
      }
    };
    if (tw == kInReg) {
      // per register: d1 where the target bit is 1, d0 (unless a phase) where 0
      if (csel.empty()) {
        scale_regs("d1r", "d1i", 1);
        if (!phase) scale_regs("d0r", "d0i", 0);
      } else {
        src_("      const bool on_ = %s;", csel.c_str());
        src_("      const R e1r = on_ ? d1r : (R)1, e1i = on_ ? d1i : (R)0;");
        scale_regs("e1r", "e1i", 1);
        if (!phase) {
          src_("      const R e0r = on_ ? d0r : (R)1, e0i = on_ ? d0i : (R)0;");
          scale_regs("e0r", "e0i", 0);
        }
      }
    } else {
      // one factor for the whole thread: the target bit is a thread bit or
      // lies outside the tile
      if (tw == kOutside && phase) {
        src_("      R fr_ = d1r, fi_ = d1i;");
      } else {
        const std::string b = tw == kInThread ? thread_bit(tix) : outside_bit(tix);
        src_("      R fr_ = %s ? d1r : d0r, fi_ = %s ? d1i : d0i;", b.c_str(), b.c_str());
      }
      if (!csel.empty()) {
        src_("      const bool on_ = %s;", csel.c_str());
        src_("      fr_ = on_ ? fr_ : (R)1; fi_ = on_ ? fi_ : (R)0;");
      }
      scale_regs("fr_", "fi_", -1);
    }
    if (!cond.empty()) src_("      }");
    src_("    }");
  }

  // Whether op i can join a diagonal block: a diagonal op whose control (if
  // any) is not a register bit, or a phase run (with its entries).
  bool block_op(int i) const {
    const int k = plan_.ops[i].kind & 255;
    if (k == kOpPhaseRun) return true;
    return k == kOpDiag && (plan_.ops[i].ctl >> 8) != kInReg;
  }
  // Index after op i (a phase run spans its entries).
  int op_next(int i) const {
    const FOp& op = plan_.ops[i];
    return (op.kind & 255) == kOpPhaseRun ? i + op.aux + 1 : i + 1;
  }
  // End of the diagonal block that starts at op i, and its number of ops.
  int diag_block_end(int i, int* count) const {
    int j = i, c = 0;
    while (j < p_.op_first + p_.nops && block_op(j)) {
      j = op_next(j);
      ++c;
    }
    *count = c;
    return j;
  }

  // The per-lane factor (pr, pi) of the phase run at op i: the product of
  // its entries' phases (explicit entries, the per-thread table and the
  // tile-index tables).
  void emit_run_factor(int i) {
    const FOp& h = plan_.ops[i];
    src_("      const QsOp* h_ = %s;", opref(i).c_str());
    if (h.m[4] != 0.0) {
      src_("      R pr = ttr%d, pi = tti%d;", i - p_.op_first, i - p_.op_first);
    } else {
      src_("      R pr = (R)1, pi = (R)0;");
    }
    for (int e = 1; e <= h.aux; ++e) {
      const FOp& en = plan_.ops[i + e];
      const int ew = en.ctl >> 8, eb = en.ctl & 255;
      src_("      {");
      src_("        const double* m_ = ops[%d].m;", i + e - p_.op_first);  // entries: read with the run
      if (ew == kNoBit) {
        src_("        const R fr = (R)m_[6], fi = (R)m_[7];");
      } else {
        const std::string b = ew == kInThread ? thread_bit(eb) : outside_bit(eb);
        src_("        const bool on_ = %s;", b.c_str());
        src_("        const R fr = on_ ? (R)m_[6] : (R)1, fi = on_ ? (R)m_[7] : (R)0;");
      }
      src_("        QS_CMUL(pr, pi, fr, fi)");
      src_("      }");
    }
    if (h.m[2] != 0.0) {
      src_("      {");
      src_("        const int lb_ = (int)h_->m[1];");
      src_("        const double* tlo = (const double*)(maps + (unsigned long long)h_->m[0]);");
      src_("        const double* thi = tlo + 2 * (1ull << lb_);");
      src_("        const unsigned long long lo = tix & ((1ull << lb_) - 1ull), hi = tix >> lb_;");
      src_("        QS_CMUL(pr, pi, (R)tlo[2 * lo], (R)tlo[2 * lo + 1])");
      src_("        QS_CMUL(pr, pi, (R)thi[2 * hi], (R)thi[2 * hi + 1])");
      src_("      }");
    }
  }

  // A block of diagonal ops [i0, i1) in one go.  Diagonal unitaries
  // commute, so the block's product is one factor per amplitude:
  //   F(r) = T * prod_k A_k[bit k of r],
  // T the product of the factors of ops whose target is a thread bit or
  // outside the tile (one value per lane), A_k[b] the product of the
  // factors on register bit k where that bit is b (a control on a thread
  // bit or outside the tile selects 1 where it is 0).  F is built over the
  // register bits as a product tree and each amplitude is scaled once.  In
  // the adjoint the gradient terms Im(conj(lambda_r) psi_r) are unchanged by
  // a diagonal unitary applied to both tiles, so they are formed once for
  // the block and each rotation's gradient is a signed sum of them.
  void emit_diag_block(int i0, int i1) {
    src_("    {  // ops %d-%d: diagonal block", i0 - p_.op_first, i1 - 1 - p_.op_first);
    bool grad = false, grad_thr = false, any_thr = false;
    for (int i = i0; i < i1; i = op_next(i)) {
      const FOp& op = plan_.ops[i];
      if ((op.tgt >> 8) != kInReg) any_thr = true;
      if (adj_ && (op.kind & 255) == kOpDiag && op.aux >= 0) {
        grad = true;
        if ((op.tgt >> 8) != kInReg) grad_thr = true;
      }
    }
    // complex64 keeps the terms (each costs four conversions to double);
    // complex128 forms them again per op (two instructions each), which
    // keeps fewer registers live
    const bool keep = g_.c64;
    auto term = [&](int r) {
      char b[96];
      if (keep)
        snprintf(b, sizeof b, "w%d_", r);
      else
        snprintf(b, sizeof b, "QS_IMC(yr[%d], yi[%d], xr[%d], xi[%d])", r, r, r, r);
      return std::string(b);
    };
    if (grad) {
      if (keep)
        for (int r = 0; r < g_.RA; ++r)
          src_("      const double w%d_ = QS_IMC(yr[%d], yi[%d], xr[%d], xi[%d]);", r, r, r, r, r);
      if (grad_thr) {
        src_("      double wt_ = 0.0;");
        for (int r = 0; r < g_.RA; ++r) src_("      wt_ += %s;", term(r).c_str());
      }
      for (int i = i0; i < i1; i = op_next(i)) {
        const FOp& op = plan_.ops[i];
        if ((op.kind & 255) != kOpDiag || op.aux < 0) continue;
        const int tw = op.tgt >> 8, tix = op.tgt & 255;
        src_("      {  // op %d: gradient, target %d/%d", i - p_.op_first, tw, tix);
        if (tw == kInReg) {
          src_("      double g_ = 0.0;");
          for (int r = 0; r < g_.RA; ++r) src_("      g_ %s= %s;", ((r >> tix) & 1) ? "-" : "+", term(r).c_str());
        } else {
          src_("      double g_ = %s ? -wt_ : wt_;",
               tw == kInThread ? thread_bit(tix).c_str() : outside_bit(tix).c_str());
        }
        emit_grad_store(op.aux);
        src_("      }");
      }
    }
    // T and the per-register-bit products
    if (any_thr) src_("      R tr_, ti_;");
    bool t_one = true;                     // T still 1
    std::vector<int> a1_one(g_.nreg, 1);   // A_k[1] still 1
    std::vector<int> a0_one(g_.nreg, 1);   // A_k[0] still 1
    // multiply (vr, vi) into factor `name` (declared on first use)
    auto mul_into = [&](const std::string& name, bool* one, const std::string& vr, const std::string& vi) {
      if (*one)
        src_("      R %sr = %s, %si = %s;", name.c_str(), vr.c_str(), name.c_str(), vi.c_str());
      else
        src_("      QS_CMUL(%sr, %si, %s, %s)", name.c_str(), name.c_str(), vr.c_str(), vi.c_str());
      *one = false;
    };
    for (int i = i0; i < i1; i = op_next(i)) {
      const FOp& op = plan_.ops[i];
      const int j = i - p_.op_first;
      const int tw = op.tgt >> 8, tix = op.tgt & 255;
      std::string f1r, f1i, f0r, f0i;  // factor where the target bit is 1 / 0 (empty: 1)
      std::string on;                  // control condition (empty: none)
      if ((op.kind & 255) == kOpPhaseRun) {
        src_("      R p%dr, p%di;", j, j);
        src_("      {  // op %d: phase run of %d explicit entries, target %d/%d", j, op.aux, tw, tix);
        emit_run_factor(i);
        src_("      p%dr = pr; p%di = pi;", j, j);
        src_("      }");
        f1r = "p" + std::to_string(j) + "r";
        f1i = "p" + std::to_string(j) + "i";
      } else {
        const int cw = op.ctl >> 8, ci = op.ctl & 255;
        const bool phase = op.m[0] == 1.0 && op.m[1] == 0.0;
        src_("      const double* m%d_ = %s->m;  // op %d: diagonal, target %d/%d, control %d/%d%s", j,
             opref(i).c_str(), j, tw, tix, cw, ci, phase ? ", phase" : "");
        char b[64];
        snprintf(b, sizeof b, "(R)m%d_[6]", j);
        f1r = b;
        snprintf(b, sizeof b, "(R)m%d_[7]", j);
        f1i = b;
        if (!phase) {
          snprintf(b, sizeof b, "(R)m%d_[0]", j);
          f0r = b;
          snprintf(b, sizeof b, "(R)m%d_[1]", j);
          f0i = b;
        }
        if (cw != kNoBit) on = cw == kInThread ? thread_bit(ci) : outside_bit(ci);
      }
      if (tw == kInReg) {
        auto put = [&](int bit, const std::string& fr, const std::string& fi) {
          if (fr.empty()) return;
          char nm[16];
          snprintf(nm, sizeof nm, "a%d%d", tix, bit);
          std::vector<int>& one = bit ? a1_one : a0_one;
          bool o = one[tix];
          if (on.empty()) {
            mul_into(nm, &o, fr, fi);
          } else {
            src_("      const bool c%d%d_ = %s;", j, bit, on.c_str());
            char sr[96], si[96];
            snprintf(sr, sizeof sr, "(c%d%d_ ? %s : (R)1)", j, bit, fr.c_str());
            snprintf(si, sizeof si, "(c%d%d_ ? %s : (R)0)", j, bit, fi.c_str());
            mul_into(nm, &o, sr, si);
          }
          one[tix] = o;
        };
        put(1, f1r, f1i);
        put(0, f0r, f0i);
      } else {
        const std::string tb = tw == kInThread ? thread_bit(tix) : outside_bit(tix);
        src_("      {");
        src_("        const bool s_ = %s;", tb.c_str());
        std::string c = on.empty() ? "" : on;
        const std::string fr0 = f0r.empty() ? "(R)1" : f0r, fi0 = f0i.empty() ? "(R)0" : f0i;
        if (c.empty()) {
          src_("        const R fr_ = s_ ? %s : %s, fi_ = s_ ? %s : %s;", f1r.c_str(), fr0.c_str(), f1i.c_str(),
               fi0.c_str());
        } else {
          src_("        const bool on_ = %s;", c.c_str());
          src_("        const R fr_ = on_ ? (s_ ? %s : %s) : (R)1, fi_ = on_ ? (s_ ? %s : %s) : (R)0;", f1r.c_str(),
               fr0.c_str(), f1i.c_str(), fi0.c_str());
        }
        if (t_one)
          src_("        tr_ = fr_; ti_ = fi_;");
        else
          src_("        QS_CMUL(tr_, ti_, fr_, fi_)");
        src_("      }");
        t_one = false;
      }
    }
    // F over the registers: level k doubles the list with A_k
    std::vector<std::string> fr(1, t_one ? "" : "tr_"), fi(1, t_one ? "" : "ti_");
    int nf = 0;
    for (int k = 0; k < g_.nreg; ++k) {
      const int m = (int)fr.size();
      std::vector<std::string> nr(2 * m), ni(2 * m);
      for (int r = 0; r < m; ++r)
        for (int bb = 0; bb < 2; ++bb) {
          const int o = r + bb * m;
          const bool a_one = bb ? a1_one[k] : a0_one[k];
          char ar[16], ai[16];
          snprintf(ar, sizeof ar, "a%d%dr", k, bb);
          snprintf(ai, sizeof ai, "a%d%di", k, bb);
          if (a_one) {
            nr[o] = fr[r];
            ni[o] = fi[r];
          } else if (fr[r].empty()) {
            nr[o] = ar;
            ni[o] = ai;
          } else {
            char v[16];
            snprintf(v, sizeof v, "f%d", nf++);
            src_("      const R %sr = %s * %s - %s * %s, %si = %s * %s + %s * %s;", v, fr[r].c_str(), ar,
                 fi[r].c_str(), ai, v, fr[r].c_str(), ai, fi[r].c_str(), ar);
            nr[o] = std::string(v) + "r";
            ni[o] = std::string(v) + "i";
          }
        }
      fr.swap(nr);
      fi.swap(ni);
    }
    // entry r + b * 2^k of level k: register bit k of r is b
    for (int r = 0; r < g_.RA; ++r) {
      if (fr[r].empty()) continue;
      src_("      QS_SC(xr, xi, %d, %s, %s)", r, fr[r].c_str(), fi[r].c_str());
      if (adj_) src_("      QS_SC(yr, yi, %d, %s, %s)", r, fr[r].c_str(), fi[r].c_str());
    }
    src_("    }");
  }

  // A phase run (forward passes only): per-lane product of the run's
  // phases, then the target-bit-1 amplitudes scaled once.
  int emit_run(int i) {
    const FOp& h = plan_.ops[i];
    const int tw = h.tgt >> 8, tix = h.tgt & 255;
    src_("    {  // op %d: phase run of %d explicit entries, target %d/%d", i - p_.op_first, h.aux, tw, tix);
    emit_run_factor(i);
    if (tw == kInReg) {
      for (int r = 0; r < g_.RA; ++r)
        if ((r >> tix) & 1) src_("      QS_SC(xr, xi, %d, pr, pi)", r);
    } else if (tw == kInThread && tix < 6) {
      src_("      const bool b_ = %s;", thread_bit(tix).c_str());
      src_("      const R fr_ = b_ ? pr : (R)1, fi_ = b_ ? pi : (R)0;");
      for (int r = 0; r < g_.RA; ++r) src_("      QS_SC(xr, xi, %d, fr_, fi_)", r);
    } else {
      const std::string b = tw == kInThread ? thread_bit(tix) : outside_bit(tix);
      src_("      if (%s) {", b.c_str());
      for (int r = 0; r < g_.RA; ++r) src_("        QS_SC(xr, xi, %d, pr, pi)", r);
      src_("      }");
    }
    src_("    }");
    return h.aux;
  }

  void emit() {
    const char* VT = g_.c64 ? "qs_f4" : "qs_d2";
    // Adjoint passes hold two tiles and a 32 KiB remap buffer plus the
    // gradient slots, so LDS admits four workgroups per CU; without a hint
    // the compiler spends registers down to two or three waves per SIMD.
    // Four (128 registers, a few spilled) measured faster at both dtypes.
    src_.s += "extern \"C\" __global__ void __launch_bounds__(256) ";
    if (adj_) src_.s += "__attribute__((amdgpu_waves_per_eu(4))) ";
    src_.s += kNamePlaceholder;
    if (adj_)
      src_("(%s* __restrict__ qa, %s* __restrict__ ql, const QsOp* __restrict__ ops, const char* __restrict__ maps, "
           "double* __restrict__ part, unsigned long long ntiles, unsigned order) {",
           VT, VT);
    else
      src_("(%s* __restrict__ qa, const QsOp* __restrict__ ops, const char* __restrict__ maps, "
           "unsigned long long ntiles, unsigned order) {",
           VT);
    src_("  typedef %s R;", g_.c64 ? "float" : "double");
    src_("  const int tid = threadIdx.x;");
    src_("  const int lane = tid & 63;");
    src_("  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);");
    const bool remaps = has_remap();
    if (remaps) {
      src_("  __shared__ %s lds[%d];", g_.c64 ? "qs_f2" : "qs_d2", g_.RA * 256);
      src_("  char* lb = (char*)lds;");
    }
    const int ngrad = adj_ ? p_.ngrad : 0;
    if (ngrad > 0) {
      src_("  __shared__ double acc[%d];", ngrad * 16);
      src_("  for (int i = tid; i < %d; i += 256) acc[i] = 0.0;", ngrad * 16);
      src_("  __syncthreads();");
    }
    src_("  R xr[%d], xi[%d];", g_.RA, g_.RA);
    if (adj_) src_("  R yr[%d], yi[%d];", g_.RA, g_.RA);
    src_("  for (unsigned long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {");
    src_("    const unsigned long long tix = qs_tile_of(tile, ntiles, order);");
    emit_base("base", "tix");
    // per-thread phase-run tables: read before this iteration's tile loads
    // so that waiting for them never waits for the tile
    for (int i = p_.op_first; i < p_.op_first + p_.nops; ++i) {
      const FOp& op = plan_.ops[i];
      if ((op.kind & 255) != kOpPhaseRun) continue;
      if (op.m[4] != 0.0) {
        const int j = i - p_.op_first;
        src_("    const double* tt%d = (const double*)(maps + (unsigned long long)ops[%d].m[3]);", j, j);
        src_("    const R ttr%d = (R)tt%d[2 * tid], tti%d = (R)tt%d[2 * tid + 1];", j, j, j, j);
      }
      i += op.aux;
    }
    emit_load("xr", "xi", "qa");
    if (adj_) emit_load("yr", "yi", "ql");
    // op records: op i's pointer is released at the start of op i - 1
    int released = p_.op_first;
    auto release_upto = [&](int last) {
      for (; released <= last && released < p_.op_first + p_.nops; ++released) {
        const int k = plan_.ops[released].kind & 255;
        if (k == kOpU || k == kOpDiag || k == kOpPhaseRun) release_op(released);
      }
    };
    for (int i = p_.op_first; i < p_.op_first + p_.nops; ++i) {
      const FOp& op = plan_.ops[i];
      const int kind = op.kind & 255;
      // a block of two or more diagonal ops is emitted as one
      int nblk = 0;
      const int blk_end = block_op(i) ? diag_block_end(i, &nblk) : i + 1;
      const bool blk = nblk >= 2;
      const int next = blk ? blk_end : kind == kOpPhaseRun ? i + op.aux + 1 : i + 1;
      release_upto(blk ? blk_end - 1 : i);
      // the next op that reads a record
      for (int j = next; j < p_.op_first + p_.nops; ++j) {
        const int k = plan_.ops[j].kind & 255;
        if (k == kOpU || k == kOpDiag || k == kOpPhaseRun) {
          release_upto(j);
          break;
        }
        if (k == kOpPhaseEntry) continue;
      }
      if (kind == kOpRemap) {
        src_("    // op %d: remap %d -> %d", i - p_.op_first, op.aux, op.tgt);
        emit_remap_tile("xr", "xi", op.aux, op.tgt);
        if (adj_) emit_remap_tile("yr", "yi", op.aux, op.tgt);
      } else if (kind == kOpU) {
        emit_u(i);
      } else if (blk) {
        emit_diag_block(i, blk_end);
        i = blk_end - 1;
      } else if (kind == kOpDiag) {
        emit_diag(i);
      } else if (kind == kOpPhaseRun) {
        i += emit_run(i);
      }
    }
    emit_store("xr", "xi", "qa");
    if (adj_) emit_store("yr", "yi", "ql");
    src_("  }");
    if (ngrad > 0) {
      src_("  __syncthreads();");
      src_("  if (tid < %d) {", ngrad);
      src_("    double s = 0.0;");
      src_("    for (int r = 0; r < 16; ++r) s += acc[tid * 16 + r];");
      // indexed by tile, so that the sum over partials is the same in either
      // tile order
      src_("    part[(unsigned long long)tid * gridDim.x + qs_tile_of(blockIdx.x, ntiles, order)] = s;");
      src_("  }");
    }
    src_("}");
  }
};

// ------------------------------------------------------------ cache

struct JitProgram {
  std::string code;                  // code object
  std::vector<hipModule_t> modules;  // per device (null until loaded)
  std::string file;                  // its file in the on-disk cache, when loaded from there
};
struct JitEntry {
  int program = -1;
  std::string name;
  std::vector<hipFunction_t> fn;  // per device
};

std::mutex g_mu;
std::unordered_map<std::string, int> g_index;  // kernel text -> entry
std::vector<JitEntry> g_entries;
std::vector<JitProgram> g_programs;
JitStats g_stats;

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 1469598103934665603ull;
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

// ------------------------------------------------------- on-disk cache
// With QS_JIT_CACHE_DIR set, every compiled program is also written there
// (p_<hash>.co) with, per kernel, its text (k_<hash>.txt, compared in full on
// lookup) and the program that holds it (k_<hash>.prog), so that other
// processes load instead of compiling.
std::string cache_dir() {
  const char* e = getenv("QS_JIT_CACHE_DIR");
  return e ? std::string(e) : std::string();
}

bool read_file(const std::string& path, std::string* out) {
  std::ifstream f(path, std::ios::binary);
  if (!f) return false;
  std::ostringstream ss;
  ss << f.rdbuf();
  *out = ss.str();
  return true;
}

void write_file(const std::string& path, const std::string& data) {
  const std::string tmp = path + ".tmp" + std::to_string((unsigned long long)std::hash<std::thread::id>()(std::this_thread::get_id()));
  {
    std::ofstream f(tmp, std::ios::binary);
    if (!f) return;
    f.write(data.data(), (std::streamsize)data.size());
    if (!f) return;
  }
  std::rename(tmp.c_str(), path.c_str());
}

std::string hex64(uint64_t h) {
  char b[20];
  snprintf(b, sizeof b, "%016llx", (unsigned long long)h);
  return b;
}

struct CompileJob {
  std::vector<std::pair<std::string, std::string>> kernels;  // (name, text)
  std::string code, error;
  double seconds = 0.0;
  bool by_clang = false;  // compiled in a child clang process (else hipRTC)
};

// The ROCm clang driver, for compiling in child processes (hipRTC
// serialises compilations inside one process); empty when not found or
// when QS_JIT_COMPILER=hiprtc.
std::string clang_path() {
  const char* mode = getenv("QS_JIT_COMPILER");
  if (mode && !strcmp(mode, "hiprtc")) return std::string();
  std::vector<std::string> cands;
  if (const char* e = getenv("QS_JIT_CLANG")) cands.push_back(e);
  if (const char* r = getenv("ROCM_PATH")) cands.push_back(std::string(r) + "/llvm/bin/clang++");
  cands.push_back("/opt/rocm/llvm/bin/clang++");
  for (const std::string& c : cands)
    if (!c.empty() && access(c.c_str(), X_OK) == 0) return c;
  return std::string();
}

// Compile `src` with the clang driver in a child process into a code
// object; false (with job->error set) if anything fails.
bool compile_with_clang(const std::string& clang, const std::string& src, CompileJob* job) {
  const char* td = getenv("TMPDIR");
  std::string dir = std::string(td && *td ? td : "/tmp") + "/qsjitXXXXXX";
  if (!mkdtemp(&dir[0])) {
    job->error = "mkdtemp failed";
    return false;
  }
  const std::string in = dir + "/pass.hip", out = dir + "/pass.hsaco";
  {
    std::ofstream f(in, std::ios::binary);
    f << src;
    if (!f) {
      job->error = "cannot write " + in;
      rmdir(dir.c_str());
      return false;
    }
  }
  std::string rocm = clang.substr(0, clang.rfind("/llvm/bin/"));
  const std::string rocm_arg = "--rocm-path=" + (rocm.empty() ? std::string("/opt/rocm") : rocm);
  std::vector<std::string> args = {clang, "-x", "hip", "-std=c++17", "--offload-arch=gfx950", "--cuda-device-only",
                                   "--no-gpu-bundle-output", "-O3", "-ffp-contract=fast", "-Xclang",
                                   "-target-feature", "-Xclang", "-packed-fp32-ops", rocm_arg, "-include",
                                   "hip/hip_runtime.h", "-w", in, "-o", out};
  std::vector<char*> argv;
  for (auto& a : args) argv.push_back(&a[0]);
  argv.push_back(nullptr);
  posix_spawn_file_actions_t fa;
  posix_spawn_file_actions_init(&fa);
  const std::string log = dir + "/log.txt";
  posix_spawn_file_actions_addopen(&fa, 1, log.c_str(), O_WRONLY | O_CREAT | O_TRUNC, 0600);
  posix_spawn_file_actions_adddup2(&fa, 1, 2);
  pid_t pid = 0;
  const int rc = posix_spawn(&pid, clang.c_str(), &fa, nullptr, argv.data(), environ);
  posix_spawn_file_actions_destroy(&fa);
  // wait for the child, at most kClangSeconds (a compile of one program
  // takes seconds; a stuck one is killed and the job falls back to hipRTC)
  constexpr int kClangSeconds = 300;
  int status = 0;
  bool exited = false;
  if (rc == 0) {
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::seconds(kClangSeconds);
    for (;;) {
      const pid_t w = waitpid(pid, &status, WNOHANG);
      if (w == pid) {
        exited = true;
        break;
      }
      if (w < 0) break;
      if (std::chrono::steady_clock::now() > deadline) {
        kill(pid, SIGKILL);
        waitpid(pid, &status, 0);
        break;
      }
      std::this_thread::sleep_for(std::chrono::milliseconds(5));
    }
  }
  bool ok = exited && WIFEXITED(status) && WEXITSTATUS(status) == 0 && read_file(out, &job->code) &&
            !job->code.empty();
  if (!ok) {
    std::string msg;
    read_file(log, &msg);
    if (msg.size() > 2000) msg.resize(2000);
    job->error = "clang (" + clang + ") failed: " + msg;
    job->code.clear();
  }
  unlink(in.c_str());
  unlink(out.c_str());
  unlink(log.c_str());
  rmdir(dir.c_str());
  return ok;
}

void compile_job(CompileJob* job) {
  const auto t0 = std::chrono::steady_clock::now();
  std::string src = kPrelude;
  for (auto& k : job->kernels) {
    // the text names its kernel kNamePlaceholder
    const size_t at = k.second.find(kNamePlaceholder);
    src += k.second.substr(0, at);
    src += k.first;
    src += k.second.substr(at + strlen(kNamePlaceholder));
  }
  const char* dump = getenv("QS_JIT_DUMP");
  if (dump && *dump) {
    std::ofstream(std::string(dump) + "/" + job->kernels[0].first + ".hip") << src;
  }
  const std::string clang = clang_path();
  if (!clang.empty()) {
    if (compile_with_clang(clang, src, job)) {
      job->by_clang = true;
      if (dump && *dump)
        std::ofstream(std::string(dump) + "/" + job->kernels[0].first + ".co", std::ios::binary)
            .write(job->code.data(), (std::streamsize)job->code.size());
      job->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      return;
    }
    job->error.clear();  // fall back to hipRTC
  }
  hiprtcProgram prog;
  hiprtcResult r = hiprtcCreateProgram(&prog, src.c_str(), "qs_pass.hip", 0, nullptr, nullptr);
  if (r != HIPRTC_SUCCESS) {
    job->error = std::string("hiprtcCreateProgram: ") + hiprtcGetErrorString(r);
    return;
  }
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-ffp-contract=fast", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops"};
  r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (r != HIPRTC_SUCCESS) {
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    std::string log(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    if (log.size() > 2000) log.resize(2000);
    job->error = std::string("hiprtcCompileProgram: ") + hiprtcGetErrorString(r) + "\n" + log;
    hiprtcDestroyProgram(&prog);
    return;
  }
  size_t sz = 0;
  hiprtcGetCodeSize(prog, &sz);
  job->code.resize(sz);
  hiprtcGetCode(prog, &job->code[0]);
  hiprtcDestroyProgram(&prog);
  if (dump && *dump) {
    std::ofstream(std::string(dump) + "/" + job->kernels[0].first + ".co", std::ios::binary)
        .write(job->code.data(), (std::streamsize)job->code.size());
  }
  job->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int compile_threads() {
  const char* e = getenv("QS_JIT_THREADS");
  int t = e ? atoi(e) : 0;
  if (t <= 0) t = (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(t, 16));
}

// Make sure every text in `texts` has a cache entry (compiling the missing
// ones); entry indices into *idx.
Status ensure_compiled(const std::vector<std::string>& texts, std::vector<int>* idx) {
  std::vector<std::string> missing;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    for (const std::string& t : texts)
      if (!g_index.count(t) && std::find(missing.begin(), missing.end(), t) == missing.end())
        missing.push_back(t);
  }
  const std::string dir = cache_dir();
  if (!dir.empty() && !missing.empty()) {
    // kernels another process compiled: load their programs
    std::vector<std::string> still;
    std::lock_guard<std::mutex> lk(g_mu);
    for (const std::string& t : missing) {
      const std::string h = hex64(fnv1a(t));
      std::string txt, prog, code;
      if (!read_file(dir + "/k_" + h + ".txt", &txt) || txt != t || !read_file(dir + "/k_" + h + ".prog", &prog) ||
          !read_file(dir + "/" + prog, &code) || code.empty()) {
        still.push_back(t);
        continue;
      }
      int pi = -1;
      for (size_t i = 0; i < g_programs.size(); ++i)
        if (g_programs[i].file == prog) pi = (int)i;
      if (pi < 0) {
        pi = (int)g_programs.size();
        g_programs.push_back(JitProgram{std::move(code), {}, prog});
      }
      JitEntry e;
      e.program = pi;
      e.name = "qs_pass_" + h;
      g_index[t] = (int)g_entries.size();
      g_entries.push_back(std::move(e));
      ++g_stats.loaded_from_disk;
    }
    missing.swap(still);
  }
  if (!missing.empty()) {
    const auto t0 = std::chrono::steady_clock::now();
    const int nthreads = std::min<int>(compile_threads(), (int)missing.size());
    std::vector<CompileJob> jobs((size_t)nthreads);
    for (size_t i = 0; i < missing.size(); ++i) {
      char name[48];
      snprintf(name, sizeof name, "qs_pass_%016llx", (unsigned long long)fnv1a(missing[i]));
      jobs[i % (size_t)nthreads].kernels.push_back({name, missing[i]});
    }
    std::vector<std::thread> th;
    for (int j = 1; j < nthreads; ++j) th.emplace_back(compile_job, &jobs[(size_t)j]);
    compile_job(&jobs[0]);
    for (auto& t : th) t.join();
    for (auto& j : jobs)
      if (!j.error.empty()) return Status{QS_EHIP, "fused-pass compile failed: " + j.error};
    if (!dir.empty()) {
      for (auto& j : jobs) {
        std::string all;
        for (auto& k : j.kernels) all += k.second;
        const std::string prog = "p_" + hex64(fnv1a(all)) + ".co";
        write_file(dir + "/" + prog, j.code);
        for (auto& k : j.kernels) {
          const std::string h = hex64(fnv1a(k.second));
          write_file(dir + "/k_" + h + ".txt", k.second);
          write_file(dir + "/k_" + h + ".prog", prog);
        }
      }
    }
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& j : jobs) {
      const int pi = (int)g_programs.size();
      g_programs.push_back(JitProgram{std::move(j.code), {}, std::string()});
      for (auto& k : j.kernels) {
        if (g_index.count(k.second)) continue;
        JitEntry e;
        e.program = pi;
        e.name = k.first;
        g_index[k.second] = (int)g_entries.size();
        g_entries.push_back(std::move(e));
      }
    }
    g_stats.kernels += (long long)missing.size();
    for (auto& j : jobs) (j.by_clang ? g_stats.programs_clang : g_stats.programs_hiprtc) += 1;
    g_stats.compile_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  std::lock_guard<std::mutex> lk(g_mu);
  idx->clear();
  for (const std::string& t : texts) idx->push_back(g_index.at(t));
  return Status::ok();
}

Status function_on(int entry, int dev, hipFunction_t* out) {
  std::lock_guard<std::mutex> lk(g_mu);
  JitEntry& e = g_entries[(size_t)entry];
  if ((int)e.fn.size() <= dev) e.fn.resize((size_t)dev + 1, nullptr);
  if (!e.fn[(size_t)dev]) {
    JitProgram& p = g_programs[(size_t)e.program];
    if ((int)p.modules.size() <= dev) p.modules.resize((size_t)dev + 1, nullptr);
    if (!p.modules[(size_t)dev]) {
      hipModule_t m = nullptr;
      hipError_t err = hipModuleLoadData(&m, p.code.data());
      if (err != hipSuccess) return hip_status(err, "load fused-pass module");
      p.modules[(size_t)dev] = m;
      ++g_stats.modules_loaded;
    }
    hipFunction_t f = nullptr;
    hipError_t err = hipModuleGetFunction(&f, p.modules[(size_t)dev], e.name.c_str());
    if (err != hipSuccess) return hip_status(err, "fused-pass kernel lookup");
    e.fn[(size_t)dev] = f;
  }
  *out = e.fn[(size_t)dev];
  return Status::ok();
}

}  // namespace

std::string jit_pass_text(const Plan& plan, const Pass& p, int n, int dtype, bool adjoint) {
  PassEmitter em(plan, p, n, dtype, adjoint);
  return em.body();
}

Status jit_prepare(const Plan& plan, int n, int dtype, bool adjoint, std::vector<JitPass>* out) {
  out->assign(plan.passes.size(), JitPass{});
  std::vector<std::string> texts;
  std::vector<int> which;
  for (size_t i = 0; i < plan.passes.size(); ++i) {
    if (plan.passes[i].kind != kPassFused) continue;
    std::string t = jit_pass_text(plan, plan.passes[i], n, dtype, adjoint);
    if (t.empty()) continue;
    texts.push_back(std::move(t));
    which.push_back((int)i);
  }
  std::vector<int> idx;
  Status st = ensure_compiled(texts, &idx);
  if (!st.good()) return st;
  for (size_t j = 0; j < which.size(); ++j) (*out)[(size_t)which[j]].entry = idx[j];
  return Status::ok();
}

Status jit_function(const JitPass& jp, int device, hipFunction_t* fn) {
  if (jp.entry < 0) return Status{QS_EINVAL, "pass has no compiled kernel"};
  return function_on(jp.entry, device, fn);
}

JitStats jit_stats() {
  std::lock_guard<std::mutex> lk(g_mu);
  JitStats s = g_stats;
  s.cached = (long long)g_entries.size();
  return s;
}

}  // namespace qs
