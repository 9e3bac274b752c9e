// C ABI and executor of the temporal-boundary contraction (include/tnc.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/tnc.h"
#include "exec.hpp"
#include "kernels.hpp"
#include "late.hpp"
#include "plan.hpp"

struct tnc_plan_s {
  std::unique_ptr<tnc::Plan> plan;
};

namespace tnc {

thread_local std::string g_err;

// The calling thread's last error message (also used by the serving loop).
int set_error_message(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

namespace {

int set_err(int code, const std::string& msg) { return set_error_message(code, msg); }

int hip_err(hipError_t e, const char* what) {
  return set_err(TNC_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Host copies of a schedule's device tables.
struct PassHost {
  int phase_off = 0, n_phases = 0;
  int op_begin = 0, op_end = 0;
  Window w;
  int R = 5;
};

struct HostTables {
  std::vector<DevOp> ops;
  std::vector<float> mats;
  std::vector<DevPhase> phases;
  std::vector<uint32_t> poffs;  // kPhaseOffs per phase
  std::vector<float4> fmats;    // kFusedWords per phase (fused phases only; empty without them)
  std::vector<PassHost> passes;
  std::vector<double2> seg;
  LatePlan late;
  std::vector<LateOpDev> prog;
  uint64_t bytes_late[2] = {0, 0};
};

// FP32 form of an update matrix K (FP64), 8 floats (re, im) row-major.
// Every update acts on the whole boundary tensor, so a rounding bias shared
// by a matrix's entries multiplies every amplitude: 1/sqrt(2) rounds to
// nearest 1.7e-8 low, and the ~900 Hadamard-like factors of a width-33
// sweep would scale every amplitude by 1 - 1.5e-5.  Each component is
// therefore rounded down or up (the two FP32 neighbours of its value).
// rho - 1 = <K, K32> / <K, K> - 1, the least-squares factor's deviation, is
// a sum of one term per component, so the components are taken in turn and
// each picks the neighbour that brings the running sum `acc` (rho - 1 of
// the sweep's earlier updates, plus this matrix's terms so far) closer to
// zero: error diffusion over the sweep.  Returns this matrix's rho - 1.
cd round_entries(const cd* K, int n, const cd& acc, float* out) {
  double nk = 0;
  for (int e = 0; e < n; ++e) nk += std::norm(K[e]);
  cd run = acc, rho = 0;
  for (int q = 0; q < 2 * n; ++q) {
    const cd ke = K[q >> 1];
    const double v = (q & 1) ? ke.imag() : ke.real();
    const float f = (float)v;
    out[q] = f;
    if ((double)f == v || nk == 0) continue;
    const float g = std::nextafter(f, (double)f < v ? INFINITY : -INFINITY);
    // term of component q: conj(K_e) (x - v) (1 or i) / <K, K>
    const cd w = std::conj(ke) * ((q & 1) ? cd(0, 1) : cd(1, 0)) / nk;
    const cd tf = w * ((double)f - v), tg = w * ((double)g - v);
    const bool up = std::abs(run + tg) < std::abs(run + tf);
    out[q] = up ? g : f;
    run += up ? tg : tf;
    rho += up ? tg : tf;
  }
  return rho;
}

cd round_matrix(const M2& K, const cd& acc, float* out) { return round_entries(K.a, 4, acc, out); }

// A fused phase's three updates as one complex 8x8 U_c per value c of op 0's
// control, on entry index e = b0 + 2 b1 + 4 b2 (b0, b1, b2 = the targets of
// ops 0, 1, 2; op 1 is controlled by b0, op 2 by b1).  U[e' * 8 + e].
void fused_matrix(const SweepOp* op, int c, cd* U) {
  for (int e = 0; e < 8; ++e) {
    cd z[8] = {};
    z[e] = 1;
    auto apply = [&](int bit, const M2& m0, const M2& m1, int cbit) {
      for (int i = 0; i < 8; ++i) {
        if (i >> bit & 1) continue;
        const int j = i | (1 << bit);
        const M2& m = (cbit >= 0 && (i >> cbit & 1)) ? m1 : m0;
        const cd a0 = z[i], a1 = z[j];
        z[i] = m.a[0] * a0 + m.a[1] * a1;
        z[j] = m.a[2] * a0 + m.a[3] * a1;
      }
    };
    apply(0, op[0].mat[0][c], op[0].mat[0][c], -1);
    apply(1, op[1].mat[0][0], op[1].mat[0][1], 0);
    apply(2, op[2].mat[0][0], op[2].mat[0][1], 1);
    for (int eo = 0; eo < 8; ++eo) U[eo * 8 + e] = z[eo];
  }
}

// A bond-four unit's two 4x4s (A on (b0, b1), then B on (b1, b2); ops
// op[0..1] and op[2..3], variant 0) as one complex 8x8 on entry index
// e = b0 + 2 b1 + 4 b2.  U[e' * 8 + e].
void unit_matrix(const SweepOp* op, cd* U) {
  auto m4 = [&](int k, int r, int c) { return (r < 2 ? op[k] : op[k + 1]).mat[0][r & 1].a[c]; };
  for (int e = 0; e < 8; ++e) {
    cd z[8] = {};
    z[e] = 1;
    for (int k = 0; k < 4; k += 2) {
      const int lo = k == 0 ? 0 : 1;  // A on bits (0, 1), B on bits (1, 2)
      cd w[8] = {};
      for (int i = 0; i < 8; ++i) {
        const int u = ((i >> lo) & 3);
        const int rest = i & ~(3 << lo);
        for (int o = 0; o < 4; ++o) w[rest | (o << lo)] += m4(k, o, u) * z[i];
      }
      std::copy(w, w + 8, z);
    }
    for (int eo = 0; eo < 8; ++eo) U[eo * 8 + e] = z[eo];
  }
}

// Matrix-core operand of a fused phase for one control value: lane l holds,
// at MFMA step s, A[l % 16][4 s + l / 16] of the real 16x16 form of U32.
// Real index 4 g + t (rows) / 4 t + g (columns) stands for entry
// e = 2 g + (t >> 1), component t & 1 (re, im), so lane group g = l / 16
// keeps entries 2g and 2g + 1 from input to output.
void fused_operand(const float* U32, float4* lanes) {
  auto comp = [&](int eo, int po, int ei, int pi) -> float {
    const float re = U32[2 * (eo * 8 + ei)], im = U32[2 * (eo * 8 + ei) + 1];
    if (po == pi) return re;
    return po == 0 ? -im : im;
  };
  for (int l = 0; l < 64; ++l) {
    float v[4];
    for (int st = 0; st < 4; ++st) {
      const int i = l % 16, k = 4 * st + l / 16;
      const int go = i >> 2, to = i & 3, gi = k & 3, ti = k >> 2;
      v[st] = comp(2 * go + (to >> 1), to & 1, 2 * gi + (ti >> 1), ti & 1);
    }
    lanes[l] = make_float4(v[0], v[1], v[2], v[3]);
  }
}

int build_tables(Plan& p, const Schedule& s, HostTables* t, std::string* err) {
  const size_t nops = s.ops.size();
  t->ops.resize(nops);
  t->mats.assign(nops * 4 * 16, 0.f);
  // fused phases: first op -> global phase index
  std::vector<int> fused_at(nops, -1);
  {
    int gp = 0;
    for (const Pass& ps : s.passes)
      for (const Phase& pp : ps.phases) {
        if (pp.mf == 1 || pp.mf == 3) {
          if (pp.op_end - pp.op_begin < (pp.mf == 1 ? 3 : 4)) {
            if (err) *err = "fused phase of too few updates";
            return TNC_E_INVALID;
          }
          fused_at[pp.op_begin] = gp;
        }
        ++gp;
      }
    if (std::find_if(fused_at.begin(), fused_at.end(), [](int v) { return v >= 0; }) != fused_at.end())
      t->fmats.assign((size_t)gp * kFusedWords, make_float4(0.f, 0.f, 0.f, 0.f));
  }
  // dense updates whose lower slot sits on the higher register bit of their
  // phase are stored with the two slots exchanged (the kernel takes bit 0 of
  // the 4x4's index from the lower register bit)
  std::vector<char> d4swap(nops, 0);
  for (const Pass& ps : s.passes)
    for (const Phase& pp : ps.phases)
      if (pp.mf == 2 || pp.mf == 3)
        for (int g = pp.mf == 3 ? 2 : 0; g < (pp.op_end - pp.op_begin) / 2 && g < 4; ++g)
          if (pp.dreg[g][0] > pp.dreg[g][1]) d4swap[pp.op_begin + 2 * g] = d4swap[pp.op_begin + 2 * g + 1] = 1;
  cd acc = 0;  // running rounding bias of the sweep (sum of rho - 1)
  size_t fused_left = 0;
  for (size_t o = 0; o < nops; ++o) {
    const SweepOp& op = s.ops[o];
    if (fused_at[o] >= 0 && op.kind == OP_D4) {
      // a bond-four unit: its two 4x4s run as one product, which carries
      // the bias (both control halves of the operand are the same)
      cd U[64];
      float U32[128];
      unit_matrix(&s.ops[o], U);
      const cd r = round_entries(U, 64, acc, U32);
      for (int c = 0; c < 2; ++c) fused_operand(U32, t->fmats.data() + (size_t)fused_at[o] * kFusedWords + c * 64);
      acc += r;
      fused_left = 4;
    } else if (fused_at[o] >= 0) {
      // the three updates run as one product: its rounding carries the bias
      cd U[64];
      float U32[128];
      for (int c = 0; c < 2; ++c) {
        fused_matrix(&s.ops[o], c, U);
        const cd r = round_entries(U, 64, acc, U32);
        fused_operand(U32, t->fmats.data() + (size_t)fused_at[o] * kFusedWords + c * 64);
        if (c == 0) acc += r;
      }
      fused_left = 3;
    }
    if (op.kind == OP_D4) {
      // a dense 4x4: its 16 entries rounded together (one bias factor), the
      // rows split over the two halves' tables
      const SweepOp& hb = s.ops[o + 1];
      cd step = 0;
      for (int var = 0; var < 4; ++var) {
        cd K[16];
        float K32[32];
        auto sw = [&](int u) { return d4swap[o] ? (((u & 1) << 1) | (u >> 1)) : u; };
        for (int rr = 0; rr < 4; ++rr)
          for (int c = 0; c < 4; ++c) K[4 * rr + c] = (sw(rr) < 2 ? op : hb).mat[var][sw(rr) & 1].a[sw(c)];
        // (updates inside a unit product keep their own tables out of the bias)
        const cd r = round_entries(K, 16, fused_left > 0 ? cd(0) : acc, K32);
        if (var == 0) step = r;
        std::copy(K32, K32 + 16, t->mats.data() + (o * 4 + var) * 16);
        std::copy(K32 + 16, K32 + 32, t->mats.data() + ((o + 1) * 4 + var) * 16);
      }
      if (fused_left > 0) fused_left = fused_left > 2 ? fused_left - 2 : 0;
      else acc += step;
      ++o;
      continue;
    }
    // updates inside a fused product keep their own tables (unused by the
    // matrix cores) out of the running bias
    const cd acc_op = fused_left > 0 ? cd(0) : acc;
    cd step = 0;
    for (int var = 0; var < 4; ++var)
      for (int c = 0; c < 2; ++c) {
        const cd r = round_matrix(op.mat[var][c], acc_op, t->mats.data() + (o * 4 + var) * 16 + c * 8);
        if (var == 0 && c == 0) step = r;
      }
    if (fused_left > 0) --fused_left;
    else acc += step;
  }
  for (const Pass& ps : s.passes) {
    PassHost ph;
    ph.w = ps.w;
    ph.R = ps.R;
    ph.phase_off = int(t->phases.size());
    ph.n_phases = int(ps.phases.size());
    ph.op_begin = ps.op_begin;
    ph.op_end = ps.op_end;
    const int R = ph.R;
    auto fail_t = [&](const char* m) {
      if (err) *err = m;
      return TNC_E_INVALID;
    };
    // at most 512 threads per tile (T - R <= 9)
    if (ps.w.tile_bits() - R > 9) return fail_t("pass tile too large for the thread block");
    if (!(ps.w.lo_bits >= 1 || ps.w.win_lo == 0)) return fail_t("pass tile lacks slot 0");
    for (const Phase& pp : ps.phases) {
      const int nops = pp.op_end - pp.op_begin;
      // a fused phase holds two targets in lane bits: up to R + 2 updates;
      // every phase must have an instantiated kernel form
      if (!phase_form_exists(R, nops, pp.mf)) return fail_t("phase size without a kernel form");
      // the bond-four kernels run dense and unit phases and single
      // uncontrolled updates only
      if (p.chi == 4 && pp.mf != 2 && pp.mf != 3 &&
          (nops != 1 || pp.mf != 0 || s.ops[pp.op_begin].kind != OP_CU || s.ops[pp.op_begin].control >= 0))
        return fail_t("bond-four phase without a kernel form");
      DevPhase dp;
      std::memset(&dp, 0, sizeof(dp));
      dp.op_begin = pp.op_begin;
      dp.n_ops = (int8_t)nops;
      dp.first_dup = s.ops[pp.op_begin].kind == OP_DUP ? 1 : 0;
      dp.cloc0 = -1;
      for (int b = 0; b < R; ++b) {
        if (pp.reg[b] < 0 || pp.reg[b] >= ps.w.tile_bits()) return fail_t("bad register map");
        for (int c = 0; c < b; ++c)
          if (pp.reg[b] == pp.reg[c]) return fail_t("bad register map");
        dp.reg[b] = (int8_t)pp.reg[b];
      }
      t->phases.push_back(dp);
      const int T = ps.w.tile_bits();
      if (pp.mf == 3) {
        // bond-four unit: A on (reg0, tpos4), B on (tpos4, tpos5); tail C on
        // (reg1, reg2), D on (reg2, reg0); every tile bit once among
        // registers and thread bits
        const int TB = T - R;
        if ((nops != 4 && nops != 8) || R < 3 || TB < 6 || TB > kMaxThreadBits) return fail_t("bad unit phase shape");
        uint32_t seen = 0;
        for (int b = 0; b < R; ++b) seen |= 1u << pp.reg[b];
        for (int q = 0; q < TB; ++q) {
          if (pp.tpos[q] < 0 || pp.tpos[q] >= T || (seen >> pp.tpos[q] & 1u)) return fail_t("bad unit thread map");
          seen |= 1u << pp.tpos[q];
        }
        auto is4 = [&](int o) {
          return s.ops[o].kind == OP_D4 && s.ops[o + 1].kind == OP_D4H && ps.w.contains(s.ops[o].target) &&
                 ps.w.contains(s.ops[o].pair);
        };
        const SweepOp& A = s.ops[pp.op_begin];
        const SweepOp& B = s.ops[pp.op_begin + 2];
        if (!is4(pp.op_begin) || !is4(pp.op_begin + 2) || ps.w.local(A.target) != pp.reg[0] ||
            ps.w.local(A.pair) != pp.tpos[4] || ps.w.local(B.target) != pp.tpos[4] || ps.w.local(B.pair) != pp.tpos[5] ||
            A.xrow[0] >= 0 || A.xrow[1] >= 0 || B.xrow[0] >= 0 || B.xrow[1] >= 0)
          return fail_t("unit phase product not canonical");
        if (nops == 8) {
          const SweepOp& C = s.ops[pp.op_begin + 4];
          const SweepOp& D = s.ops[pp.op_begin + 6];
          if (!is4(pp.op_begin + 4) || !is4(pp.op_begin + 6) || ps.w.local(C.target) != pp.reg[1] ||
              ps.w.local(C.pair) != pp.reg[2] || ps.w.local(D.target) != pp.reg[2] || ps.w.local(D.pair) != pp.reg[0] ||
              pp.dreg[2][0] != 1 || pp.dreg[2][1] != 2 || pp.dreg[3][0] != 2 || pp.dreg[3][1] != 0)
            return fail_t("unit phase tail not canonical");
        }
        t->phases.back().pad = 3;
        for (int i = 0; i < kPhaseOffs; ++i) {
          uint32_t w = 0;
          if (i < (1 << R)) w = phase_entry_offset(dp, R, i);
          else if (i >= kPhaseEntries && i - kPhaseEntries < TB) w = swz(1u << pp.tpos[i - kPhaseEntries]) << 3;
          t->poffs.push_back(w);
        }
        for (int b = 0; b < nops; ++b) {
          const int o = pp.op_begin + b;
          DevOp d;
          std::memset(&d, 0, sizeof(d));
          d.cloc = -1;
          d.xrow0 = (int16_t)s.ops[o].xrow[0];
          d.xrow1 = (int16_t)s.ops[o].xrow[1];
          d.mat = o;
          t->ops[o] = d;
        }
        continue;
      }
      if (pp.mf == 1) {
        // fused phase: targets reg[0], tpos[4], tpos[5]; op 0's control (if
        // any) reg[R-1]; every tile bit exactly once among registers and
        // thread bits
        const int TB = T - R;
        const int ctl_regs = s.ops[pp.op_begin].control >= 0 ? 1 : 0;
        if (nops < 3 || nops - 2 + ctl_regs > R || R < 3 || TB < 6 || TB > kMaxThreadBits)
          return fail_t("bad fused phase shape");
        uint32_t seen = 0;
        for (int b = 0; b < R; ++b) seen |= 1u << pp.reg[b];
        for (int q = 0; q < TB; ++q) {
          if (pp.tpos[q] < 0 || pp.tpos[q] >= T || (seen >> pp.tpos[q] & 1u)) return fail_t("bad fused thread map");
          seen |= 1u << pp.tpos[q];
        }
        const int tg[3] = {pp.reg[0], pp.tpos[4], pp.tpos[5]};
        for (int b = 0; b < 3; ++b) {
          const SweepOp& op = s.ops[pp.op_begin + b];
          if (op.kind != OP_CU || op.xrow[0] >= 0 || op.xrow[1] >= 0) return fail_t("fused update with variants");
          if (!ps.w.contains(op.target) || ps.w.local(op.target) != tg[b]) return fail_t("fused target not canonical");
          if (b > 0 && (op.control < 0 || !ps.w.contains(op.control) || ps.w.local(op.control) != tg[b - 1]))
            return fail_t("fused control not canonical");
          if (b == 0 && op.control >= 0 && (!ps.w.contains(op.control) || ps.w.local(op.control) != pp.reg[R - 1]))
            return fail_t("fused op 0 control not in the top register bit");
        }
        // the staircase tail on the vector ALUs
        for (int b = 3; b < nops; ++b) {
          const SweepOp& op = s.ops[pp.op_begin + b];
          const int ctl = b == 3 ? pp.tpos[5] : pp.reg[b - 3];
          if (op.kind != OP_CU || !ps.w.contains(op.target) || ps.w.local(op.target) != pp.reg[b - 2] ||
              op.control < 0 || !ps.w.contains(op.control) || ps.w.local(op.control) != ctl)
            return fail_t("fused phase tail not canonical");
          if (pp.reg[b - 2] == pp.reg[R - 1] && s.ops[pp.op_begin].control >= 0)
            return fail_t("fused phase tail on op 0's control bit");
        }
        t->phases.back().pad = 1;
        for (int i = 0; i < kPhaseOffs; ++i) {
          uint32_t w = 0;
          if (i < (1 << R)) w = phase_entry_offset(dp, R, i);
          else if (i >= kPhaseEntries && i - kPhaseEntries < TB) w = swz(1u << pp.tpos[i - kPhaseEntries]) << 3;
          t->poffs.push_back(w);
        }
        for (int b = 0; b < nops; ++b) {
          const int o = pp.op_begin + b;
          DevOp d;
          std::memset(&d, 0, sizeof(d));
          d.cloc = -1;
          d.xrow0 = (int16_t)s.ops[o].xrow[0];
          d.xrow1 = (int16_t)s.ops[o].xrow[1];
          d.mat = o;
          t->ops[o] = d;
        }
        continue;
      }
      if (pp.mf == 2) {
        // dense phase: update g = ops (2g, 2g+1) on register bits dreg[g];
        // its code (the register-bit pair, lower bit first) in 4 bits of
        // reg[6..7]
        uint32_t codes = 0;
        for (int g = 0; g < nops / 2; ++g) {
          const SweepOp& a = s.ops[pp.op_begin + 2 * g];
          const SweepOp& b = s.ops[pp.op_begin + 2 * g + 1];
          const int P = pp.dreg[g][0], Q = pp.dreg[g][1];
          if (a.kind != OP_D4 || b.kind != OP_D4H || b.target != a.target || b.pair != a.pair || P == Q || P < 0 ||
              Q < 0 || P >= R || Q >= R || !ps.w.contains(a.target) || !ps.w.contains(a.pair) ||
              ps.w.local(a.target) != pp.reg[P] || ps.w.local(a.pair) != pp.reg[Q] || b.xrow[0] != a.xrow[0] ||
              b.xrow[1] != a.xrow[1])
            return fail_t("dense phase not canonical");
          codes |= (uint32_t)dense_pair_code(std::min(P, Q), std::max(P, Q)) << (4 * g);
        }
        if (!dense_form_exists(R, nops / 2, codes)) return fail_t("dense phase pattern without a kernel form");
        t->phases.back().pad = 2;
        t->phases.back().reg[6] = (int8_t)(codes & 0xFFu);
        t->phases.back().reg[7] = (int8_t)((codes >> 8) & 0xFFu);
      }
      // thread bits: every tile bit outside the registers exactly once
      {
        const int TB = T - R;
        if (TB > kMaxThreadBits) return fail_t("too many thread bits");
        uint32_t seen = 0;
        for (int b = 0; b < R; ++b) seen |= 1u << pp.reg[b];
        for (int q = 0; q < TB; ++q) {
          if (pp.tpos[q] < 0 || pp.tpos[q] >= T || (seen >> pp.tpos[q] & 1u)) return fail_t("bad thread map");
          seen |= 1u << pp.tpos[q];
        }
        for (int i = 0; i < kPhaseOffs; ++i) {
          uint32_t w = 0;
          if (i < (1 << R)) w = phase_entry_offset(dp, R, i);
          else if (i >= kPhaseEntries && i - kPhaseEntries < TB) w = swz(1u << pp.tpos[i - kPhaseEntries]) << 3;
          t->poffs.push_back(w);
        }
      }
      for (int b = 0; b < nops; ++b) {
        const int o = pp.op_begin + b;
        const SweepOp& op = s.ops[o];
        if (pp.mf == 2) {
          DevOp d;
          std::memset(&d, 0, sizeof(d));
          d.cloc = -1;
          d.xrow0 = (int16_t)op.xrow[0];
          d.xrow1 = (int16_t)op.xrow[1];
          d.mat = o;
          t->ops[o] = d;
          continue;
        }
        if (op.kind != OP_CU && op.kind != OP_DUP) return fail_t("dense update outside a dense phase");
        if (!ps.w.contains(op.target) || ps.w.local(op.target) != pp.reg[b]) return fail_t("op target not canonical");
        DevOp d;
        std::memset(&d, 0, sizeof(d));
        d.cloc = -1;
        if (b == 0) {
          if (op.kind == OP_CU && op.control >= 0) {
            if (!ps.w.contains(op.control)) return fail_t("op control outside the tile");
            const int lc = ps.w.local(op.control);
            for (int q = 0; q < R; ++q)
              if (pp.reg[q] == lc) return fail_t("first op control held in registers");
            int tb = -1;
            for (int q = 0; q < T - R; ++q)
              if (pp.tpos[q] == lc) tb = q;
            if (tb < 0) return fail_t("first op control on no thread bit");
            d.cloc = (int8_t)lc;
            t->phases.back().cloc0 = (int8_t)tb;
          }
        } else {
          if (op.kind != OP_CU || op.control < 0 || !ps.w.contains(op.control) ||
              ps.w.local(op.control) != pp.reg[b - 1])
            return fail_t("op control not canonical");
        }
        d.xrow0 = (int16_t)op.xrow[0];
        d.xrow1 = (int16_t)op.xrow[1];
        d.mat = o;
        t->ops[o] = d;
      }
    }
    t->passes.push_back(ph);
  }
  t->seg.resize((size_t)std::max(0, p.m0 - 1) * 4);
  for (int j = 1; j < p.m0; ++j)
    for (int e = 0; e < 4; ++e)
      t->seg[(size_t)(j - 1) * 4 + e] = make_double2(p.init_seg[j - 1].a[e].real(), p.init_seg[j - 1].a[e].imag());
  int rc = build_late(p, s, &t->late, err);
  if (rc) return rc;
  for (const LateOp& lo : s.late) {
    LateOpDev d;
    std::memset(&d, 0, sizeof(d));
    d.kind = lo.kind;
    d.a = lo.a;
    d.xrow = lo.xrow;
    for (size_t e = 0; e < lo.m.size() && e < 16; ++e) d.m[e] = make_double2(lo.m[e].real(), lo.m[e].imag());
    t->prog.push_back(d);
  }
  // late buffers: first output -> buffer 0, ops launch i -> buffer (i+1)&1
  const LateFirst& F = t->late.first;
  if (!F.final) t->bytes_late[0] = align256((uint64_t)F.M * F.N * 16);
  for (size_t i = 0; i < t->late.ops.size(); ++i) {
    const LateOpsLaunch& ln = t->late.ops[i];
    if (ln.final) continue;
    const uint64_t bytes = align256((uint64_t)(ln.rows_in >> ln.j) * (16ull << t->late.s));
    uint64_t& slot = t->bytes_late[(i + 1) & 1];
    slot = std::max(slot, bytes);
  }
  return 0;
}

// Per-batch workspace for a storage mode: the boundary tensor, two arrays of
// block scales (16-bit storage: read by a launch / written by it, swapped
// after every writer), the batch's resolved update matrices and the two
// late-phase buffers.
struct BatchLayout {
  uint64_t tensor = 0, scales = 0, rmats = 0, late0 = 0, late1 = 0;
  uint64_t per_batch() const { return tensor + 2 * scales + rmats + late0 + late1; }
};

bool is_s16(int storage) { return storage == TNC_STORE_F16_BLOCKSCALE || storage == TNC_STORE_BF16_BLOCKSCALE; }

// Block-scale layout of the row-0 build-up (blocks of 2^min(12, h)
// consecutive entries) and of a pass (its tiles, split in 4096-entry blocks).
ScaleMap init_map(const Plan& p) {
  const int b = std::min(12, p.h);
  return ScaleMap{0, 0, b, b, b};
}

ScaleMap pass_map(const PassHost& ph) {
  const int T = ph.w.tile_bits();
  return ScaleMap{ph.w.lo_bits, ph.w.win_lo, ph.w.win_len, T, std::min(12, T)};
}

BatchLayout batch_layout(const Plan& p, const HostTables& t, int storage) {
  BatchLayout L;
  const bool s16 = is_s16(storage);
  L.tensor = align256((uint64_t)(s16 ? 4 : 8) << p.h);
  if (s16) {
    int blk = std::min(12, p.h);
    for (const PassHost& ph : t.passes) blk = std::min(blk, std::min(12, ph.w.tile_bits()));
    L.scales = align256((uint64_t)4 << (p.h - blk));
  }
  L.rmats = align256((uint64_t)t.ops.size() * 16 * sizeof(float));
  L.late0 = t.bytes_late[0];
  L.late1 = t.bytes_late[1];
  return L;
}

// 16-bit storage reads 2 or 4 consecutive entries per access: every tile
// with a split window must keep at least 2 contiguous low slots.
int check_storage(const HostTables& t, int storage) {
  if (storage != TNC_STORE_C64 && !is_s16(storage)) return set_err(TNC_E_INVALID, "unknown storage mode");
  if (is_s16(storage))
    for (const PassHost& ph : t.passes) {
      if (ph.w.lo_bits == 1) return set_err(TNC_E_INVALID, "16-bit storage needs low_bits >= 2");
      if (ph.w.tile_bits() - ph.R > 9)
        return set_err(TNC_E_INVALID, "16-bit storage needs max_tile_bits - reg_bits <= 9");
    }
  return TNC_OK;
}

// Device copy of the tables for one (k, device).
struct DevSched {
  int device = -1;
  HostTables host;
  DevOp* d_ops = nullptr;
  float* d_mats = nullptr;
  DevPhase* d_phases = nullptr;
  uint32_t* d_poffs = nullptr;
  float4* d_fmats = nullptr;
  double2* d_seg = nullptr;
  double2* d_J = nullptr;
  LateOpDev* d_prog = nullptr;
  // the complex128 reference sweep's updates (built on its first use)
  std::mutex mu64;
  Op64* d_ops64 = nullptr;
  ~DevSched() {
    int prev = 0;
    if (device >= 0 && hipGetDevice(&prev) == hipSuccess) {
      (void)hipSetDevice(device);
      void* ptrs[] = {d_ops, d_mats, d_phases, d_poffs, d_fmats, d_seg, d_J, d_prog, d_ops64};
      for (void* q : ptrs)
        if (q) (void)hipFree(q);
      (void)hipSetDevice(prev);
    }
  }
};

struct PlanDevice {
  std::mutex mu;
  std::map<std::pair<int, int>, std::shared_ptr<DevSched>> m;
};

void free_plan_device(void* p) { delete static_cast<PlanDevice*>(p); }

PlanDevice& plan_device(Plan& p) {
  std::lock_guard<std::mutex> lk(p.mu);
  if (!p.device) {
    p.device = new PlanDevice();
    p.device_free = free_plan_device;
  }
  return *static_cast<PlanDevice*>(p.device);
}

template <typename T>
int upload(T** dst, const std::vector<T>& src) {
  if (src.empty()) return 0;
  hipError_t e = hipMalloc((void**)dst, src.size() * sizeof(T));
  if (e != hipSuccess) return set_err(TNC_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(e, "hipMemcpy");
  return 0;
}

int get_dev_sched(Plan& p, int k, std::shared_ptr<DevSched>* out) {
  if (p.h > kMaxDeviceWidth) return set_err(TNC_E_DOMAIN, "boundary tensors above 2^40 entries are planned only");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(e, "hipGetDevice");
  PlanDevice& pd = plan_device(p);
  std::lock_guard<std::mutex> lk(pd.mu);
  auto it = pd.m.find({k, dev});
  if (it != pd.m.end()) {
    *out = it->second;
    return 0;
  }
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(p, k, &s, &err);
  if (rc) return set_err(rc, err);
  auto ds = std::make_shared<DevSched>();
  ds->device = dev;
  rc = build_tables(p, *s, &ds->host, &err);
  if (rc) return set_err(rc, err);
  std::vector<double2> J;
  for (const cd& z : ds->host.late.first.J) J.push_back(make_double2(z.real(), z.imag()));
  if ((rc = upload(&ds->d_ops, ds->host.ops)) || (rc = upload(&ds->d_mats, ds->host.mats)) ||
      (rc = upload(&ds->d_phases, ds->host.phases)) || (rc = upload(&ds->d_poffs, ds->host.poffs)) ||
      (rc = upload(&ds->d_fmats, ds->host.fmats)) ||
      (rc = upload(&ds->d_seg, ds->host.seg)) ||
      (rc = upload(&ds->d_J, J)) || (rc = upload(&ds->d_prog, ds->host.prog)))
    return rc;
  pd.m[{k, dev}] = ds;
  *out = ds;
  return 0;
}

// The device tables for (k, current device) if they were already built,
// else null; never builds, uploads or allocates.
std::shared_ptr<DevSched> find_dev_sched(Plan& p, int k) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  {
    std::lock_guard<std::mutex> lk(p.mu);
    if (!p.device) return nullptr;
  }
  PlanDevice& pd = plan_device(p);
  std::lock_guard<std::mutex> lk(pd.mu);
  auto it = pd.m.find({k, dev});
  return it == pd.m.end() ? nullptr : it->second;
}

// Scratch memory of tnc_amplitudes_noalloc: one copy of this array on each
// GPU the library runs on, held until the process ends.  In host code the
// name stands for a host-side handle, never for the device address: every
// host use goes through the per-device address from hipGetSymbolAddress.
constexpr uint64_t kNoAllocScratchBytes = 256ull << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;  // device -> address of `scratch` there

// The scratch address on the current device (looked up once per device,
// with that device current).
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_err(e, "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return TNC_OK;
  }
  void* ptr = nullptr;
  e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_err(e, "hipGetSymbolAddress of the scratch array");
  g_scratch_ptr[dev] = ptr;
  *out = ptr;
  return TNC_OK;
}

// Process-wide event timing of kernel launches (tnc_profile_*).
struct Profiler {
  std::mutex mu;
  bool active = false;
  struct Rec {
    int cls;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<Rec> recs;
};
Profiler g_prof;
// per-launch durations of the last finished profiling session (class, ms)
std::vector<std::pair<int, double>> g_prof_last;

// Records an event pair around `launch` when profiling is on.
template <typename F>
hipError_t timed(int cls, double bytes, hipStream_t s, F&& launch) {
  bool on;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    on = g_prof.active;
  }
  if (!on) return launch();
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  e = hipEventRecord(b, s);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.recs.push_back({cls, a, b, bytes});
  return hipSuccess;
}

InitArgs init_args(const Plan& p, const HostTables& t, float2* B, const uint8_t* bits, int nb,
                   const double2* d_seg) {
  InitArgs a;
  std::memset(&a, 0, sizeof(a));
  a.B = B;
  a.bits = bits;
  a.seg = d_seg;
  for (int w = 0; w < 2; ++w) a.v[w] = make_double2(p.init_v[w].real(), p.init_v[w].imag());
  for (int x = 0; x < 2; ++x)
    for (int w = 0; w < 2; ++w) a.f[x][w] = make_double2(p.init_f[x][w].real(), p.init_f[x][w].imag());
  a.m0 = p.m0;
  a.h = p.h;
  a.n = p.n;
  a.n_batches = nb;
  (void)t;
  return a;
}

PassArgs pass_args(const Plan& p, const PassHost& ph, const DevPhase* phases, const uint32_t* poffs,
                   const float4* fmats, float2* B, const uint8_t* bits, int nb) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.phases = phases + ph.phase_off;
  a.poffs = poffs + (size_t)ph.phase_off * kPhaseOffs;
  a.fmats = fmats ? fmats + (size_t)ph.phase_off * kFusedWords : nullptr;
  a.B = B;
  a.bits = bits;
  a.n_phases = ph.n_phases;
  a.n = p.n;
  a.h = p.h;
  a.T = ph.w.tile_bits();
  a.lo_bits = ph.w.lo_bits;
  a.win_lo = ph.w.win_lo;
  a.win_len = ph.w.win_len;
  a.n_tiles = nb << (p.h - a.T);
  a.kind = p.chi == 4 ? 1 : 0;
  return a;
}

LateArgs first_args(const Plan& p, const HostTables& t, const void* in, double2* out, long long out_stride,
                    const double2* J, const uint8_t* bits, int nb) {
  const LateFirst& F = t.late.first;
  LateArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.J = J;
  a.bits = bits;
  a.in_batch_stride = 1ll << p.h;
  a.out_batch_stride = out_stride;
  a.M = (int)F.M;
  a.K = F.K;
  a.N = F.N;
  a.n_batches = nb;
  a.xrow = F.xrow;
  a.n = p.n;
  return a;
}

LateOpsArgs ops_args(const Plan& p, const HostTables& t, const LateOpsLaunch& ln, const double2* in, double2* out,
                     long long out_stride, const LateOpDev* prog, const uint8_t* bits, int nb, int k) {
  LateOpsArgs a;
  std::memset(&a, 0, sizeof(a));
  a.in = in;
  a.out = out;
  a.bits = bits;
  a.prog = prog + ln.op_begin;
  a.n_prog = ln.op_end - ln.op_begin;
  a.s = t.late.s;
  a.j = ln.j;
  a.in_batch_stride = ln.rows_in << t.late.s;
  a.out_batch_stride = out_stride;
  a.rows_out = ln.rows_in >> ln.j;
  a.n_batches = nb;
  a.n = p.n;
  a.k = k;
  a.final_kind = ln.final ? t.late.final_kind : 0;
  a.final_xrow = t.late.final_xrow;
  if (t.late.final_kind == L_DOT)
    for (int x = 0; x < 2; ++x)
      for (int w = 0; w < 2; ++w)
        a.dot[x][w] = make_double2(t.late.dot[2 * x + w].real(), t.late.dot[2 * x + w].imag());
  return a;
}

// Every launch of one amplitude call, in order, recorded with its arguments:
// for each group of batches that fits the workspace, the row-0 build-up, the
// variant resolution, the passes, the join and the late launches.
int record_launches(Plan& p, DevSched& ds, int nb_total, const uint8_t* d_bits, int k, int storage, tnc_c128* d_out,
                    void* ws, uint64_t ws_bytes, std::vector<Launch>* out) {
  const HostTables& t = ds.host;
  int rc = check_storage(t, storage);
  if (rc) return rc;
  const bool s16 = is_s16(storage);
  const BatchLayout L = batch_layout(p, t, storage);
  const uint64_t per = L.per_batch();
  const uint64_t fit = ws_bytes / per;
  if (fit < 1) return set_err(TNC_E_NOMEM, "workspace smaller than one batch");
  const int chunk = (int)std::min<uint64_t>(fit, (uint64_t)std::min(nb_total, 65535));
  char* base = static_cast<char*>(ws);
  const long long sstride = (long long)(L.scales / 4);
  auto shape_err = [&](const char* what) {
    return set_err(TNC_E_INVALID, std::string("launch shape out of range: ") + what);
  };
  out->clear();
  Launch rec;
  for (int b0 = 0; b0 < nb_total; b0 += chunk) {
    const int nb = std::min(chunk, nb_total - b0);
    char* q = base;
    float2* B = reinterpret_cast<float2*>(q);
    q += L.tensor * nb;
    float* sc[2] = {reinterpret_cast<float*>(q), reinterpret_cast<float*>(q + L.scales * nb)};
    q += 2 * L.scales * nb;
    float* rmats = reinterpret_cast<float*>(q);
    const long long rstride = (long long)(L.rmats / 4);
    q += L.rmats * nb;
    double2* L0 = reinterpret_cast<double2*>(q);
    double2* L1 = reinterpret_cast<double2*>(q + L.late0 * nb);
    const uint8_t* bits = d_bits + (size_t)b0 * p.n;
    double2* outp = reinterpret_cast<double2*>(d_out) + ((size_t)b0 << k);
    InitArgs ia = init_args(p, t, B, bits, nb, ds.d_seg);
    if (s16) {
      ia.store = storage;
      ia.scale_out = sc[0];
      ia.scale_stride = sstride;
      ia.blk_bits = std::min(12, p.h);
    }
    if (record_init(ia, &rec) != hipSuccess) return shape_err("row-0 build-up");
    out->push_back(rec);
    ResolveArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.ops = ds.d_ops;
    ra.mats = ds.d_mats;
    ra.bits = bits;
    ra.rmats = rmats;
    ra.rstride = rstride;
    ra.n_ops = (int)t.ops.size();
    ra.n = p.n;
    ra.n_batches = nb;
    if (ra.n_ops > 0) {
      if (record_resolve(ra, &rec) != hipSuccess) return shape_err("variant resolution");
      out->push_back(rec);
    }
    const double pass_bytes = 2.0 * (s16 ? 4.0 : 8.0) * (double)(1ull << p.h) * nb;
    int cur = 0;
    ScaleMap map = init_map(p);
    for (const PassHost& ph : t.passes) {
      PassArgs a = pass_args(p, ph, ds.d_phases, ds.d_poffs, ds.d_fmats, B, bits, nb);
      a.rmats = rmats;
      a.rstride = rstride;
      if (s16) {
        a.store = storage;
        a.scale_in = sc[cur];
        a.scale_out = sc[cur ^ 1];
        a.scale_stride = sstride;
        a.in_map = map;
      }
      if (record_pass(a, ph.R, &rec) != hipSuccess) return shape_err("pass");
      rec.bytes = pass_bytes;
      out->push_back(rec);
      if (s16) {
        cur ^= 1;
        map = pass_map(ph);
      }
    }
    const LateFirst& F = t.late.first;
    double2* fout = F.final ? outp : L0;
    const long long fstride = F.final ? (1ll << k) : (long long)(t.bytes_late[0] / 16);
    LateArgs fa = first_args(p, t, B, fout, fstride, ds.d_J, bits, nb);
    if (s16) {
      fa.store = storage;
      fa.scale_in = sc[cur];
      fa.scale_stride = sstride;
      fa.in_map = map;
    }
    if (record_late(fa, true, &rec) != hipSuccess) return shape_err("join");
    out->push_back(rec);
    const double2* curl = L0;
    long long cur_stride = fstride;
    for (size_t i = 0; i < t.late.ops.size(); ++i) {
      const LateOpsLaunch& ln = t.late.ops[i];
      double2* dst = ln.final ? outp : ((i + 1) & 1 ? L1 : L0);
      const long long dstride = ln.final ? (1ll << k) : (long long)(t.bytes_late[(i + 1) & 1] / 16);
      LateOpsArgs a = ops_args(p, t, ln, curl, dst, dstride, ds.d_prog, bits, nb, k);
      a.in_batch_stride = cur_stride;
      if (record_late_ops(a, &rec) != hipSuccess) return shape_err("late program");
      out->push_back(rec);
      curl = dst;
      cur_stride = dstride;
    }
  }
  return TNC_OK;
}

// Issues recorded launches on `stream`; every launch's own status is
// checked (nothing pending on the calling thread is read or cleared).
int issue_all(const std::vector<Launch>& ls, hipStream_t stream) {
  for (const Launch& L : ls) {
    const hipError_t e = timed(L.cls, L.bytes, stream, [&] { return issue(L, stream); });
    if (e != hipSuccess) return hip_err(e, "kernel launch");
  }
  return TNC_OK;
}

int run_device(Plan& p, DevSched& ds, int nb_total, const uint8_t* d_bits, int k, int storage, tnc_c128* d_out,
               void* ws, uint64_t ws_bytes, hipStream_t stream) {
  std::vector<Launch> ls;
  const int rc = record_launches(p, ds, nb_total, d_bits, k, storage, d_out, ws, ws_bytes, &ls);
  if (rc) return rc;
  return issue_all(ls, stream);
}

// The complex128 reference path (tests): per batch the 2^h complex128
// tensor and the two late-phase buffers.
uint64_t c128_per_batch(const Plan& p, const HostTables& t) {
  return align256((uint64_t)16 << p.h) + t.bytes_late[0] + t.bytes_late[1];
}

int run_c128(Plan& p, DevSched& ds, int nb_total, const uint8_t* d_bits, int k, tnc_c128* d_out, void* ws,
             uint64_t ws_bytes, hipStream_t stream) {
  const HostTables& t = ds.host;
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(p, k, &s, &err);
  if (rc) return set_err(rc, err);
  {
    std::lock_guard<std::mutex> lk(ds.mu64);
    if (!ds.d_ops64 && !s->ops.empty()) {
      std::vector<Op64> ops(s->ops.size());
      for (size_t o = 0; o < s->ops.size(); ++o) {
        const SweepOp& so = s->ops[o];
        Op64& d = ops[o];
        std::memset(&d, 0, sizeof(d));
        d.kind = so.kind == OP_DUP ? 1 : 0;
        d.target = so.target;
        d.control = so.control;
        d.xrow0 = so.xrow[0];
        d.xrow1 = so.xrow[1];
        for (int v = 0; v < 4; ++v)
          for (int c = 0; c < 2; ++c)
            for (int e = 0; e < 4; ++e) d.m[v][c][e] = make_double2(so.mat[v][c].a[e].real(), so.mat[v][c].a[e].imag());
      }
      if ((rc = upload(&ds.d_ops64, ops))) return rc;
    }
  }
  const uint64_t per = c128_per_batch(p, t);
  const uint64_t fit = ws_bytes / per;
  if (fit < 1) return set_err(TNC_E_NOMEM, "workspace smaller than one batch");
  const int chunk = (int)std::min<uint64_t>(fit, (uint64_t)std::min(nb_total, 65535));
  const uint64_t tensor = align256((uint64_t)16 << p.h);
  for (int b0 = 0; b0 < nb_total; b0 += chunk) {
    const int nb = std::min(chunk, nb_total - b0);
    char* q = static_cast<char*>(ws);
    double2* B = reinterpret_cast<double2*>(q);
    q += tensor * nb;
    double2* L0 = reinterpret_cast<double2*>(q);
    double2* L1 = reinterpret_cast<double2*>(q + t.bytes_late[0] * nb);
    const uint8_t* bits = d_bits + (size_t)b0 * p.n;
    double2* outp = reinterpret_cast<double2*>(d_out) + ((size_t)b0 << k);
    InitArgs ia = init_args(p, t, reinterpret_cast<float2*>(B), bits, nb, ds.d_seg);
    hipError_t e = launch_init64(ia, stream);
    if (e != hipSuccess) return hip_err(e, "complex128 build-up launch");
    for (size_t o = 0; o < s->ops.size(); ++o) {
      Op64Args a{B, bits, ds.d_ops64 + o, p.h, p.n, nb};
      if ((e = launch_op64(a, stream)) != hipSuccess) return hip_err(e, "complex128 update launch");
    }
    // the late phase reads the complex128 tensor (the FP64 join kernel)
    const LateFirst& F = t.late.first;
    double2* fout = F.final ? outp : L0;
    const long long fstride = F.final ? (1ll << k) : (long long)(t.bytes_late[0] / 16);
    LateArgs fa = first_args(p, t, B, fout, fstride, ds.d_J, bits, nb);
    std::vector<Launch> ls(1);
    if (record_late(fa, false, &ls[0]) != hipSuccess) return set_err(TNC_E_INVALID, "launch shape out of range: join");
    const double2* curl = L0;
    long long cur_stride = fstride;
    for (size_t i = 0; i < t.late.ops.size(); ++i) {
      const LateOpsLaunch& ln = t.late.ops[i];
      double2* dst = ln.final ? outp : ((i + 1) & 1 ? L1 : L0);
      const long long dstride = ln.final ? (1ll << k) : (long long)(t.bytes_late[(i + 1) & 1] / 16);
      LateOpsArgs a = ops_args(p, t, ln, curl, dst, dstride, ds.d_prog, bits, nb, k);
      a.in_batch_stride = cur_stride;
      Launch L;
      if (record_late_ops(a, &L) != hipSuccess) return set_err(TNC_E_INVALID, "launch shape out of range: late");
      ls.push_back(L);
      curl = dst;
      cur_stride = dstride;
    }
    if ((rc = issue_all(ls, stream))) return rc;
  }
  return TNC_OK;
}

// Host emulation of the whole device pipeline with the same tables.
int emulate(Plan& p, int k, int nb, const uint8_t* bits, int storage, cd* out) {
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(p, k, &s, &err);
  if (rc) return set_err(rc, err);
  HostTables t;
  rc = build_tables(p, *s, &t, &err);
  if (rc) return set_err(rc, err);
  if (p.h > 24) return set_err(TNC_E_DOMAIN, "emulation limited to width 24");
  if ((rc = check_storage(t, storage))) return rc;
  const bool s16 = is_s16(storage);
  const size_t dim = size_t(1) << p.h;
  // complex64 tensor, or (16-bit storage) the packed words in its first half
  std::vector<float2> B(dim * nb);
  uint32_t* Bw = reinterpret_cast<uint32_t*>(B.data());
  const BatchLayout L = batch_layout(p, t, storage);
  const long long sstride = (long long)(L.scales / 4);
  std::vector<float> sc[2] = {std::vector<float>((size_t)sstride * nb), std::vector<float>((size_t)sstride * nb)};
  // init (same arithmetic as k_init / k_init16: FP64 product rounded to FP32)
  const int ib = std::min(12, p.h);
  for (int b = 0; b < nb; ++b) {
    std::vector<float2> row(dim);
    for (size_t i = 0; i < dim; ++i) {
      cd v = 0;
      if (i < (size_t(1) << p.m0)) {
        v = p.init_v[i & 1];
        for (int j = 1; j < p.m0; ++j) v *= p.init_seg[j - 1](int(i >> j & 1), int(i >> (j - 1) & 1));
        v *= p.init_f[bits[(size_t)b * p.n]][int(i >> (p.m0 - 1) & 1)];
      }
      row[i] = make_float2((float)v.real(), (float)v.imag());
    }
    if (!s16) {
      std::copy(row.begin(), row.end(), B.begin() + (size_t)b * dim);
      continue;
    }
    for (size_t blk = 0; blk < (dim >> ib); ++blk) {
      float amax = 0.f;
      for (size_t i = blk << ib; i < (blk + 1) << ib; ++i)
        amax = std::max(amax, std::max(std::fabs(row[i].x), std::fabs(row[i].y)));
      const int e = block_exponent(amax);
      const float inv = std::ldexp(1.f, -e);
      for (size_t i = blk << ib; i < (blk + 1) << ib; ++i)
        Bw[(size_t)b * dim + i] = storage == TNC_STORE_F16_BLOCKSCALE ? pack16<STORE_F16>(row[i].x, row[i].y, inv)
                                                                      : pack16<STORE_BF16>(row[i].x, row[i].y, inv);
      sc[0][(size_t)b * sstride + blk] = std::ldexp(1.f, e);
    }
  }
  // variant resolution (k_resolve)
  const long long rstride = (long long)(L.rmats / 4);
  std::vector<float> rmats((size_t)rstride * nb);
  for (int b = 0; b < nb; ++b)
    for (size_t o = 0; o < t.ops.size(); ++o) {
      const DevOp& op = t.ops[o];
      const uint8_t* x = bits + (size_t)b * p.n;
      const int var = (op.xrow0 >= 0 ? 2 * (x[op.xrow0] & 1) : 0) + (op.xrow1 >= 0 ? (x[op.xrow1] & 1) : 0);
      for (int e = 0; e < 16; ++e)
        rmats[(size_t)b * rstride + o * 16 + e] = t.mats[((size_t)op.mat * 4 + var) * 16 + e];
    }
  int cur = 0;
  ScaleMap map = init_map(p);
  for (const PassHost& ph : t.passes) {
    PassArgs a = pass_args(p, ph, t.phases.data(), t.poffs.data(), t.fmats.empty() ? nullptr : t.fmats.data(), B.data(),
                           bits, nb);
    a.rmats = rmats.data();
    a.rstride = rstride;
    if (s16) {
      a.store = storage;
      a.scale_in = sc[cur].data();
      a.scale_out = sc[cur ^ 1].data();
      a.scale_stride = sstride;
      a.in_map = map;
    }
    emulate_pass_host(a, ph.R);
    if (s16) {
      cur ^= 1;
      map = pass_map(ph);
    }
  }
  // the first late launch's input, decoded
  auto entry = [&](int b, uint64_t g) -> cd {
    if (!s16) {
      const float2 x = B[(size_t)b * dim + g];
      return cd(x.x, x.y);
    }
    const float scl = sc[cur][(size_t)b * sstride + scale_slot(g, map)];
    const uint32_t w = Bw[(size_t)b * dim + g];
    const float2 x = storage == TNC_STORE_F16_BLOCKSCALE ? unpack16<STORE_F16>(w, scl) : unpack16<STORE_BF16>(w, scl);
    return cd(x.x, x.y);
  };
  // late (FP64), same tables
  const LateFirst& F = t.late.first;
  const int sb = t.late.s;
  for (int b = 0; b < nb; ++b) {
    const int var = F.xrow >= 0 ? bits[(size_t)b * p.n + F.xrow] : 0;
    std::vector<cd> cur((size_t)F.M * F.N);
    for (long long r = 0; r < F.M; ++r)
      for (int c = 0; c < F.N; ++c) {
        cd acc = 0;
        for (int kk = 0; kk < F.K; ++kk) acc += entry(b, (uint64_t)r * F.K + kk) * F.J[((size_t)var * F.K + kk) * F.N + c];
        cur[(size_t)r * F.N + c] = acc;
      }
    for (const LateOpsLaunch& ln : t.late.ops) {
      const long long rows_out = ln.rows_in >> ln.j;
      std::vector<cd> nxt((size_t)rows_out << sb);
      for (long long ro = 0; ro < rows_out; ++ro) {
        std::vector<cd> st(cur.begin() + ((size_t)ro << (ln.j + sb)), cur.begin() + ((size_t)(ro + 1) << (ln.j + sb)));
        int l = 0;
        for (int o = ln.op_begin; o < ln.op_end; ++o) {
          const LateOp& op = s->late[o];
          const int live = ln.j - l;
          for (int r = 0; r < (1 << live); ++r) {
            const int row = r << l;
            cd* v = st.data() + ((size_t)row << sb);
            if (op.kind == L_U1) {
              for (int i = 0; i < (1 << sb); ++i) {
                if (i >> op.a & 1) continue;
                const int i1 = i | (1 << op.a);
                const cd a0 = v[i], a1 = v[i1];
                v[i] = op.m[0] * a0 + op.m[1] * a1;
                v[i1] = op.m[2] * a0 + op.m[3] * a1;
              }
            } else if (op.kind == L_G4) {
              for (int i = 0; i < (1 << sb); ++i) {
                if ((i >> op.a & 1) || (i >> (op.a + 1) & 1)) continue;
                const int idx[4] = {i, i | (1 << (op.a + 1)), i | (1 << op.a), i | (3 << op.a)};
                cd x[4], y[4];
                for (int u = 0; u < 4; ++u) x[u] = v[idx[u]];
                for (int q = 0; q < 4; ++q) {
                  y[q] = 0;
                  for (int u = 0; u < 4; ++u) y[q] += op.m[4 * q + u] * x[u];
                }
                for (int u = 0; u < 4; ++u) v[idx[u]] = y[u];
              }
            } else if ((op.kind == L_REMOVE && (r & 1) == 0) || (op.kind == L_REMOVE2 && (r & 3) == 0)) {
              const int nu = op.kind == L_REMOVE ? 2 : 4;
              const int off = (op.kind == L_REMOVE && op.xrow >= 0 && (bits[(size_t)b * p.n + op.xrow] & 1)) ? 8 : 0;
              for (int i = 0; i < (1 << sb); i += 2) {
                cd y0 = 0, y1 = 0;
                for (int u = 0; u < nu; ++u) {
                  const cd* w = st.data() + ((size_t)(row | (u << l)) << sb);
                  const cd* m = op.m.data() + off + 4 * u;
                  y0 += m[0] * w[i] + m[1] * w[i + 1];
                  y1 += m[2] * w[i] + m[3] * w[i + 1];
                }
                v[i] = y0;
                v[i + 1] = y1;
              }
            }
          }
          if (op.kind == L_REMOVE) ++l;
          else if (op.kind == L_REMOVE2) l += 2;
        }
        for (int q = 0; q < (1 << sb); ++q) nxt[((size_t)ro << sb) + q] = st[q];
      }
      cur.swap(nxt);
    }
    cd* o = out + ((size_t)b << k);
    if (F.final) {
      for (int c = 0; c < (1 << k); ++c) o[c] = cur[c];
    } else if (t.late.final_kind == L_OUT) {
      for (int bb = 0; bb < (1 << k); ++bb) {
        int tt = 0;
        for (int q = 0; q < k; ++q) tt |= ((bb >> (k - 1 - q)) & 1) << q;
        o[bb] = cur[tt];
      }
    } else {
      const int x = bits[(size_t)b * p.n + t.late.final_xrow];
      o[0] = t.late.dot[2 * x] * cur[0] + t.late.dot[2 * x + 1] * cur[1];
    }
  }
  return TNC_OK;
}

Plan* get(tnc_plan_t h) { return h ? h->plan.get() : nullptr; }

}  // namespace

int record_amplitudes(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, int32_t storage,
                      tnc_c128* d_out, void* d_workspace, uint64_t workspace_bytes, std::vector<Launch>* out) {
  Plan* p = get(plan);
  out->clear();
  if (!p || n_batches < 0 || (n_batches > 0 && (!d_bits || !d_out || !d_workspace)))
    return set_err(TNC_E_INVALID, "bad argument");
  if (storage != TNC_STORE_C64 && !is_s16(storage)) return set_err(TNC_E_INVALID, "unknown storage mode");
  if (n_batches == 0) return TNC_OK;
  std::shared_ptr<DevSched> ds;
  int rc = get_dev_sched(*p, k, &ds);
  if (rc) return rc;
  return record_launches(*p, *ds, n_batches, d_bits, k, storage, d_out, d_workspace, workspace_bytes, out);
}

int issue_recorded(const std::vector<Launch>& ls, hipStream_t stream) { return issue_all(ls, stream); }
}  // namespace tnc

using namespace tnc;

extern "C" {

int tnc_plan(int32_t n, int32_t d, const tnc_c128* one_qubit, int32_t n_gate2, const tnc_gate2* gates,
             const tnc_options* opt, tnc_plan_t* out) {
  if (!out || !one_qubit || (n_gate2 > 0 && !gates) || n_gate2 < 0) return set_err(TNC_E_INVALID, "null argument");
  *out = nullptr;
  Options o;
  if (opt) {
    if (opt->max_tile_bits) o.max_tile_bits = opt->max_tile_bits;
    if (opt->reg_bits) o.reg_bits = opt->reg_bits;
    if (opt->low_bits) o.low_bits = opt->low_bits;
    o.math = opt->math;
    o.late_fold = opt->late_fold;
    o.reg_adapt = opt->reg_adapt;
    o.bond = opt->bond;
    o.mem_cap_bytes = opt->mem_cap_bytes;
  }
  if (o.max_tile_bits < 6 || o.max_tile_bits > 14 || o.reg_bits < 1 || o.reg_bits > 5 || o.low_bits < 1 ||
      o.low_bits > o.max_tile_bits - 2 || (o.math != 0 && o.math != 2) || o.late_fold < -1 || o.late_fold > 8 ||
      o.reg_adapt < 0 || o.reg_adapt > 1 || o.max_tile_bits - o.reg_bits > 9 ||
      (o.bond != 0 && o.bond != 2 && o.bond != 4))
    return set_err(TNC_E_INVALID, "tile options out of range");
  if (n < 2 || d < 2 || (int64_t)n * (d + 1) > (1 << 24)) return set_err(TNC_E_DOMAIN, "need n >= 2, d >= 2");
  std::vector<cd> one((size_t)(d + 1) * n * 4);
  for (size_t i = 0; i < one.size(); ++i) one[i] = cd(one_qubit[i].re, one_qubit[i].im);
  std::vector<std::vector<cd>> mats(n_gate2);
  std::vector<Gate2In> g(n_gate2);
  for (int i = 0; i < n_gate2; ++i) {
    mats[i].resize(16);
    for (int e = 0; e < 16; ++e) mats[i][e] = cd(gates[i].m[e].re, gates[i].m[e].im);
    g[i] = Gate2In{gates[i].layer, gates[i].q, gates[i].kind, mats[i].data()};
  }
  std::unique_ptr<Plan> p;
  std::string err;
  int rc = build_plan(n, d, one.data(), n_gate2, g.data(), o, &p, &err);
  if (rc) return set_err(rc, err);
  auto* h = new tnc_plan_s();
  h->plan = std::move(p);
  *out = h;
  return TNC_OK;
}

int tnc_plan_info(tnc_plan_t plan, int32_t k, tnc_info* info) {
  Plan* p = get(plan);
  if (!p || !info) return set_err(TNC_E_INVALID, "null argument");
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(*p, k, &s, &err);
  if (rc) return set_err(rc, err);
  HostTables t;
  rc = build_tables(*p, *s, &t, &err);
  if (rc) return set_err(rc, err);
  std::memset(info, 0, sizeof(*info));
  info->width = s->width;
  info->boundary_bits = p->h;
  info->live_slots_fixed = s->m_fix;
  info->n_ops = (int32_t)std::count_if(s->ops.begin(), s->ops.end(), [](const SweepOp& o) { return o.kind != OP_D4H; });
  info->n_passes = (int32_t)s->passes.size();
  info->n_phases = (int32_t)t.phases.size();
  info->n_late_launches = 1 + (int32_t)t.late.ops.size();
  info->fixed_rows = s->last_fixed_row + 1;
  info->early_layers = k >= 1 ? 2 * k : 0;
  info->late_layers = k >= 1 ? p->d - 2 * k : 0;
  info->log2_cost = s->log2_cost;
  info->workspace_per_batch = p->h <= kMaxDeviceWidth ? batch_layout(*p, t, TNC_STORE_C64).per_batch() : 0;
  info->bond = p->chi;
  return TNC_OK;
}

int tnc_prepare(tnc_plan_t plan, int32_t k) {
  Plan* p = get(plan);
  if (!p) return set_err(TNC_E_INVALID, "null plan");
  std::shared_ptr<DevSched> ds;
  return get_dev_sched(*p, k, &ds);
}

int tnc_workspace_bytes(tnc_plan_t plan, int32_t k, int32_t n_batches, int32_t storage, uint64_t* bytes) {
  Plan* p = get(plan);
  if (!p || !bytes || n_batches < 0) return set_err(TNC_E_INVALID, "bad argument");
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(*p, k, &s, &err);
  if (rc) return set_err(rc, err);
  HostTables t;
  rc = build_tables(*p, *s, &t, &err);
  if (rc) return set_err(rc, err);
  if ((rc = check_storage(t, storage))) return rc;
  if (p->h > kMaxDeviceWidth) return set_err(TNC_E_DOMAIN, "boundary tensors above 2^40 entries are planned only");
  const uint64_t per = batch_layout(*p, t, storage).per_batch();
  if (p->opt.mem_cap_bytes && per > p->opt.mem_cap_bytes)
    return set_err(TNC_E_NOMEM, "one batch's workspace (" + std::to_string(per) + " bytes) exceeds mem_cap_bytes");
  *bytes = (uint64_t)n_batches * per;
  return TNC_OK;
}

int tnc_amplitudes(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, int32_t storage,
                   tnc_c128* d_out, void* d_workspace, uint64_t workspace_bytes, void* stream) {
  Plan* p = get(plan);
  if (!p || n_batches < 0 || (n_batches > 0 && (!d_bits || !d_out || !d_workspace)))
    return set_err(TNC_E_INVALID, "bad argument");
  if (storage != TNC_STORE_C64 && !is_s16(storage)) return set_err(TNC_E_INVALID, "unknown storage mode");
  if (n_batches == 0) return TNC_OK;
  std::shared_ptr<DevSched> ds;
  int rc = get_dev_sched(*p, k, &ds);
  if (rc) return rc;
  // the cap bounds the part of the caller's workspace in use
  if (p->opt.mem_cap_bytes) workspace_bytes = std::min<uint64_t>(workspace_bytes, p->opt.mem_cap_bytes);
  return run_device(*p, *ds, n_batches, d_bits, k, storage, d_out, d_workspace, workspace_bytes,
                    static_cast<hipStream_t>(stream));
}

int tnc_amplitudes_noalloc(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, int32_t storage,
                           tnc_c128* d_out, void* stream) {
  Plan* p = get(plan);
  if (!p || n_batches < 0 || (n_batches > 0 && (!d_bits || !d_out))) return set_err(TNC_E_INVALID, "bad argument");
  if (storage != TNC_STORE_C64 && !is_s16(storage)) return set_err(TNC_E_INVALID, "unknown storage mode");
  if (n_batches == 0) return TNC_OK;
  std::shared_ptr<DevSched> ds = find_dev_sched(*p, k);
  if (!ds)
    return set_err(TNC_E_INVALID, "device tables for these open legs are not prepared on this device "
                                  "(call tnc_prepare first; this entry point allocates nothing)");
  int rc = check_storage(ds->host, storage);
  if (rc) return rc;
  const uint64_t per = batch_layout(*p, ds->host, storage).per_batch();
  if (per > kNoAllocScratchBytes)
    return set_err(TNC_E_NOMEM, "one batch needs " + std::to_string(per) + " bytes of workspace, above the " +
                                    std::to_string(kNoAllocScratchBytes) + "-byte scratch of tnc_amplitudes_noalloc");
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  std::vector<Launch> ls;
  rc = record_launches(*p, *ds, n_batches, d_bits, k, storage, d_out, ws, kNoAllocScratchBytes, &ls);
  if (rc) return rc;
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (const Launch& L : ls) {
    const hipError_t e = issue(L, st);
    if (e != hipSuccess) return hip_err(e, "kernel launch");
  }
  return TNC_OK;
}

uint64_t tnc_noalloc_scratch_bytes(void) { return kNoAllocScratchBytes; }

int tnc_debug_workspace_c128(tnc_plan_t plan, int32_t k, int32_t n_batches, uint64_t* bytes) {
  Plan* p = get(plan);
  if (!p || !bytes || n_batches < 0) return set_err(TNC_E_INVALID, "bad argument");
  if (p->chi == 4) return set_err(TNC_E_DOMAIN, "the complex128 reference sweep covers bond dimension 2 only");
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(*p, k, &s, &err);
  if (rc) return set_err(rc, err);
  HostTables t;
  rc = build_tables(*p, *s, &t, &err);
  if (rc) return set_err(rc, err);
  *bytes = (uint64_t)n_batches * c128_per_batch(*p, t);
  return TNC_OK;
}

int tnc_debug_amplitudes_c128(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, tnc_c128* d_out,
                              void* d_workspace, uint64_t workspace_bytes, void* stream) {
  Plan* p = get(plan);
  if (!p || n_batches < 0 || (n_batches > 0 && (!d_bits || !d_out || !d_workspace)))
    return set_err(TNC_E_INVALID, "bad argument");
  if (p->chi == 4) return set_err(TNC_E_DOMAIN, "the complex128 reference sweep covers bond dimension 2 only");
  if (n_batches == 0) return TNC_OK;
  std::shared_ptr<DevSched> ds;
  int rc = get_dev_sched(*p, k, &ds);
  if (rc) return rc;
  return run_c128(*p, *ds, n_batches, d_bits, k, d_out, d_workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

int tnc_amplitudes_host(tnc_plan_t plan, int32_t n_batches, const uint8_t* bits, int32_t k, int32_t storage,
                        tnc_c128* out) {
  Plan* p = get(plan);
  if (!p || n_batches < 0 || (n_batches > 0 && (!bits || !out))) return set_err(TNC_E_INVALID, "bad argument");
  if (n_batches == 0) return TNC_OK;
  uint64_t ws = 0;
  int rc = tnc_workspace_bytes(plan, k, n_batches, storage, &ws);
  if (rc) return rc;
  const size_t nbits = (size_t)n_batches * p->n, nout = (size_t)n_batches << k;
  if (p->opt.mem_cap_bytes) {
    // at most the cap in all: bits, output, and a workspace for as many
    // batches as fit (tnc_amplitudes runs the batches in groups)
    const uint64_t per = ws / (uint64_t)n_batches, fixed = nbits + nout * 16 + 512;
    if (fixed + per > p->opt.mem_cap_bytes) return set_err(TNC_E_NOMEM, "one batch does not fit in mem_cap_bytes");
    ws = std::min<uint64_t>(ws, (p->opt.mem_cap_bytes - fixed) / per * per);
  }
  uint8_t* d_bits = nullptr;
  tnc_c128* d_out = nullptr;
  void* d_ws = nullptr;
  hipStream_t st = nullptr;
  hipError_t e;
  // a stream of this call's own: waiting for it never waits for (or fails
  // on) other work on the device
  auto cleanup = [&]() {
    if (st) (void)hipStreamSynchronize(st);
    if (d_bits) (void)hipFree(d_bits);
    if (d_out) (void)hipFree(d_out);
    if (d_ws) (void)hipFree(d_ws);
    if (st) (void)hipStreamDestroy(st);
  };
  if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess) {
    st = nullptr;
    return hip_err(e, "hipStreamCreate");
  }
  if ((e = hipMalloc((void**)&d_bits, nbits)) != hipSuccess || (e = hipMalloc((void**)&d_out, nout * 16)) != hipSuccess ||
      (e = hipMalloc(&d_ws, ws)) != hipSuccess) {
    cleanup();
    return set_err(TNC_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  if ((e = hipMemcpyAsync(d_bits, bits, nbits, hipMemcpyHostToDevice, st)) != hipSuccess) {
    cleanup();
    return hip_err(e, "hipMemcpyAsync");
  }
  rc = tnc_amplitudes(plan, n_batches, d_bits, k, storage, d_out, d_ws, ws, st);
  if (rc == TNC_OK) {
    if ((e = hipMemcpyAsync(out, d_out, nout * 16, hipMemcpyDeviceToHost, st)) != hipSuccess)
      rc = hip_err(e, "hipMemcpyAsync");
    else if ((e = hipStreamSynchronize(st)) != hipSuccess)
      rc = hip_err(e, "kernel execution");
  }
  cleanup();
  return rc;
}

int tnc_logxeb(const tnc_c128* d_amp, int32_t n_batches, int32_t k, const int32_t* d_select, int32_t n_qubits,
               double* d_result, void* stream) {
  if (!d_amp || !d_result || n_batches <= 0 || k < 0 || k > 30) return set_err(TNC_E_INVALID, "bad argument");
  hipError_t e = launch_logxeb(reinterpret_cast<const double2*>(d_amp), n_batches, k, d_select, n_qubits, d_result,
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_err(e, "logxeb launch");
  return TNC_OK;
}

int tnc_sample_batched(const tnc_c128* d_amp, int32_t n_batches, int32_t k, const double* d_u, int32_t* d_b,
                       double* d_q, void* stream) {
  if (n_batches < 0 || k < 0 || k > 10) return set_err(TNC_E_INVALID, "need n_batches >= 0 and 0 <= k <= 10");
  if (n_batches == 0) return TNC_OK;
  if (!d_amp || !d_u || !d_b || !d_q) return set_err(TNC_E_INVALID, "null argument");
  hipError_t e = launch_sample_batched(reinterpret_cast<const double2*>(d_amp), n_batches, k, d_u, d_b, d_q,
                                       static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_err(e, "batched sampling launch");
  return TNC_OK;
}

int tnc_frugal_accept(const tnc_c128* d_amp, int64_t count, int32_t n_qubits, double M, const double* d_u,
                      uint8_t* d_accept, double* d_z, void* stream) {
  if (count < 0 || n_qubits < 1 || n_qubits > 1000 || !(M > 0.0) || !std::isfinite(M))
    return set_err(TNC_E_INVALID, "need count >= 0, 1 <= n_qubits <= 1000 and a finite M > 0");
  if (count == 0) return TNC_OK;
  if (!d_amp || !d_u || !d_accept || !d_z) return set_err(TNC_E_INVALID, "null argument");
  hipError_t e = launch_frugal_accept(reinterpret_cast<const double2*>(d_amp), (long long)count, n_qubits, M, d_u,
                                      d_accept, d_z, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_err(e, "frugal rejection launch");
  return TNC_OK;
}

int tnc_profile_begin(void) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  for (auto& r : g_prof.recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  g_prof.recs.clear();
  g_prof.active = true;
  return TNC_OK;
}

int tnc_profile_end(tnc_profile* out) {
  if (!out) return set_err(TNC_E_INVALID, "null argument");
  std::vector<Profiler::Rec> recs;
  {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.active = false;
    recs.swap(g_prof.recs);
  }
  std::memset(out, 0, sizeof(*out));
  int rc = TNC_OK;
  std::vector<std::pair<int, double>> last;
  for (auto& r : recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e != hipSuccess && rc == TNC_OK) rc = hip_err(e, "event timing");
    last.emplace_back(r.cls, (double)ms);
    if (r.cls == 0) out->init_ms += ms, out->init_launches++;
    if (r.cls == 1) out->pass_ms += ms, out->pass_launches++, out->pass_bytes += r.bytes;
    if (r.cls == 2) out->late_ms += ms, out->late_launches++;
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof_last.swap(last);
  return rc;
}

int tnc_profile_launches(int32_t* cls, double* ms, int64_t cap, int64_t* n) {
  if (!n || cap < 0 || (cap > 0 && (!cls || !ms))) return set_err(TNC_E_INVALID, "bad argument");
  std::lock_guard<std::mutex> lk(g_prof.mu);
  *n = (int64_t)g_prof_last.size();
  for (int64_t i = 0; i < cap && i < *n; ++i) {
    cls[i] = g_prof_last[(size_t)i].first;
    ms[i] = g_prof_last[(size_t)i].second;
  }
  return TNC_OK;
}

int tnc_plan_passes(tnc_plan_t plan, int32_t k, int32_t* out, int32_t cap, int32_t* n_passes) {
  Plan* p = get(plan);
  if (!p || !n_passes || cap < 0 || (cap > 0 && !out)) return set_err(TNC_E_INVALID, "bad argument");
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(*p, k, &s, &err);
  if (rc) return set_err(rc, err);
  *n_passes = (int32_t)s->passes.size();
  for (int32_t i = 0; i < cap && i < *n_passes; ++i) {
    const Pass& ps = s->passes[(size_t)i];
    int fused = 0;
    for (const Phase& ph : ps.phases) fused += (ph.mf == 1 || ph.mf == 3) ? 1 : 0;
    int32_t* o = out + 7 * (size_t)i;
    o[0] = ps.w.lo_bits;
    o[1] = ps.w.win_lo;
    o[2] = ps.w.win_len;
    o[3] = ps.R;
    o[4] = ps.op_end - ps.op_begin;
    o[5] = (int32_t)ps.phases.size();
    o[6] = fused;
  }
  return TNC_OK;
}

void tnc_release(tnc_plan_t plan) {
  if (!plan) return;
  Plan* p = plan->plan.get();
  if (p && p->device && p->device_free) p->device_free(p->device);
  delete plan;
}

const char* tnc_strerror(int code) {
  switch (code) {
    case TNC_OK: return "ok";
    case TNC_E_INVALID: return "invalid argument";
    case TNC_E_DOMAIN: return "outside the supported domain";
    case TNC_E_RANK: return "entangler operator Schmidt rank above 2";
    case TNC_E_NOMEM: return "out of memory";
    case TNC_E_DEVICE: return "device error";
    default: return "unknown status";
  }
}

const char* tnc_last_error(void) { return g_err.c_str(); }

int tnc_debug_lds_conflicts(tnc_plan_t plan, int32_t k, int64_t* stats) {
  Plan* p = get(plan);
  if (!p || !stats) return set_err(TNC_E_INVALID, "bad argument");
  std::shared_ptr<Schedule> s;
  std::string err;
  int rc = get_schedule(*p, k, &s, &err);
  if (rc) return set_err(rc, err);
  HostTables t;
  rc = build_tables(*p, *s, &t, &err);
  if (rc) return set_err(rc, err);
  // lanes 0..63 of a wave (thread index = lane); slot of register entry 0
  // (the other entries differ by a constant XOR); a group of g lanes
  // conflicts when two of its lanes meet the same slot modulo g
  int64_t phases = 0, c16 = 0, c32 = 0;
  for (const PassHost& ph : t.passes) {
    const int TB = ph.w.tile_bits() - ph.R;
    for (int q = 0; q < ph.n_phases; ++q) {
      const uint32_t* po = t.poffs.data() + (size_t)(ph.phase_off + q) * kPhaseOffs;
      const int lanes = std::min(64, 1 << TB);
      uint32_t slot[64];
      for (int l = 0; l < lanes; ++l) {
        uint32_t vb = 0;
        for (int b = 0; b < TB; ++b)
          if ((l >> b) & 1) vb ^= po[kPhaseEntries + b];
        slot[l] = (vb ^ po[0]) >> 3;
      }
      auto conflicted = [&](int g) {
        for (int l0 = 0; l0 + g <= lanes; l0 += g)
          for (int a = l0; a < l0 + g; ++a)
            for (int b = a + 1; b < l0 + g; ++b)
              if ((slot[a] & (uint32_t)(g - 1)) == (slot[b] & (uint32_t)(g - 1))) return true;
        return false;
      };
      ++phases;
      if (lanes >= 16 && conflicted(16)) ++c16;
      if (lanes >= 32 && conflicted(32)) ++c32;
    }
  }
  stats[0] = phases;
  stats[1] = c16;
  stats[2] = c32;
  return TNC_OK;
}

int tnc_debug_execute_host(tnc_plan_t plan, int32_t n_batches, const uint8_t* bits, int32_t k, tnc_c128* out) {
  Plan* p = get(plan);
  if (!p || !bits || !out || n_batches < 0) return set_err(TNC_E_INVALID, "bad argument");
  std::vector<cd> o((size_t)n_batches << k);
  std::string err;
  int rc = execute_host(*p, k, n_batches, bits, o.data(), &err);
  if (rc) return set_err(rc, err);
  for (size_t i = 0; i < o.size(); ++i) out[i] = tnc_c128{o[i].real(), o[i].imag()};
  return TNC_OK;
}

int tnc_debug_emulate_device(tnc_plan_t plan, int32_t n_batches, const uint8_t* bits, int32_t k, int32_t storage,
                             tnc_c128* out) {
  Plan* p = get(plan);
  if (!p || !bits || !out || n_batches < 0) return set_err(TNC_E_INVALID, "bad argument");
  std::vector<cd> o((size_t)n_batches << k);
  int rc = emulate(*p, k, n_batches, bits, storage, o.data());
  if (rc) return rc;
  for (size_t i = 0; i < o.size(); ++i) out[i] = tnc_c128{o[i].real(), o[i].imag()};
  return TNC_OK;
}

}  // extern "C"
