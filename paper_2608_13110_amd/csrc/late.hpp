// Late-phase launch construction (host).
//
// After the fixed sweep the boundary tensor holds m live slots.  The late
// program of a schedule (plan.hpp) is split into device launches:
//  * the first launch is a folded contraction
//        out[r][c] = sum_kk B[r][kk] * J[kk][c],
//    where J combines, in FP64 on the host, the early-region tensor Z_early of
//    Alg. 2 (the join over the first k slots) with the late layers up to and
//    including the first crossing removal (k >= 1), or, for k = 0, the start
//    of the last row's worldline with up to 12 of its crossings;
//  * later launches run the remaining late program (one- and two-qubit
//    gates on the open band and crossing removals) on a state of s bits per
//    row, 2^j rows per block, in FP64 on the device.
#pragma once

#include <vector>

#include "plan.hpp"

namespace tnc {

struct LateFirst {
  int K = 0, N = 0;
  long long M = 0;   // rows per batch
  int xrow = -1;     // >= 0: two variants of J selected by that row's output bit
  int nvar = 1;
  int j = 0;         // removals folded
  bool final = false;
  std::vector<cd> J;  // [nvar][K][N]
};

struct LateOpsLaunch {
  int op_begin = 0, op_end = 0;  // range in Schedule::late (excluding L_OUT / L_DOT)
  int j = 0;                     // removals in this launch (rows per block = 2^j)
  long long rows_in = 0;         // rows per batch of the input
  bool final = false;            // writes the amplitudes
};

struct LatePlan {
  LateFirst first;
  std::vector<LateOpsLaunch> ops;
  int s = 1;
  int final_kind = 0;    // L_OUT or L_DOT (applies to the last launch)
  int final_xrow = -1;
  std::vector<cd> dot;   // L_DOT: f_0, f_1
};

int build_late(const Plan& p, const Schedule& s, LatePlan* out, std::string* err);

}  // namespace tnc
