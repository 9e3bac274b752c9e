// Device-resident tables of a prepared schedule, shared by host and kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#if defined(__HIPCC__)
#define TNC_HD __host__ __device__ __attribute__((always_inline))
#else
#define TNC_HD
#endif

namespace tnc {

// One boundary-tensor update inside a pass (16 bytes).
//   kind 0 (CU): pairs along register bit `treg`; the 2x2 is chosen by the
//                control value: register bit `creg` (0..R-1), or, when
//                creg == R, the tile bit `cloc` of the thread part (cloc < 0:
//                no control, value 0).
//   kind 1 (DUP): the register half with bit `treg` = 1 is overwritten by
//                the half with bit `treg` = 0.
// The matrices live at mats[(mat*4 + var)*16 .. +16): [ctl][m00 m01 m10 m11]
// as (re, im) float pairs, var = 2*x[xrow0] + x[xrow1].
struct DevOp {
  int8_t kind;
  int8_t treg;
  int8_t creg;
  int8_t cloc;
  int16_t xrow0;
  int16_t xrow1;
  int32_t mat;
  int32_t pad;
};
static_assert(sizeof(DevOp) == 16, "DevOp layout");

// A register phase of a pass: ops [op_begin, op_end) run with local tile
// bits reg[0..R-1] held in registers (register bit b <-> local bit reg[b]).
struct DevPhase {
  int32_t op_begin;
  int32_t op_end;
  int8_t reg[8];
};
static_assert(sizeof(DevPhase) == 16, "DevPhase layout");

// Launch parameters of one pass (a kernel argument).
struct PassArgs {
  const DevPhase* phases;
  const DevOp* ops;
  const float* mats;
  float2* B;             // boundary tensors, batch stride 2^h entries
  const uint8_t* bits;   // output bits, batch stride n
  int n_phases;
  int n;
  int h;                 // log2 batch stride
  int T;                 // tile bits
  int lo_bits, win_lo, win_len;
  int n_tiles;           // batches << (h - T)
};

// Launch parameters of a late-phase folded contraction:
//   out[b][r][c] = sum_kk in[b][r][kk] * J[var(b)][kk][c]
struct LateArgs {
  const void* in;        // float2 (first launch) or double2
  double2* out;
  const double2* J;      // [vars][K][N]
  const uint8_t* bits;
  long long in_batch_stride;   // elements
  long long out_batch_stride;  // elements
  int M, K, N;
  int n_batches;
  int xrow;              // -1: one variant; else var = x[xrow]
  int n;
};

// One op of a late program (device copy of LateOp, plan.hpp).
struct LateOpDev {
  int32_t kind;  // 1 U1, 2 G4, 3 REMOVE
  int32_t a;
  int32_t xrow;
  int32_t pad;
  double2 m[16];
};

// Launch parameters of a late-program launch: each block takes 2^j rows of
// 2^s state entries (contiguous), runs prog[0..n_prog) with j removals and
// writes one row (or, when final, the amplitudes).
struct LateOpsArgs {
  const double2* in;
  double2* out;
  const uint8_t* bits;
  const LateOpDev* prog;
  long long in_batch_stride;
  long long out_batch_stride;
  long long rows_out;
  int n_prog;
  int s;
  int j;
  int n_batches;
  int n;
  int k;
  int final_kind;  // 0: write the row; 5: amplitudes (bit-reversed index); 4: dot
  int final_xrow;
  double2 dot[2][2];
};

struct InitArgs {
  float2* B;
  const uint8_t* bits;
  const double2* seg;    // (m0-1) x 4 entries, seg_j[a_j][a_{j-1}] row-major
  double2 v[2];
  double2 f[2][2];
  int m0;
  int h;
  int n;
  int n_batches;
};

}  // namespace tnc
