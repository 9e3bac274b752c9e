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

// One boundary-tensor update inside a pass (16 bytes).  Within a register
// phase, op b acts on the pairs along register bit b; ops b >= 1 are
// controlled by register bit b-1, op 0 by the tile bit `cloc` of the thread
// part (cloc < 0: no control), or op 0 is the phase's DUP.
// Matrices: mats[(mat*4 + var)*16 ..+16): [ctl][k00 k01 k10 k11 as (re, im)],
// var = 2*x[xrow0] + x[xrow1] (an absent row reads as 0).
struct DevOp {
  int16_t xrow0;
  int16_t xrow1;
  int8_t cloc;
  int8_t pad0[3];
  int32_t mat;
  int32_t pad1;
};
static_assert(sizeof(DevOp) == 16, "DevOp layout");

// A register phase: n_ops consecutive ops from op_begin, run with local tile
// bits reg[0..R-1] held in registers (register bit b <-> local bit reg[b]).
// first_dup: op 0 copies the register half with bit 0 clear onto the half
// with bit 0 set (the top-slot expand of odd depth).
struct DevPhase {
  int32_t op_begin;
  int8_t n_ops;
  int8_t first_dup;
  int8_t reg[8];
  int16_t pad;
};
static_assert(sizeof(DevPhase) == 16, "DevPhase layout");

// Launch parameters of one pass (a kernel argument).
//   mats:  per op [var 4][ctl 2][k00 k01 k10 k11 as (re, im)]  (16 floats / var)
//   mrows: per op [var 4][ctl 2][row 4][4]: the real 4x4 form of the same
//          2x2, acting on (re b0, im b0, re b1, im b1); row r feeds the
//          matrix-core update's A operand of lane r (mod 4)
struct PassArgs {
  const DevPhase* phases;
  const DevOp* ops;
  const float* mats;
  const float4* mrows;
  float2* B;             // boundary tensors, batch stride 2^h entries
  const uint8_t* bits;   // output bits, batch stride n
  int n_phases;
  int n;
  int h;                 // log2 batch stride
  int T;                 // tile bits
  int lo_bits, win_lo, win_len;
  int n_tiles;           // batches << (h - T)
  int mfma;              // register-controlled updates on the matrix cores
  int pipeline;          // persistent blocks prefetching the next tile
  int op_begin;          // this pass's ops: [op_begin, op_begin + n_ops)
  int n_ops;
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
