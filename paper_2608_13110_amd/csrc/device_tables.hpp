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

// Storage of the boundary tensor in HBM.  C64: complex64 (re, im floats).
// F16 / BF16: each entry is two 16-bit halves (re low, im high) of the value
// divided by its block's FP32 power-of-two scale; a block is the 4096
// entries (fewer in tiles below 2^12) that one tile wrote together.
enum StoreMode : int { STORE_C64 = 0, STORE_F16 = 1, STORE_BF16 = 2 };

// How the block scales of a 16-bit tensor were laid out by their writer:
// tiles of the slots [0, lo_bits) and [win_lo, win_lo + win_len) (tile_bits
// slots in all), each split into blocks of 2^blk_bits entries along its
// highest local bits.  Scale slot of entry g (index within its batch):
//   (tile(g) << (tile_bits - blk_bits)) | (local(g) >> blk_bits).
struct ScaleMap {
  int lo_bits, win_lo, win_len, tile_bits, blk_bits;
};

// One boundary-tensor update inside a pass (16 bytes).  Within a register
// phase, op b acts on the pairs along register bit b; ops b >= 1 are
// controlled by register bit b-1, op 0 by a thread bit (DevPhase.cloc0) or
// by nothing, or op 0 is the phase's DUP.  cloc: op 0's control as a local
// tile bit (-1: none; a planner record, not read by the kernels).
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
// bits reg[0..R-1] held in registers (register bit b <-> local bit reg[b]);
// the thread bits sit on the other tile bits in the order the planner chose
// (their LDS offsets are in the phase's offset table).  first_dup: op 0
// copies the register half with bit 0 clear onto the half with bit 0 set (the
// top-slot expand of odd depth).  cloc0: the thread bit whose value controls
// op 0 (-1: uncontrolled).
struct DevPhase {
  int32_t op_begin;
  int8_t n_ops;
  int8_t first_dup;
  int8_t reg[8];
  int8_t cloc0;
  int8_t pad;   // 1: a fused phase (three updates as one 8x8 on the matrix cores);
                // 2: a dense phase (n_ops / 2 dense 4x4 updates in order, update g
                // on the register-bit pair coded in bits 4g..4g+3 of reg[6..7]
                // (dense_pair_code), its matrix rows in ops op_begin + 2g and
                // op_begin + 2g + 1)
};
static_assert(sizeof(DevPhase) == 16, "DevPhase layout");

// Launch parameters of one pass (a kernel argument).
//   mats:  per op [var 4][ctl 2][k00 k01 k10 k11 as (re, im)]  (16 floats / var)
// A phase's LDS offset table: one word per register entry (up to 2^5), then
// one per thread bit: the offset of the tile bit it sits on.
constexpr int kPhaseEntries = 32;
constexpr int kPhaseOffs = 48;
// Matrix-core operands of a fused phase: [control 2][lane 64] float4.
constexpr int kFusedWords = 128;

struct PassArgs {
  const DevPhase* phases;
  // per phase of the pass: kPhaseOffs byte offsets in the LDS tile of the
  // phase's register entries (tile index with register bits = the entry's
  // bits, after the LDS swizzle)
  const uint32_t* poffs;
  // per phase of the pass: kFusedWords float4, the fused phases' matrix-core
  // operands (null when the pass tables have no fused phase)
  const float4* fmats;
  // the batch's own matrices: rmats[b][op][ctl][k00 k01 k10 k11 as (re, im)]
  // (the variant of every op already picked from batch b's output bits)
  const float* rmats;
  long long rstride;     // floats per batch in rmats
  float2* B;             // boundary tensors, batch stride 2^h entries
  const uint8_t* bits;   // output bits, batch stride n
  int n_phases;
  int n;
  int h;                 // log2 batch stride
  int T;                 // tile bits
  int lo_bits, win_lo, win_len;
  int n_tiles;           // batches << (h - T)
  int store;             // StoreMode of B
  int kind;              // phase forms: 0 bond two, 1 bond four (dense)
  // 16-bit storage only: scales read (written by the previous writer, laid
  // out by in_map) and written (laid out by this pass's own tiles); batch
  // stride scale_stride floats
  const float* scale_in;
  float* scale_out;
  long long scale_stride;
  ScaleMap in_map;
};

// Launch parameters of a late-phase folded contraction:
//   out[b][r][c] = sum_kk in[b][r][kk] * J[var(b)][kk][c]
struct LateArgs {
  const void* in;        // boundary tensor (first launch, storage `store`) or double2
  double2* out;
  const double2* J;      // [vars][K][N]
  const uint8_t* bits;
  long long in_batch_stride;   // elements
  long long out_batch_stride;  // elements
  int M, K, N;
  int n_batches;
  int xrow;              // -1: one variant; else var = x[xrow]
  int n;
  int store;             // StoreMode of `in` (first launch)
  const float* scale_in; // 16-bit storage: block scales, laid out by in_map
  long long scale_stride;
  ScaleMap in_map;
};

// One op of a late program (device copy of LateOp, plan.hpp).
struct LateOpDev {
  int32_t kind;  // 1 U1, 2 G4, 3 REMOVE (xrow >= 0: m[8..16) when x[xrow] = 1), 6 REMOVE2
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

// Resolution of the op variants of a batch group: for batch b and op o,
// rmats[b][o][0..16) = mats[(o*4 + var(b, o))*16 .. +16).
struct ResolveArgs {
  const DevOp* ops;
  const float* mats;
  const uint8_t* bits;
  float* rmats;
  long long rstride;
  int n_ops;
  int n;
  int n_batches;
};

// One boundary update of the unfused complex128 reference sweep (a test
// path, not the hot loop): the pair along `target` of every index becomes
// m[var][c] * pair (c = the control bit, var = 2 x[xrow0] + x[xrow1]), or
// (kind 1) the half with target bit 1 becomes a copy of the half with 0.
struct Op64 {
  int32_t kind;
  int32_t target, control;
  int32_t xrow0, xrow1;
  int32_t pad[3];
  double2 m[4][2][4];  // [var][ctl][k00 k01 k10 k11]
};

struct Op64Args {
  double2* B;            // complex128 boundary tensors, batch stride 2^h entries
  const uint8_t* bits;
  const Op64* op;
  int h;
  int n;
  int n_batches;
};

struct InitArgs {
  float2* B;             // complex64 tensor, or the 16-bit tensor (store != C64)
  const uint8_t* bits;
  const double2* seg;    // (m0-1) x 4 entries, seg_j[a_j][a_{j-1}] row-major
  double2 v[2];
  double2 f[2][2];
  int m0;
  int h;
  int n;
  int n_batches;
  int store;             // StoreMode of B
  float* scale_out;      // 16-bit storage: one scale per 2^blk_bits consecutive entries
  long long scale_stride;
  int blk_bits;
};

}  // namespace tnc
