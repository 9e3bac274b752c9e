// Host-side planner of the temporal-boundary contraction.
//
// The planner fixes the unsliced sweep of the deterministic temporal-state
// contraction (Sec. 3.1, Alg. 1) and of its batched extension with k open
// output legs (Sec. 4.3, Alg. 2) for an open-chain brickwork circuit whose
// entanglers have operator Schmidt rank <= 2 (Sec. 2.1-2.2), and, for
// entanglers of rank 4 (generic two-qubit gates, Sec. 6.2 "Effect of bond
// dimension"), the sweep of bond dimension four described in plan4.cpp
// (even depth, k = 0).
//
// Lowering used here (derived from the tensor network of Sec. 2.2):
//  * every entangler on (q, q+1) is written as
//        U = (post (x) I) [ sum_a |a><a| (x) C_a ] (pre (x) I),
//    a copy tensor on the upper qubit q and a 2x2 C_a on the lower one;
//  * the boundary tensor after rows 0..r is indexed by the worldline values of
//    qubit r at the crossing layers of cut (r|r+1), one binary slot per
//    crossing in layer order ("slot s" = bit s of the linear index);
//  * absorbing a middle row is a staircase of h two-slot updates
//        B'[a@c, x@t] = sum_b K_a[x][b] B[a@c, b@t]
//    (a 2x2 on slot t selected by the bit of the neighbouring slot c), run
//    upward in slot index when the row's first event consumes a slot
//    ("ascending") and downward otherwise; odd depth adds the top-slot
//    remove / expand turn of the proof's case (b) in Prop. constructive-memory.
//  * for k >= 1 the fixed region ends at row n-k-1; the early region of the
//    open band is contracted on the host into Z_early[u][t] (2^k x 2^k), joined
//    with the boundary tensor over its first k slots, and the late layers are
//    absorbed in causal order (Alg. 2 and Prop. batched width).
#pragma once

#include <complex>
#include <cstdint>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

namespace tnc {

using cd = std::complex<double>;

struct M2 {
  cd a[4] = {cd(1), cd(0), cd(0), cd(1)};  // row-major [out][in]
  cd& operator()(int r, int c) { return a[2 * r + c]; }
  const cd& operator()(int r, int c) const { return a[2 * r + c]; }
  static M2 zero() {
    M2 m;
    m.a[0] = m.a[3] = 0;
    return m;
  }
};
M2 operator*(const M2& x, const M2& y);

// U = (post (x) I) [sum_a P_a (x) C_a] (pre (x) I) on (upper, lower).
struct Split {
  M2 pre, post;
  M2 C[2];
};

enum SweepKind { OP_CU = 0, OP_DUP = 1, OP_D4 = 2, OP_D4H = 3 };

// One update of the boundary tensor.  OP_CU: for every index whose control
// bit is c (c = 0 if control < 0), the pair (b0, b1) along `target` becomes
// mat[var][c] * (b0, b1).  OP_DUP: the half with target bit 1 is overwritten
// by the half with target bit 0 (the top-slot expand of odd depth).
// OP_D4 + OP_D4H (always adjacent, in this order): one dense 4x4 M on the
// slot pair (target, pair): the four entries with u = bit(target) +
// 2 bit(pair) become M (b_0 .. b_3); OP_D4 holds rows 0 and 1 of M, OP_D4H
// rows 2 and 3, as mat[var][r].a[c] = M[row r of the half][c] (c = 0..3).
// var = 2*x[xrow0] + x[xrow1] (an unused xrow reads as 0).
struct SweepOp {
  int kind = OP_CU;
  int target = -1;
  int control = -1;
  int pair = -1;  // OP_D4 / OP_D4H: the upper slot of the pair
  int xrow[2] = {-1, -1};
  M2 mat[4][2];
  int row = -1;
};

enum LateKind { L_U1 = 1, L_G4 = 2, L_REMOVE = 3, L_DOT = 4, L_OUT = 5, L_REMOVE2 = 6 };

// Late program on a state of s bits (s = k for k >= 1, s = 1 for k = 0):
//  L_U1 a:       2x2 on state bit a (m: 4 entries)
//  L_G4 a:       4x4 on state bits (a, a+1), basis 2*bit_a + bit_{a+1} (m: 16)
//  L_REMOVE:     sum out the lowest remaining slot u with C_u on state bit 0
//                (m: C_0 then C_1, 8 entries; with xrow >= 0 a second set of
//                8 for output bit x[xrow] = 1)
//  L_REMOVE2:    sum out the two lowest remaining slots (u0 the lower, u1)
//                with C_u, u = u0 + 2 u1, on state bit 0 (m: C_0..C_3, 16)
//  L_DOT xrow:   k = 0 only: amplitude = sum_w f_x[w] state[w]  (m: f_0, f_1)
//  L_OUT:        k >= 1: out[b] = state[bit-reverse_k(b)]
struct LateOp {
  int kind = 0;
  int a = -1;
  int xrow = -1;
  std::vector<cd> m;
};

// A pass tile: global slots [0, lo_bits) and [win_lo, win_lo + win_len).
struct Window {
  int lo_bits = 0, win_lo = 0, win_len = 0;
  int tile_bits() const { return lo_bits + win_len; }
  bool contains(int s) const { return s < lo_bits || (s >= win_lo && s < win_lo + win_len); }
  int local(int s) const { return s < lo_bits ? s : s - win_lo + lo_bits; }
  int global(int l) const { return l < lo_bits ? l : l - lo_bits + win_lo; }
};

constexpr int kMaxReg = 8;

// Boundary tensors the device path runs: up to 2^40 entries.  Bond-four
// plans are built (width, cost, schedule; no device tables) up to width 69,
// the n = d = 70 point of Sec. 6.2 (the late buffers' byte counts stay below
// 2^64 there).
constexpr int kMaxDeviceWidth = 40;
constexpr int kMaxPlanWidth = 69;

// Register bits of a pass with 2^T-entry tiles: at most R, and at least one
// bit left for the thread part so that op 0's control is never a register.
inline int pass_reg_bits(int R, int T) { return T <= 1 ? 1 : (R < T - 1 ? R : T - 1); }

constexpr int kMaxThreadBits = 9;

// A register phase.  mf = 0: the canonical staircase on the vector ALUs.
// mf = 1: its first three updates fused into one complex 8x8 per value of
// op 0's control, on the matrix cores, with targets reg[0] (a register bit)
// and tpos[4], tpos[5] (lane bits 4 and 5); op 0's control, if any, is
// reg[R-1]; the staircase goes on on the vector ALUs: update 3 targets
// reg[1] under tpos[5], update b > 3 reg[b-2] under reg[b-3].  mf = 2: a
// dense phase of up to four 4x4 updates (OP_D4 + OP_D4H each), update g on
// register bits dreg[g] (its lower, upper slot).  tpos[t] is the tile bit
// of thread bit t.
struct Phase {
  int op_begin = 0, op_end = 0;
  int reg[kMaxReg] = {0};  // local tile bits held in registers, in register-bit order
  int mf = 0;
  int tpos[kMaxThreadBits] = {0};
  int dreg[4][2] = {};     // dense phases: register bits of update g's lower and upper slot
};

struct Pass {
  Window w;
  int op_begin = 0, op_end = 0;
  int R = 0;  // register bits of this pass's phases
  std::vector<Phase> phases;
};

struct Options {
  int max_tile_bits = 13;   // tile of one pass: 2^max_tile_bits entries
  int reg_bits = 5;         // entries per thread = 2^reg_bits
  int low_bits = 4;         // contiguous low slots kept in every non-bottom tile
  int math = 0;             // 0: vector ALU updates; 2: runs of three updates fused into 8x8 products
                            // on the matrix cores
  int late_fold = 0;        // removals folded into the join launch (0 auto, -1 none, 1..8)
  int reg_adapt = 0;        // 1: a pass uses reg_bits - 1 when that needs no more phases; 0: never
  int bond = 0;             // entangler bond dimension of the lowering: 0 the smallest that holds
                            // every gate, 2, or 4
  uint64_t mem_cap_bytes = 0;  // device memory per call (0: no cap)
};

// Everything that depends on k (the number of open output legs).
struct Schedule {
  int k = 0;
  int last_fixed_row = 0;  // sweep covers rows 1..last_fixed_row (row 0 is the build-up)
  int m_fix = 0;           // live slots after the fixed sweep
  std::vector<SweepOp> ops;
  std::vector<Pass> passes;
  int reg_bits = 5;
  int s_bits = 1;            // late state bits
  int join_u_bits = 0;       // slots consumed by the join (k, or 0 for k = 0)
  std::vector<cd> join;      // k>=1: Z_early[u*2^k + t]; k=0: start vector v[2]
  std::vector<LateOp> late;  // after the join
  int n_remove = 0;
  double log2_cost = 0;
  int width = 0;
};

struct Plan {
  int n = 0, d = 0, h = 0;
  int chi = 2;                           // bond dimension of the lowering (2 or 4)
  bool spatial = false;                  // bond 4 with n below the temporal width: the boundary
                                         // is the n-qubit state, swept layer by layer (plan4.cpp)
  int parity1 = 1;                       // upper-qubit parity of layer 1's pairs
  std::vector<M2> one;                   // (d+1)*n one-qubit gates
  std::vector<std::vector<int>> X;       // X[c] = crossing layers of cut c, ascending
  std::vector<Split> split;              // per (layer-1)*(n-1) + cut (pattern pairs only)
  std::vector<std::vector<cd>> g4;       // original 4x4 per (layer-1)*(n-1)+cut (identity if absent)
  // row 0 build-up: B0[a_0..a_{m-1}] = v[a_0] prod_j seg_j[a_j][a_{j-1}] f_x[a_{m-1}]
  int m0 = 0;
  cd init_v[2];
  std::vector<M2> init_seg;              // m0-1 entries, seg_j at index j-1
  cd init_f[2][2];                       // [x][a]
  std::vector<std::vector<SweepOp>> row_ops;  // row_ops[r] for middle rows 1..n-2
  std::vector<int> row_ascending;        // per row (1..n-2)
  Options opt;

  std::mutex mu;
  std::map<int, std::shared_ptr<Schedule>> sched;

  // device-side state is owned by the executor (opaque here)
  void* device = nullptr;
  void (*device_free)(void*) = nullptr;
};

struct Gate2In {
  int layer, q, kind;
  const cd* m;  // 16 entries for DENSE4
};

// Build a plan.  Returns 0 or a negative status; `err` receives a message.
int build_plan(int n, int d, const cd* one_qubit, int n_gate2, const Gate2In* gates,
               const Options& opt, std::unique_ptr<Plan>* out, std::string* err);

// The schedule for k open legs (cached in the plan).
int get_schedule(Plan& p, int k, std::shared_ptr<Schedule>* out, std::string* err);

// FP64 host execution of the plan's own tables (planner self-check; the GPU
// path never calls this).  out: n_batches * 2^k amplitudes.
int execute_host(Plan& p, int k, int n_batches, const uint8_t* bits, cd* out, std::string* err);

// The bond-dimension-four lowering (plan4.cpp): fills row 0's build-up,
// the row updates and p.h of a plan whose gates, one-qubit layers and
// crossing lists are set.
int build_rows4(Plan& p, std::string* err);
// Its late program (k = 0: the last row's absorption).
int build_late4(const Plan& p, Schedule& s, std::string* err);

// Decompose a 4x4 (basis 2*x_upper + x_lower) into copy-on-upper form.
// Returns 0, or TNC_E_RANK-equivalent (-3) when the operator Schmidt rank
// exceeds 2 or the form does not exist.
int split_entangler(const cd* u16, Split* s, std::string* err);

}  // namespace tnc
