// Kernel launchers (host side) and the shared per-thread helpers of the
// pass kernel, usable on host and device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device_tables.hpp"

namespace tnc {

constexpr int kBlock = 256;

// LDS placement of tile entry i: bits 1..5 are XORed with bits 6..10 and
// 11..15 so that strided register layouts spread over the banks.  The map is
// linear over GF(2): swz(a ^ b) = swz(a) ^ swz(b); bit 0 is kept, so the
// pair (2i, 2i+1) stays adjacent and ordered.
TNC_HD inline uint32_t swz(uint32_t i) { return i ^ ((((i >> 6) ^ (i >> 11)) & 31u) << 1); }

// Offset of local tile entry i inside its batch, without the block part.
TNC_HD inline uint64_t tile_offset(uint32_t i, int lo_bits, int win_lo) {
  const uint32_t lo_mask = (1u << lo_bits) - 1u;
  return (uint64_t)(i & lo_mask) | ((uint64_t)(i >> lo_bits) << win_lo);
}

// Offset of block `blk` (the slots outside the tile) inside its batch.
TNC_HD inline uint64_t block_offset(uint64_t blk, int lo_bits, int win_lo, int win_len) {
  const int gap = win_lo - lo_bits;
  const uint64_t low = blk & ((1ull << gap) - 1ull);
  const uint64_t high = blk >> gap;
  return (low << lo_bits) | (high << (win_lo + win_len));
}

// Scatter the bits of `x` into the set bits of `mask` (ascending).
TNC_HD inline uint32_t pdep32(uint32_t x, uint32_t mask) {
  uint32_t r = 0;
  int b = 0;
  while (mask) {
    const uint32_t low = mask & (~mask + 1u);
    if ((x >> b) & 1u) r |= low;
    mask &= mask - 1u;
    ++b;
  }
  return r;
}

// out = K * (b0, b1) with K = [k0 k1; k2 k3] given as 8 floats (re, im).
TNC_HD inline void cmat2(const float* __restrict__ k, float2& b0, float2& b1) {
  float2 o0, o1;
  o0.x = k[0] * b0.x - k[1] * b0.y + k[2] * b1.x - k[3] * b1.y;
  o0.y = k[0] * b0.y + k[1] * b0.x + k[2] * b1.y + k[3] * b1.x;
  o1.x = k[4] * b0.x - k[5] * b0.y + k[6] * b1.x - k[7] * b1.y;
  o1.y = k[4] * b0.y + k[5] * b0.x + k[6] * b1.y + k[7] * b1.x;
  b0 = o0;
  b1 = o1;
}

template <int R, int A, int C>
TNC_HD inline void op_reg(float2 (&v)[1 << R], const float* __restrict__ m) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << A)) continue;
    cmat2(m + 8 * ((i >> C) & 1), v[i], v[i | (1 << A)]);
  }
}

template <int R, int A>
TNC_HD inline void op_sel(float2 (&v)[1 << R], const float* __restrict__ k) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << A)) continue;
    cmat2(k, v[i], v[i | (1 << A)]);
  }
}

template <int R, int A>
TNC_HD inline void op_dup(float2 (&v)[1 << R]) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << A)) continue;
    v[i | (1 << A)] = v[i];
  }
}

template <int R, int A, int C>
struct RegDispatch {
  static TNC_HD inline void run(float2 (&v)[1 << R], int a, int c, const float* __restrict__ m) {
    if (a == A && c == C) {
      if constexpr (A != C) op_reg<R, A, C>(v, m);
      return;
    }
    if constexpr (C + 1 < R) {
      RegDispatch<R, A, C + 1>::run(v, a, c, m);
    } else if constexpr (A + 1 < R) {
      RegDispatch<R, A + 1, 0>::run(v, a, c, m);
    }
  }
};

template <int R, int A>
struct SelDispatch {
  static TNC_HD inline void run(float2 (&v)[1 << R], int a, const float* __restrict__ k, bool dup) {
    if (a == A) {
      if (dup) op_dup<R, A>(v);
      else op_sel<R, A>(v, k);
      return;
    }
    if constexpr (A + 1 < R) SelDispatch<R, A + 1>::run(v, a, k, dup);
  }
};

// Apply the ops of one phase to a thread's registers.
//   tb: the thread part of the local tile index in this phase.
//   xb: the output bits of this tile's batch.
template <int R>
TNC_HD inline void run_phase_ops(float2 (&v)[1 << R], const DevPhase& P, const DevOp* __restrict__ ops,
                                 const float* __restrict__ mats, const uint8_t* __restrict__ xb,
                                 uint32_t tb) {
  for (int o = P.op_begin; o < P.op_end; ++o) {
    const DevOp op = ops[o];
    int var = 0;
    if (op.xrow0 >= 0) var += 2 * xb[op.xrow0];
    if (op.xrow1 >= 0) var += xb[op.xrow1];
    const float* m = mats + ((size_t)op.mat * 4 + var) * 16;
    if (op.kind == 1) {
      SelDispatch<R, 0>::run(v, op.treg, m, true);
    } else if (op.creg >= R) {
      const int ctl = op.cloc >= 0 ? int((tb >> op.cloc) & 1u) : 0;
      SelDispatch<R, 0>::run(v, op.treg, m + 8 * ctl, false);
    } else {
      RegDispatch<R, 0, 0>::run(v, op.treg, op.creg, m);
    }
  }
}

// Launchers (kernels.hip).
hipError_t launch_init(const InitArgs& a, hipStream_t s);
hipError_t launch_pass(const PassArgs& a, int R, hipStream_t s);
hipError_t launch_late(const LateArgs& a, bool in_c64, hipStream_t s);
hipError_t launch_late_ops(const LateOpsArgs& a, hipStream_t s);
hipError_t launch_logxeb(const double2* amps, int n_batches, int k, const int32_t* sel, int n_qubits,
                         double* result, hipStream_t s);

// Host emulation of the pass kernel (exact thread / LDS mapping), for tests.
void emulate_pass_host(const PassArgs& a, int R);

}  // namespace tnc
