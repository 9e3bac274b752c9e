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

// Register-resident complex64 entries of a thread: separate real and
// imaginary float arrays (keeps every element promotable to a VGPR).
template <int R>
struct Regs {
  float x[1 << R];
  float y[1 << R];
};

// (b0, b1) <- K (b0, b1) with K = [k0 k1; k2 k3] given as 8 floats (re, im).
TNC_HD inline void cmat2(const float* __restrict__ k, float& x0, float& y0, float& x1, float& y1) {
  const float ox0 = k[0] * x0 - k[1] * y0 + k[2] * x1 - k[3] * y1;
  const float oy0 = k[0] * y0 + k[1] * x0 + k[2] * y1 + k[3] * x1;
  const float ox1 = k[4] * x0 - k[5] * y0 + k[6] * x1 - k[7] * y1;
  const float oy1 = k[4] * y0 + k[5] * x0 + k[6] * y1 + k[7] * x1;
  x0 = ox0;
  y0 = oy0;
  x1 = ox1;
  y1 = oy1;
}

// The variants take and return the register set by value: the branches of
// a dispatch then merge values, never element addresses, so every element
// stays in a VGPR.
template <int R, int A, int C>
TNC_HD inline Regs<R> op_reg(Regs<R> v, const float* __restrict__ m) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << A)) continue;
    const int j = i | (1 << A);
    cmat2(m + 8 * ((i >> C) & 1), v.x[i], v.y[i], v.x[j], v.y[j]);
  }
  return v;
}

template <int R, int A>
TNC_HD inline Regs<R> op_sel(Regs<R> v, const float* __restrict__ k) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << A)) continue;
    const int j = i | (1 << A);
    cmat2(k, v.x[i], v.y[i], v.x[j], v.y[j]);
  }
  return v;
}

template <int R, int A>
TNC_HD inline Regs<R> op_dup(Regs<R> v) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << A)) continue;
    v.x[i | (1 << A)] = v.x[i];
    v.y[i | (1 << A)] = v.y[i];
  }
  return v;
}

template <int R, int A, int C>
struct RegDispatch {
  static TNC_HD inline Regs<R> run(const Regs<R>& v, int a, int c, const float* __restrict__ m) {
    if (a == A && c == C) {
      if constexpr (A != C) return op_reg<R, A, C>(v, m);
      return v;
    }
    if constexpr (C + 1 < R) {
      return RegDispatch<R, A, C + 1>::run(v, a, c, m);
    } else if constexpr (A + 1 < R) {
      return RegDispatch<R, A + 1, 0>::run(v, a, c, m);
    }
    return v;
  }
};

template <int R, int A>
struct SelDispatch {
  static TNC_HD inline Regs<R> run(const Regs<R>& v, int a, const float* __restrict__ k, bool dup) {
    if (a == A) return dup ? op_dup<R, A>(v) : op_sel<R, A>(v, k);
    if constexpr (A + 1 < R) return SelDispatch<R, A + 1>::run(v, a, k, dup);
    return v;
  }
};

// Apply the ops of one phase to a thread's registers.
//   tb: the thread part of the local tile index in this phase.
//   xb: the output bits of this tile's batch.
template <int R>
TNC_HD inline void run_phase_ops(Regs<R>& v, const DevPhase& P, const DevOp* __restrict__ ops,
                                 const float* __restrict__ mats, const uint8_t* __restrict__ xb,
                                 uint32_t tb) {
  for (int o = P.op_begin; o < P.op_end; ++o) {
    const DevOp op = ops[o];
    int var = 0;
    if (op.xrow0 >= 0) var += 2 * xb[op.xrow0];
    if (op.xrow1 >= 0) var += xb[op.xrow1];
    const float* m = mats + ((size_t)op.mat * 4 + var) * 16;
    if (op.kind == 1) {
      v = SelDispatch<R, 0>::run(v, op.treg, m, true);
    } else if (op.creg >= R) {
      const int ctl = op.cloc >= 0 ? int((tb >> op.cloc) & 1u) : 0;
      v = SelDispatch<R, 0>::run(v, op.treg, m + 8 * ctl, false);
    } else {
      v = RegDispatch<R, 0, 0>::run(v, op.treg, op.creg, m);
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
