// Kernel launchers (host side) and the shared per-thread helpers of the
// pass kernel, usable on host and device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device_tables.hpp"
#include "lds_layout.hpp"

namespace tnc {

constexpr int kBlock = 256;

// A float4 holding the entry pair (i, i + 1) in index order, as stored in
// (or to be stored to) its LDS slot, whose order is swapped when s is set.
// A bitwise select (no branch, no wait on a load beyond this value's own).
TNC_HD inline float4 pair_order(float4 v, bool s) {
  const uint32_t m = 0u - (uint32_t)s;
  const uint32_t x = __float_as_uint(v.x), y = __float_as_uint(v.y), z = __float_as_uint(v.z), w = __float_as_uint(v.w);
  return make_float4(__uint_as_float(x ^ ((x ^ z) & m)), __uint_as_float(y ^ ((y ^ w) & m)),
                     __uint_as_float(z ^ ((z ^ x) & m)), __uint_as_float(w ^ ((w ^ y) & m)));
}

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

// ---------------------------------------------------------------------------
// 16-bit block-scaled storage.

// Scale slot of entry g (index within its batch) under the writer's layout.
TNC_HD inline uint64_t scale_slot(uint64_t g, const ScaleMap& m) {
  const uint64_t lo_mask = (1ull << m.lo_bits) - 1ull;
  const uint64_t local = (g & lo_mask) | (((g >> m.win_lo) & ((1ull << m.win_len) - 1ull)) << m.lo_bits);
  const int gap = m.win_lo - m.lo_bits;
  const uint64_t tile = ((g >> m.lo_bits) & ((1ull << gap) - 1ull)) | ((g >> (m.win_lo + m.win_len)) << gap);
  return (tile << (m.tile_bits - m.blk_bits)) | (local >> m.blk_bits);
}

// Exponent e of the power-of-two block scale 2^e that puts the block's
// largest component amax in [2^14, 2^15): below the FP16 maximum (65504)
// with a full binade of headroom, and far inside the BF16 range.  e is kept
// in [-100, 100] so that 2^e and 2^-e are normal FP32 numbers; a block whose
// largest component is below 2^-86 (rounding residue of exact zeros) is
// stored below the top of the range.
TNC_HD inline int block_exponent(float amax) {
  if (!(amax > 0.f)) return 0;
  int e = 0;
  (void)frexpf(amax, &e);  // amax in [2^(e-1), 2^e)
  e -= 15;
  return e < -100 ? -100 : (e > 100 ? 100 : e);
}

// One component stored in 16 bits (round to nearest even) and read back.
template <int S>
TNC_HD inline uint32_t to16(float x) {
  if constexpr (S == STORE_F16) {
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)x);
  } else {
    uint32_t u = __builtin_bit_cast(uint32_t, x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
  }
}

template <int S>
TNC_HD inline float from16(uint32_t v) {
  if constexpr (S == STORE_F16) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xFFFFu));
  } else {
    return __builtin_bit_cast(float, v << 16);
  }
}

// An entry (re, im) as one 32-bit word of two 16-bit halves.
template <int S>
TNC_HD inline uint32_t pack16(float re, float im, float inv_scale) {
  return to16<S>(re * inv_scale) | (to16<S>(im * inv_scale) << 16);
}

template <int S>
TNC_HD inline float2 unpack16(uint32_t w, float scale) {
  return make_float2(from16<S>(w) * scale, from16<S>(w >> 16) * scale);
}

// The pass tables (phases, ops, matrices) are read through the constant
// address space on the device: wave-uniform reads become scalar loads, which
// are counted apart from vector memory, so reading them never waits for
// vector loads in flight (such as the prefetch of the next tile).
#if defined(__HIP_DEVICE_COMPILE__)
#define TNC_TBL __attribute__((address_space(4)))
#else
#define TNC_TBL
#endif

// Phase p of a pass table, read as four 32-bit words (one scalar load
// when p is wave-uniform; byte fields read one by one would become vector
// loads).
TNC_HD inline DevPhase load_phase(const DevPhase* phases, int p) {
  const uint4 w = ((const TNC_TBL uint4*)phases)[p];
  return __builtin_bit_cast(DevPhase, w);
}

// The LDS address of a pointer into LDS (0 on the host, whose emulation
// addresses its tile from the region pointer).
TNC_HD inline uint32_t lds_address(const void* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
#else
  (void)p;
  return 0u;
#endif
}
#if defined(__HIP_DEVICE_COMPILE__)
// The LDS entry at LDS address `off`: the phase offsets are whole LDS
// addresses (the tile's region base folded in once per block), so no
// per-entry addition of the array's base.  Moved as one 64-bit word, so each
// access stays a single ds_read_b64 / ds_write_b64 (the bank-cycle placement
// is laid out for 8-byte accesses).
__device__ __attribute__((always_inline)) inline float2 lds_get(char*, uint32_t off) {
  return __builtin_bit_cast(float2, *(const __attribute__((address_space(3))) uint64_t*)(uintptr_t)off);
}
__device__ __attribute__((always_inline)) inline void lds_put(char*, uint32_t off, float2 v) {
  *(__attribute__((address_space(3))) uint64_t*)(uintptr_t)off = __builtin_bit_cast(uint64_t, v);
}
#else
inline float2 lds_get(char* base, uint32_t off) { return *reinterpret_cast<const float2*>(base + off); }
inline void lds_put(char* base, uint32_t off, float2 v) { *reinterpret_cast<float2*>(base + off) = v; }
#endif

// Register-resident complex64 entries of a thread: separate real and
// imaginary float arrays (keeps every element promotable to a VGPR).
template <int R>
struct Regs {
  float x[1 << R];
  float y[1 << R];
};

// (b0, b1) <- K (b0, b1) with K = [k0 k1; k2 k3] given as 8 floats (re, im).
template <class P>
TNC_HD inline void cmat2(P k, float& x0, float& y0, float& x1, float& y1) {
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
TNC_HD inline Regs<R> op_reg(Regs<R> v, const TNC_TBL float* __restrict__ m) {
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & (1 << A)) continue;
    const int j = i | (1 << A);
    cmat2(m + 8 * ((i >> C) & 1), v.x[i], v.y[i], v.x[j], v.y[j]);
  }
  return v;
}

// A dense 4x4 on register bits (A, B), A < B: the entries with u = bit A +
// 2 bit B become M (e_0 .. e_3); m: M row-major, 32 floats (re, im).
template <int R, int A, int B, class P>
TNC_HD inline Regs<R> op_dense(Regs<R> v, P m) {
  float k[32];
#pragma unroll
  for (int e = 0; e < 32; ++e) k[e] = m[e];
#pragma unroll
  for (int i = 0; i < (1 << R); ++i) {
    if (i & ((1 << A) | (1 << B))) continue;
    float ix[4], iy[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int j = i | ((u & 1) << A) | ((u >> 1) << B);
      ix[u] = v.x[j];
      iy[u] = v.y[j];
    }
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      float ox = 0.f, oy = 0.f;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ox = ox + k[8 * o + 2 * u] * ix[u] - k[8 * o + 2 * u + 1] * iy[u];
        oy = oy + k[8 * o + 2 * u] * iy[u] + k[8 * o + 2 * u + 1] * ix[u];
      }
      const int j = i | ((o & 1) << A) | ((o >> 1) << B);
      v.x[j] = ox;
      v.y[j] = oy;
    }
  }
  return v;
}

template <int R, int A, class P>
TNC_HD inline Regs<R> op_sel(Regs<R> v, P k) {
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

constexpr int kMaxThreadBitsDev = 9;

#if defined(__HIP_DEVICE_COMPILE__)
typedef float tnc_floatx4 __attribute__((ext_vector_type(4)));
#endif

template <int R>
struct PhaseCtx {
  const TNC_TBL float* __restrict__ rm;  // the tile's batch: resolved matrices, 16 floats per op
  uint32_t tb;                           // the thread's index within its tile
  bool uniform;
};

// Output bit at byte `pos` of the bit array.  On the device the byte is cut
// from the aligned 32-bit word that holds it, read through the constant
// address space: one scalar load when `pos` is wave-uniform.  The word never
// crosses a 4-byte boundary, so it stays inside the page of the byte.
TNC_HD inline int out_bit(const uint8_t* bits, size_t pos) {
#if defined(__HIP_DEVICE_COMPILE__)
  const uintptr_t addr = reinterpret_cast<uintptr_t>(bits) + pos;
  const uint32_t w = *(const TNC_TBL uint32_t*)(addr & ~(uintptr_t)3);
  return int((w >> (8 * (addr & 3))) & 1u);
#else
  return bits[pos] & 1;
#endif
}

// A value read at a wave-uniform address (valid only where the address is
// the same for every lane of the wave).  Selecting between two such values
// per lane must not be turned into a load from a per-lane address (a vector
// load); pinning each value to the wave keeps both loads scalar.
TNC_HD inline float uniform_value(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
#else
  return x;
#endif
}

// Ops 1..N-1 of a canonical phase: op b on register bit b controlled by b-1.
template <int R, int B, int N>
TNC_HD inline Regs<R> stair_rest(Regs<R> v, const PhaseCtx<R>& c, int op_begin) {
  if constexpr (B < N) {
    v = op_reg<R, B, B - 1>(v, c.rm + (size_t)(op_begin + B) * 16);
    return stair_rest<R, B + 1, N>(v, c, op_begin);
  }
  return v;
}

// A whole canonical phase of N ops on a thread's registers.  K0 is the
// form of op 0: 0 a duplication, 1 an update with no control, 2 an update
// controlled by a thread bit (cloc0).  Each form is its own code path, so no
// register values merge across forms.
template <int R, int N, int K0>
TNC_HD inline Regs<R> stair(Regs<R> v, const DevPhase& P, const PhaseCtx<R>& c) {
  if constexpr (K0 == 0) {
    v = op_dup<R, 0>(v);
  } else {
    const TNC_TBL float* m = c.rm + (size_t)P.op_begin * 16;
    if constexpr (K0 == 1) {
      v = op_sel<R, 0>(v, m);
    } else {
      const bool hi = (c.tb >> P.cloc0) & 1u;  // op 0's control: thread bit cloc0
      if (c.uniform) {
        // thread-controlled: pick the values per thread from the
        // wave-uniform pair of matrices (a per-thread address would need
        // vector loads)
        // (both matrices pinned first, unconditionally: a pinning under
        // the per-lane condition would become divergent branches)
        float lo[8], up[8], k[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          lo[e] = uniform_value(m[e]);
          up[e] = uniform_value(m[8 + e]);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) k[e] = hi ? up[e] : lo[e];
        v = op_sel<R, 0>(v, static_cast<const float*>(k));
      } else {
        v = op_sel<R, 0>(v, m + 8 * int(hi));
      }
    }
  }
  return stair_rest<R, 1, N>(v, c, P.op_begin);
}

// LDS byte offset of a thread's base entry in a phase: thread bit t adds the
// tile bit the planner placed it on, whose offset is po[kPhaseEntries + t]
// (wave-uniform table reads: one wide scalar load).  No test of t against
// the phase's thread-bit count: the table holds zero past it and the thread
// index has no bit set there, so the loop is straight-line code.
TNC_HD inline uint32_t phase_thread_base(uint32_t rbase, const TNC_TBL uint32_t* po, uint32_t tt) {
  uint32_t vb = rbase;
#pragma unroll
  for (int t = 0; t < kMaxThreadBitsDev; ++t) vb ^= (0u - ((tt >> t) & 1u)) & po[kPhaseEntries + t];
  return vb;
}

// One register phase: LDS -> registers (phase layout), the phase's ops,
// registers -> LDS.  Each thread writes back exactly the entries it read.
// The tile sits at byte offset `rbase` of `base`, with rbase's bits above
// the tile's own (rbase = 0 or a multiple of 2^(T+3)).  po[i] (from the pass
// tables) is swz(r_i) << 3 for the tile index r_i of register entry i; the
// swizzle is linear, so an entry's offset is the thread's base ^ po[i].
template <int R, int N, int K0>
TNC_HD inline void phase_exec(char* base, uint32_t rbase, const DevPhase& P, const TNC_TBL uint32_t* po,
                              const PhaseCtx<R>& c0, uint32_t tt, int TB) {
  constexpr int E = 1 << R;
  PhaseCtx<R> c = c0;
  c.tb = tt;
  const uint32_t vbase = phase_thread_base(rbase, po, tt);
  uint32_t off[E];
#pragma unroll
  for (int i = 0; i < E; ++i) off[i] = vbase ^ po[i];
  Regs<R> v;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const float2 t = lds_get(base, off[i]);
    v.x[i] = t.x;
    v.y[i] = t.y;
  }
  v = stair<R, N, K0>(v, P, c);
#pragma unroll
  for (int i = 0; i < E; ++i) lds_put(base, off[i], make_float2(v.x[i], v.y[i]));
}

// Between the updates of a dense phase: keeps each update's 32 matrix
// values from being loaded ahead of the previous update (four updates' worth
// would not fit the scalar registers and would move to vector registers).
TNC_HD inline void dense_fence() {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_amdgcn_sched_barrier(0);
#endif
}

// A dense phase: n_ops / 2 dense 4x4 updates in order, update g on the
// register-bit pair of its code (4 bits of reg[6..7]) with the 32 floats of
// ops op_begin + 2g, op_begin + 2g + 1 (rows 0-1, rows 2-3).  Same register
// entries and LDS placement as phase_exec.
template <int R>
TNC_HD inline void phase_dense(char* base, uint32_t rbase, const DevPhase& P, const TNC_TBL uint32_t* po,
                               const PhaseCtx<R>& c, uint32_t tt, int TB) {
  constexpr int E = 1 << R;
  const uint32_t vbase = phase_thread_base(rbase, po, tt);
  uint32_t off[E];
#pragma unroll
  for (int i = 0; i < E; ++i) off[i] = vbase ^ po[i];
  Regs<R> v;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const float2 t = lds_get(base, off[i]);
    v.x[i] = t.x;
    v.y[i] = t.y;
  }
  const int G = P.n_ops / 2;
  const uint32_t codes = (uint32_t)(uint8_t)P.reg[6] | ((uint32_t)(uint8_t)P.reg[7] << 8);
  const TNC_TBL float* m = c.rm + (size_t)P.op_begin * 16;
  // one straight-line form per pattern (dense_form_exists)
  switch ((uint32_t)G << 16 | codes) {
    case 1u << 16 | 0x0u:
      v = op_dense<R, 0, 1>(v, m);
      break;
    case 2u << 16 | 0x40u:
      if constexpr (R >= 3) {
        v = op_dense<R, 0, 1>(v, m);
        v = op_dense<R, 1, 2>(v, m + 32);
      }
      break;
    case 2u << 16 | 0x70u:
      if constexpr (R >= 4) {
        v = op_dense<R, 0, 1>(v, m);
        v = op_dense<R, 2, 3>(v, m + 32);
      }
      break;
    case 3u << 16 | 0x940u:
      if constexpr (R >= 5) {
        v = op_dense<R, 0, 1>(v, m);
        dense_fence();
        v = op_dense<R, 1, 2>(v, m + 32);
        dense_fence();
        v = op_dense<R, 3, 4>(v, m + 64);
      }
      break;
    case 4u << 16 | 0x3940u:
      if constexpr (R >= 5) {
        v = op_dense<R, 0, 1>(v, m);
        dense_fence();
        v = op_dense<R, 1, 2>(v, m + 32);
        dense_fence();
        v = op_dense<R, 3, 4>(v, m + 64);
        dense_fence();
        v = op_dense<R, 0, 4>(v, m + 96);
      }
      break;
    default:
      break;  // excluded on the host (dense_form_exists)
  }
#pragma unroll
  for (int i = 0; i < E; ++i) lds_put(base, off[i], make_float2(v.x[i], v.y[i]));
}

template <int R, int N>
TNC_HD inline void phase_forms(char* base, uint32_t rbase, const DevPhase& P, const TNC_TBL uint32_t* po,
                               const PhaseCtx<R>& c, uint32_t tt, int TB) {
  if (P.first_dup) phase_exec<R, N, 0>(base, rbase, P, po, c, tt, TB);
  else if (P.cloc0 < 0) phase_exec<R, N, 1>(base, rbase, P, po, c, tt, TB);
  else phase_exec<R, N, 2>(base, rbase, P, po, c, tt, TB);
}

#if defined(__HIP_DEVICE_COMPILE__)
// A fused phase (three staircase updates as one complex 8x8 U_c per value c
// of op 0's control) on v_mfma_f32_16x16x4f32.  Lane l = 16 g + j holds,
// for each of its 2^(R-1) groups, the entries b0 = 0, 1 (register bit 0)
// of vector j with (b1, b2) = g: four floats, MFMA steps s = 0..3 in the
// order (re, im) of b0 = 0, then of b0 = 1.  Step s takes A[j'][4 s + g]
// from lane 16 g + j' and B[4 s + g][j] from lane 16 g + j; the result
// D[4 g + r][j] lands in lane 16 g + j as component r, the same layout.
// Groups with register bit R-1 set use U_1 (op 0's control sits there; an
// uncontrolled op 0 has U_1 = U_0).  Thread bit t of the tile adds tile bit
// tpos[t], whose LDS offset is po[kPhaseEntries + t].  Updates 3..N-1 then
// go on on the vector ALUs: update 3 on register bit 1 under lane bit 5
// (b2), update b > 3 on register bit b - 2 under register bit b - 3.
// The complex 8x8 of a fused phase on the matrix cores (layout above): the
// operands for groups with register bit R-1 clear are F[lane], for those
// with it set F[64 + lane].
template <int R>
__device__ __attribute__((always_inline)) inline Regs<R> tri_product(Regs<R> v, const float4* __restrict__ F,
                                                                     int lane) {
  constexpr int G = (1 << R) / 2;
  const float4 a0 = F[lane];
  const float4 a1 = F[64 + lane];
#pragma unroll
  for (int j = 0; j < G; ++j) {
    const float4 a = j >= G / 2 ? a1 : a0;
    tnc_floatx4 d = {0.f, 0.f, 0.f, 0.f};
    d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, v.x[2 * j], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, v.y[2 * j], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, v.x[2 * j + 1], d, 0, 0, 0);
    d = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, v.y[2 * j + 1], d, 0, 0, 0);
    v.x[2 * j] = d[0];
    v.y[2 * j] = d[1];
    v.x[2 * j + 1] = d[2];
    v.y[2 * j + 1] = d[3];
  }
  return v;
}

template <int R, int N>
__device__ __attribute__((always_inline)) inline void phase_tri(char* base, uint32_t rbase, const DevPhase& P,
                                                                const TNC_TBL uint32_t* po, const float4* __restrict__ F,
                                                                const PhaseCtx<R>& c, uint32_t tt, int TB) {
  constexpr int E = 1 << R;
  const int lane = (int)(tt & 63u);
  const uint32_t vb = phase_thread_base(rbase, po, tt);
  uint32_t off[E];
#pragma unroll
  for (int i = 0; i < E; ++i) off[i] = vb ^ po[i];
  Regs<R> v;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const float2 t = lds_get(base, off[i]);
    v.x[i] = t.x;
    v.y[i] = t.y;
  }
  // every LDS read in flight before the first product (the scheduler would
  // otherwise wait on each read in turn)
  __builtin_amdgcn_sched_barrier(0);
  v = tri_product<R>(v, F, lane);
  if constexpr (N >= 4) {
    const TNC_TBL float* m = c.rm + (size_t)(P.op_begin + 3) * 16;
    const bool hi = (lane >> 5) & 1;
    float lo[8], up[8], k[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      lo[e] = uniform_value(m[e]);
      up[e] = uniform_value(m[8 + e]);
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) k[e] = hi ? up[e] : lo[e];
    v = op_sel<R, 1>(v, static_cast<const float*>(k));
  }
  if constexpr (N >= 5) v = op_reg<R, 2, 1>(v, c.rm + (size_t)(P.op_begin + 4) * 16);
  if constexpr (N >= 6) v = op_reg<R, 3, 2>(v, c.rm + (size_t)(P.op_begin + 5) * 16);
  if constexpr (N >= 7) v = op_reg<R, 4, 3>(v, c.rm + (size_t)(P.op_begin + 6) * 16);
#pragma unroll
  for (int i = 0; i < E; ++i) lds_put(base, off[i], make_float2(v.x[i], v.y[i]));
}

// A bond-four unit phase (P.pad = 3): one wavefront step, the 4x4 on (b0,
// b1) then the 4x4 on (b1, b2), as one complex 8x8 on the matrix cores (the
// layout of phase_tri: b0 = register bit 0, b1 and b2 = lane bits 4 and 5);
// with n_ops = 8, the next step's two updates follow on the vector ALUs, on
// register bits (1, 2) and then (0, 2) (ops op_begin + 4 .. + 7; the first
// of them does not read the product and can run beside it).
template <int R>
__device__ __attribute__((always_inline)) inline void phase_unit(char* base, uint32_t rbase, const DevPhase& P,
                                                                 const TNC_TBL uint32_t* po, const float4* __restrict__ F,
                                                                 const PhaseCtx<R>& c, uint32_t tt, int TB) {
  constexpr int E = 1 << R;
  const int lane = (int)(tt & 63u);
  const uint32_t vb = phase_thread_base(rbase, po, tt);
  uint32_t off[E];
#pragma unroll
  for (int i = 0; i < E; ++i) off[i] = vb ^ po[i];
  Regs<R> v;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const float2 t = lds_get(base, off[i]);
    v.x[i] = t.x;
    v.y[i] = t.y;
  }
  __builtin_amdgcn_sched_barrier(0);
  v = tri_product<R>(v, F, lane);
  if constexpr (R >= 3) {
    if (P.n_ops == 8) {
      const TNC_TBL float* m = c.rm + (size_t)(P.op_begin + 4) * 16;
      v = op_dense<R, 1, 2>(v, m);
      v = op_dense<R, 0, 2>(v, m + 32);
    }
  }
#pragma unroll
  for (int i = 0; i < E; ++i) lds_put(base, off[i], make_float2(v.x[i], v.y[i]));
}
#endif

// Register phases with an instantiated form: a canonical phase of 1..R
// updates (form 0), a fused phase of 3..R+2 updates (form 1), a dense phase
// of one to four 4x4s (two ops each; form 2), or a bond-four unit phase of
// two or four 4x4s (form 3);
// the planner checks every phase against this before the tables reach the
// device.
TNC_HD constexpr bool phase_form_exists(int R, int n_ops, int form) {
  return form == 1   ? (R >= 3 && n_ops >= 3 && n_ops <= R + 2 && n_ops <= 7)
         : form == 2 ? (R >= 2 && R <= 5 && n_ops >= 2 && n_ops <= 8 && n_ops % 2 == 0)
         : form == 3 ? (R >= 3 && R <= 5 && (n_ops == 4 || n_ops == 8))
                     : (n_ops >= 1 && n_ops <= R && R <= 5);
}

// TRI: the kernel runs fused phases (P.pad = 1); the host plans them only for
// kernels whose waves each lie inside one tile.  KIND 0: the bond-two forms;
// KIND 1: the bond-four forms, dense phases (P.pad = 2) and single
// uncontrolled updates (the host checks that a bond-four plan has no other).
template <int R, bool TRI = false, int KIND = 0>
TNC_HD inline void phase_dispatch(char* base, uint32_t rbase, const DevPhase& P, const TNC_TBL uint32_t* po,
                                  const PhaseCtx<R>& c, uint32_t tt, int TB, const float4* fm = nullptr) {
  if constexpr (KIND == 1) {
    if (P.pad == 2) {
      if constexpr (R >= 2) phase_dense<R>(base, rbase, P, po, c, tt, TB);
#if defined(__HIP_DEVICE_COMPILE__)
    } else if (P.pad == 3) {
      if constexpr (TRI && R >= 3) phase_unit<R>(base, rbase, P, po, fm, c, tt, TB);
#endif
    } else {
      phase_exec<R, 1, 1>(base, rbase, P, po, c, tt, TB);
    }
    return;
  }
#if defined(__HIP_DEVICE_COMPILE__)
  if constexpr (TRI && R >= 3) {
    if (P.pad == 1) {
      // update b > 2 targets register bit b - 2: up to R + 2 updates
      switch (P.n_ops) {
        case 3: phase_tri<R, 3>(base, rbase, P, po, fm, c, tt, TB); break;
        case 4: phase_tri<R, 4>(base, rbase, P, po, fm, c, tt, TB); break;
        case 5: phase_tri<R, 5>(base, rbase, P, po, fm, c, tt, TB); break;
        case 6: if constexpr (R >= 4) phase_tri<R, 6>(base, rbase, P, po, fm, c, tt, TB); break;
        case 7: if constexpr (R >= 5) phase_tri<R, 7>(base, rbase, P, po, fm, c, tt, TB); break;
        default: break;  // excluded on the host (phase_form_exists)
      }
      return;
    }
  }
#endif
  switch (P.n_ops) {
    case 1: phase_forms<R, 1>(base, rbase, P, po, c, tt, TB); break;
    case 2: if constexpr (R >= 2) phase_forms<R, 2>(base, rbase, P, po, c, tt, TB); break;
    case 3: if constexpr (R >= 3) phase_forms<R, 3>(base, rbase, P, po, c, tt, TB); break;
    case 4: if constexpr (R >= 4) phase_forms<R, 4>(base, rbase, P, po, c, tt, TB); break;
    case 5: if constexpr (R >= 5) phase_forms<R, 5>(base, rbase, P, po, c, tt, TB); break;
    default: break;  // excluded on the host (phase_form_exists)
  }
}

// Byte offsets of a phase's register entries in the LDS tile: entry i holds
// the tile index whose register bits reg[b] are the bits of i, placed by
// swz (the po[] table of phase_exec).
TNC_HD inline uint32_t phase_entry_offset(const DevPhase& P, int R, int i) {
  uint32_t r = 0;
  for (int b = 0; b < R; ++b)
    if (i & (1 << b)) r |= 1u << P.reg[b];
  return swz(r) << 3;
}

// ---------------------------------------------------------------------------
// Launch records.  A kernel launch of the amplitude path is recorded first:
// the kernel, its grid and block, its LDS size and a copy of its single
// by-value argument.  A record is then issued on a stream (issue), added to a
// HIP graph as a kernel node (graph_add; no stream capture involved), or
// merged with records of the same kernel for other requests into one grouped
// launch (issue_grouped): the grouped entry point gfn runs segment blockIdx.z
// of a device table of segments, each the argument and grid of one record.
constexpr int kMaxArgBytes = 256;
constexpr int kSegHeader = 16;

template <class A>
struct Seg {
  uint32_t gx, gy;  // the record's own grid; blocks of a grouped launch outside it return
  uint32_t pad[2];
  A a;
};

struct Launch {
  const void* fn = nullptr;   // the kernel
  const void* gfn = nullptr;  // its grouped entry point (null: never grouped)
  dim3 grid{1, 1, 1}, block{1, 1, 1};
  uint32_t shmem = 0;
  uint32_t arg_bytes = 0;
  uint32_t seg_stride = 0;    // bytes of one segment of the grouped entry's table
  int cls = 0;                // profiling class: 0 build-up and resolution, 1 pass, 2 late phase
  double bytes = 0.0;         // algorithmic bytes (passes)
  alignas(16) unsigned char arg[kMaxArgBytes] = {};
};

// Record builders (kernels.hip); hipErrorInvalidValue for a shape the
// kernels do not take.
hipError_t record_init(const InitArgs& a, Launch* L);
hipError_t record_resolve(const ResolveArgs& a, Launch* L);
hipError_t record_pass(const PassArgs& a, int R, Launch* L);
hipError_t record_late(const LateArgs& a, bool in_c64, Launch* L);
hipError_t record_late_ops(const LateOpsArgs& a, Launch* L);

hipError_t issue(const Launch& L, hipStream_t s);
hipError_t graph_add(const Launch& L, hipGraph_t g, hipGraphNode_t* node, const hipGraphNode_t* dep, size_t n_dep);
// Records of the same kernel with a grouped entry point and the same block.
bool groupable(const Launch& a, const Launch& b);
// Segment table of n groupable records, written to host memory at dst (n *
// seg_stride bytes); returns the bytes written.
size_t write_segments(const Launch* const* members, int n, unsigned char* dst);
// One launch running every member; d_segs: the segment table in device
// memory (kept valid until the launch has run).
hipError_t issue_grouped(const Launch* const* members, int n, const void* d_segs, hipStream_t s);

// The complex128 reference sweep (tests): row-0 build-up stored in FP64
// (a.B holds double2 entries) and one unfused update per launch.
hipError_t launch_init64(const InitArgs& a, hipStream_t s);
hipError_t launch_op64(const Op64Args& a, hipStream_t s);

// Launchers of the kernels outside the amplitude path (kernels.hip).
hipError_t launch_fill_zero(double2* out, long long count, hipStream_t s);
// out[i] += sum over r < rows of in[r * stride + i], added in row order.
hipError_t launch_accumulate_rows(double2* out, const double2* in, long long stride, int rows, long long count,
                                  hipStream_t s);
// Batched sampling handles up to 2^10 suffixes per batch: 4 per thread.
constexpr int kMaxSampleEntries = 4;
hipError_t launch_sample_batched(const double2* amps, int n_batches, int k, const double* u, int32_t* b, double* q,
                                 hipStream_t s);
hipError_t launch_frugal_accept(const double2* amps, long long count, int n, double M, const double* u,
                                uint8_t* accept, double* z, hipStream_t s);
hipError_t launch_logxeb(const double2* amps, int n_batches, int k, const int32_t* sel, int n_qubits,
                         double* result, hipStream_t s);

// Host emulation of the pass kernel (exact thread / LDS mapping), for tests.
void emulate_pass_host(const PassArgs& a, int R);

}  // namespace tnc
