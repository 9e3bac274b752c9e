// HIP kernels for gfx950 (CDNA4) of the temporal-boundary contraction.
//
//  k_init     row-0 build-up of the boundary tensor (one write pass)
//  k_resolve  per-batch choice of every update's matrix variant
//  k_pass     one fused window of staircase updates over every tile of the
//             boundary tensor (the hot loop); in place, HBM-streaming
//  k_late     the folded late-phase contraction: the Alg. 2 join and the late
//             layers, FP64 accumulation (k_late_mf: the same on FP64 matrix
//             cores), and k_late_ops, the rest of the late program
//  k_logxeb   FP64 log-XEB reduction; samplers
//
// The kernels of the amplitude path are recorded as launches (Launch, see
// kernels.hpp) before they run.  Each such kernel has a body taking its block
// index explicitly, a plain entry point, and (complex64 path) a grouped entry
// point that runs segment blockIdx.z of a table of (argument, grid) segments:
// launches of one kernel for different requests merged into one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstring>
#include <vector>

#include "kernels.hpp"

namespace tnc {

// The segment of a grouped launch that this block belongs to, or null when
// the block lies outside its segment's own grid.
template <class A>
__device__ __attribute__((always_inline)) inline const Seg<A>* group_seg(const Seg<A>* segs) {
  const Seg<A>* s = segs + blockIdx.z;
  if (blockIdx.x >= s->gx || blockIdx.y >= s->gy) return nullptr;
  return s;
}

// ---------------------------------------------------------------------------
// Row-0 build-up.  The first row only creates slots: its boundary tensor is
// the product  v[a_0] * prod_{j>=1} seg_j[a_j][a_{j-1}] * f_x[a_{m-1}]
// (copy tensors of the down-bonds joined by the one-qubit segments).
// For h >= 11 each wave writes 2048 consecutive entries, lane l taking the
// entries 64 e + l (e < 32): every store is one contiguous 512-byte run, and
// the factors of bits 0..5 (the lane) and >= 11 (the wave) are multiplied
// once per thread, those of bits 6..10 per entry.  Entries above 2^m are
// zero.
__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __attribute__((always_inline)) inline void init_body(const InitArgs& a, uint32_t bx) {
  __shared__ double2 seg[4 * 64];
  const int nseg = a.m0 - 1;
  for (int i = threadIdx.x; i < 4 * nseg; i += blockDim.x) seg[i] = a.seg[i];
  __syncthreads();
  const int m = a.m0;
  const long long gid = (long long)bx * blockDim.x + threadIdx.x;
  auto sg = [&](int j, unsigned long long i) {
    return seg[4 * (j - 1) + 2 * (int)((i >> j) & 1ull) + (int)((i >> (j - 1)) & 1ull)];
  };
  if (a.h < 11) {
    const long long total = (long long)a.n_batches << a.h;
    if (gid >= total) return;
    const long long batch = gid >> a.h;
    const unsigned long long i = (unsigned long long)gid & ((1ull << a.h) - 1ull);
    float2* out = a.B + gid;
    if (i >> m) {
      *out = make_float2(0.f, 0.f);
      return;
    }
    const int x0 = a.bits[batch * a.n];
    double2 val = a.v[i & 1ull];
    for (int j = 1; j < m; ++j) val = zmul(val, sg(j, i));
    val = zmul(val, a.f[x0][(i >> (m - 1)) & 1ull]);
    *out = make_float2((float)val.x, (float)val.y);
    return;
  }
  const long long wave = gid >> 6;
  const unsigned long long lane = (unsigned long long)(gid & 63);
  if (wave >= (((long long)a.n_batches << a.h) >> 11)) return;
  const long long first = wave << 11;
  const long long batch = first >> a.h;
  const unsigned long long i0 = ((unsigned long long)first & ((1ull << a.h) - 1ull)) | lane;
  float2* out = a.B + first + (long long)lane;
  const int x0 = a.bits[batch * a.n];
  // factors fixed for the thread: bits 0..5 (lane) and >= 11 (wave)
  double2 fixed = a.v[lane & 1ull];
  for (int j = 1; j < m && j <= 5; ++j) fixed = zmul(fixed, sg(j, i0));
  for (int j = 12; j < m; ++j) fixed = zmul(fixed, sg(j, i0));
  const bool f_var = m - 1 >= 6 && m - 1 <= 10;
  if (!f_var) fixed = zmul(fixed, a.f[x0][(i0 >> (m - 1)) & 1ull]);
  const int jhi = m - 1 < 11 ? m - 1 : 11;
  for (int e = 0; e < 32; ++e) {
    const unsigned long long i = i0 + ((unsigned long long)e << 6);
    if (i >> m) {
      out[e << 6] = make_float2(0.f, 0.f);
      continue;
    }
    double2 val = fixed;
    for (int j = 6; j <= jhi; ++j) val = zmul(val, sg(j, i));
    if (f_var) val = zmul(val, a.f[x0][(i >> (m - 1)) & 1ull]);
    out[e << 6] = make_float2((float)val.x, (float)val.y);
  }
}

__global__ __launch_bounds__(kBlock) void k_init(InitArgs a) { init_body(a, blockIdx.x); }

__global__ __launch_bounds__(kBlock) void k_init_g(const Seg<InitArgs>* __restrict__ segs) {
  const Seg<InitArgs>* s = group_seg(segs);
  if (!s) return;
  const InitArgs a = s->a;
  init_body(a, blockIdx.x);
}

// Row-0 build-up into 16-bit block-scaled storage: one workgroup per block
// of 2^blk_bits consecutive entries (the scale block of this writer); the
// FP64 product is rounded to FP32 as in the complex64 path, then the block
// maximum fixes the power-of-two scale.
template <int S>
__global__ __launch_bounds__(kBlock) void k_init16(InitArgs a) {
  constexpr int kMaxPer = 4096 / kBlock;
  __shared__ double2 seg[4 * 64];
  __shared__ uint32_t smax;
  const int nseg = a.m0 - 1;
  for (int i = threadIdx.x; i < 4 * nseg; i += blockDim.x) seg[i] = a.seg[i];
  if (threadIdx.x == 0) smax = 0u;
  __syncthreads();
  const int bb = a.blk_bits;
  const int per_batch_blocks_log = a.h - bb;
  const long long batch = (long long)blockIdx.x >> per_batch_blocks_log;
  const unsigned long long sblk = (unsigned long long)blockIdx.x & ((1ull << per_batch_blocks_log) - 1ull);
  const unsigned long long i0 = sblk << bb;
  const int nper = 1 << bb;
  const int x0 = a.bits[batch * a.n];
  const int m = a.m0;
  float2 val[kMaxPer];
  float amax = 0.f;
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q) {
    const int off = q * kBlock + (int)threadIdx.x;
    val[q] = make_float2(0.f, 0.f);
    if (off >= nper) continue;
    const unsigned long long i = i0 + (unsigned long long)off;
    if (i >> m) continue;
    double2 v = a.v[i & 1ull];
    for (int j = 1; j < m; ++j) {
      const int aj = (int)((i >> j) & 1ull), ajm = (int)((i >> (j - 1)) & 1ull);
      v = zmul(v, seg[4 * (j - 1) + 2 * aj + ajm]);
    }
    v = zmul(v, a.f[x0][(i >> (m - 1)) & 1ull]);
    val[q] = make_float2((float)v.x, (float)v.y);
    amax = fmaxf(amax, fmaxf(fabsf(val[q].x), fabsf(val[q].y)));
  }
  if (amax > 0.f) atomicMax(&smax, __float_as_uint(amax));
  __syncthreads();
  const int e = block_exponent(__uint_as_float(smax));
  const float inv = ldexpf(1.f, -e);
  uint32_t* out = reinterpret_cast<uint32_t*>(a.B) + (batch << a.h) + i0;
#pragma unroll
  for (int q = 0; q < kMaxPer; ++q) {
    const int off = q * kBlock + (int)threadIdx.x;
    if (off < nper) out[off] = pack16<S>(val[q].x, val[q].y, inv);
  }
  if (threadIdx.x == 0) a.scale_out[batch * a.scale_stride + (long long)sblk] = ldexpf(1.f, e);
}

// ---------------------------------------------------------------------------
// Variant resolution: every op's matrix pair for each batch of the group,
// picked once from the batch's output bits, so the pass kernels read their
// matrices at addresses that depend on the op only.
__device__ __attribute__((always_inline)) inline void resolve_body(const ResolveArgs& a, uint32_t bx) {
  const long long gid = (long long)bx * blockDim.x + threadIdx.x;
  const long long total = (long long)a.n_batches * a.n_ops;
  if (gid >= total) return;
  const int b = (int)(gid / a.n_ops);
  const int o = (int)(gid - (long long)b * a.n_ops);
  const DevOp op = a.ops[o];
  const uint8_t* x = a.bits + (size_t)b * a.n;
  const int var = (op.xrow0 >= 0 ? 2 * (x[op.xrow0] & 1) : 0) + (op.xrow1 >= 0 ? (x[op.xrow1] & 1) : 0);
  const float4* src = reinterpret_cast<const float4*>(a.mats + ((size_t)op.mat * 4 + var) * 16);
  float4* dst = reinterpret_cast<float4*>(a.rmats + (size_t)b * a.rstride + (size_t)o * 16);
#pragma unroll
  for (int q = 0; q < 4; ++q) dst[q] = src[q];
}

__global__ __launch_bounds__(kBlock) void k_resolve(ResolveArgs a) { resolve_body(a, blockIdx.x); }

__global__ __launch_bounds__(kBlock) void k_resolve_g(const Seg<ResolveArgs>* __restrict__ segs) {
  const Seg<ResolveArgs>* s = group_seg(segs);
  if (!s) return;
  const ResolveArgs a = s->a;
  resolve_body(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// The pass kernel.  A tile is 2^T entries of one batch's boundary tensor: the
// global slots [0, lo_bits) and [win_lo, win_lo + win_len).  A block holds
// one tile (T - R = 8 thread bits with 256 threads, 9 with 512) or several
// small ones.  Data path:
//   HBM -> LDS with 16-byte accesses along the contiguous low slots,
//   per phase: LDS -> registers (2^R entries per thread, the phase's target
//   slots as register bits), the phase's updates in registers, registers ->
//   LDS,
//   LDS -> HBM, in place.
// WU: every wave lies inside one tile (one tile per block, or T - R >= 6),
// so the batch and everything read through it are wave-uniform; such
// kernels also run the fused matrix-core phases.
// NT: threads per block (256; 512 for one 2^(R+9)-entry tile per block).
// Resident waves per SIMD the register allocation must allow: LDS admits
// five 2^12-entry (32 KiB) single-tile blocks per CU, so 16-entry phases in
// 256-thread blocks ask for five; fused phases keep two.
template <int R, bool WU, int NT>
constexpr int pass_waves_per_eu() {
  return WU ? 2 : (R == 4 && NT == 256 ? 5 : 1);
}

// Blocks are dispatched round-robin over the 8 XCDs; each XCD takes a
// contiguous range of tiles instead, so the blocks in flight on one XCD read
// and write neighbouring runs (measured: 3.7 % more bandwidth on the loads
// and stores alone, about 1 % per pass).
__device__ __attribute__((always_inline)) inline unsigned xcd_block(uint32_t bx, uint32_t gx) {
  return (gx & 7u) == 0u ? (bx & 7u) * (gx >> 3) + (bx >> 3) : bx;
}

// LDS slots of the iteration parts it << shift (it < 32) of the entries a
// thread stages: swz is linear, so the slot of it << shift is the XOR of the
// slots of its set bits, taken from five values computed once per thread.
struct IterSlots {
  uint32_t b[5];
  __device__ __attribute__((always_inline)) explicit IterSlots(int shift) {
#pragma unroll
    for (int q = 0; q < 5; ++q) b[q] = swz(1u << (shift + q));
  }
  // `it` is a compile-time constant in the unrolled staging loops
  __device__ __attribute__((always_inline)) uint32_t of(int it) const {
    uint32_t s = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q)
      if ((it >> q) & 1) s ^= b[q];
    return s;
  }
};

template <int R, bool MULTI, bool WU, int NT, int KIND>
__device__ __attribute__((always_inline)) inline void pass_body(const PassArgs& a, float2* lds, uint32_t bx,
                                                                uint32_t gx) {
  constexpr int E = 1 << R;
  const int T = a.T;
  const int TB = T - R;
  const int tid = threadIdx.x;
  const int tile_in_block = MULTI ? (tid >> TB) : 0;
  const uint32_t tt = MULTI ? (uint32_t)(tid & ((1 << TB) - 1)) : (uint32_t)tid;
  const int tiles_per_block = MULTI ? (NT >> TB) : 1;
  const long long tile = (long long)xcd_block(bx, gx) * tiles_per_block + tile_in_block;
  const bool active = tile < a.n_tiles;
  const int tbits = a.h - T;
  long long batch = active ? (tile >> tbits) : 0;
  if constexpr (WU) batch = __builtin_amdgcn_readfirstlane((int)batch);
  const unsigned long long blk = active ? ((unsigned long long)tile & ((1ull << tbits) - 1ull)) : 0ull;
  float2* __restrict__ Bt = a.B + (batch << a.h) + block_offset(blk, a.lo_bits, a.win_lo, a.win_len);
  char* region = reinterpret_cast<char*>(lds) + ((size_t)tile_in_block << (T + 3));
  const int tpt = 1 << TB;

  // LDS slot of entry i = (it * tpt + tt) * 2: the thread part and the
  // (wave-uniform) iteration part occupy disjoint bits, so their slots XOR;
  // the iteration part's slot is the XOR of the slots of its set bits
  const uint32_t st = swz(tt * 2u);
  const IterSlots isl(TB + 1);
  if (active) {
    // every load in flight before the first LDS write
    float4 ld[E / 2];
#pragma unroll
    for (int it = 0; it < E / 2; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * 2u;
      ld[it] = *reinterpret_cast<const float4*>(Bt + tile_offset(i, a.lo_bits, a.win_lo));
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int it = 0; it < E / 2; ++it) {
      const uint32_t si = isl.of(it) ^ st;
      *reinterpret_cast<float4*>(region + pair_slot(si)) = pair_order(ld[it], pair_swapped(si));
    }
  }
  __syncthreads();

  PhaseCtx<R> ctx;
  ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
  ctx.tb = 0;
  ctx.uniform = WU;
  // the phases address the LDS by whole LDS addresses: the tile's region
  // base with the array's own address ORed in (the pass kernels declare no
  // static LDS, so the dynamic array starts at LDS address 0)
  const uint32_t rbase = lds_address(lds) | ((uint32_t)tile_in_block << (T + 3));
  for (int p = 0; p < a.n_phases; ++p) {
    const DevPhase P = load_phase(a.phases, p);
    phase_dispatch<R, WU, KIND>(reinterpret_cast<char*>(lds), rbase, P, (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs,
                          ctx, tt, TB, a.fmats + (size_t)p * kFusedWords);
    __syncthreads();
  }

  if (active) {
#pragma unroll
    for (int it = 0; it < E / 2; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * 2u;
      const uint32_t si = isl.of(it) ^ st;
      const float4 val = *reinterpret_cast<const float4*>(region + pair_slot(si));
      *reinterpret_cast<float4*>(Bt + tile_offset(i, a.lo_bits, a.win_lo)) = pair_order(val, pair_swapped(si));
    }
  }
}

// KIND 0: the bond-two phase forms (staircases, DUP, fused); KIND 1: the
// bond-four ones (dense phases and single uncontrolled updates).
template <int R, bool MULTI, bool WU, int NT = kBlock, int KIND = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(pass_waves_per_eu<R, WU, NT>()))) void k_pass(
    PassArgs a) {
  extern __shared__ float2 lds[];
  pass_body<R, MULTI, WU, NT, KIND>(a, lds, blockIdx.x, gridDim.x);
}

template <int R, bool MULTI, bool WU, int NT = kBlock, int KIND = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(pass_waves_per_eu<R, WU, NT>()))) void k_pass_g(
    const Seg<PassArgs>* __restrict__ segs) {
  extern __shared__ float2 lds[];
  const Seg<PassArgs>* s = group_seg(segs);
  if (!s) return;
  const PassArgs a = s->a;
  pass_body<R, MULTI, WU, NT, KIND>(a, lds, blockIdx.x, s->gx);
}

// The pass kernel on 16-bit block-scaled storage: the same tiles, phases,
// block shapes and XCD-contiguous tile order as k_pass, with the entries
// decoded (value = stored x block scale of the previous writer) on the way
// into LDS, and re-encoded on the way out with a fresh power-of-two scale
// per block of this pass's tiles (taken from the block's largest component
// after the pass).  4 entries (16 bytes) per HBM access, 2 when a thread
// holds only 2 entries.
template <int R, bool MULTI, int S, bool WU, int NT = kBlock, int KIND = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(pass_waves_per_eu<R, WU, NT>()))) void k_pass16(
    PassArgs a) {
  extern __shared__ float2 lds[];
  constexpr int E = 1 << R;
  constexpr int U = E >= 4 ? 4 : 2;
  const int T = a.T;
  const int TB = T - R;
  const int tid = threadIdx.x;
  const int tile_in_block = MULTI ? (tid >> TB) : 0;
  const uint32_t tt = MULTI ? (uint32_t)(tid & ((1 << TB) - 1)) : (uint32_t)tid;
  const int tiles_per_block = MULTI ? (NT >> TB) : 1;
  const long long tile = (long long)xcd_block(blockIdx.x, gridDim.x) * tiles_per_block + tile_in_block;
  const bool active = tile < a.n_tiles;
  const int tbits = a.h - T;
  long long batch = active ? (tile >> tbits) : 0;
  if constexpr (WU) batch = __builtin_amdgcn_readfirstlane((int)batch);
  const unsigned long long blk = active ? ((unsigned long long)tile & ((1ull << tbits) - 1ull)) : 0ull;
  const uint64_t boff = block_offset(blk, a.lo_bits, a.win_lo, a.win_len);
  uint32_t* __restrict__ Bw = reinterpret_cast<uint32_t*>(a.B) + (batch << a.h);
  const float* __restrict__ sin = a.scale_in + batch * a.scale_stride;
  char* region = reinterpret_cast<char*>(lds) + ((size_t)tile_in_block << (T + 3));
  uint32_t* smax = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(lds) + ((size_t)tiles_per_block << (T + 3)));
  const int tpt = 1 << TB;
  const int blk_bits = T < 12 ? T : 12;
  const int nblk = 1 << (T - blk_bits);  // scale blocks per tile (1, 2 or 4)
  if (tid < nblk * tiles_per_block) smax[tid] = 0u;

  // A scale slot gathers bit fields of the entry index, and the block part
  // (boff), the thread part (tt) and the iteration part (it) of an entry's
  // index occupy disjoint bits, so its slot is the OR of the three parts'
  // slots; the iteration part is the same for every thread (scalar work).
  const uint64_t slot_t = scale_slot(boff, a.in_map) |
                          scale_slot(tile_offset(tt * (uint32_t)U, a.lo_bits, a.win_lo), a.in_map);
  const uint32_t st = swz(tt * (uint32_t)U);  // LDS slot of the thread part (see k_pass)
  const IterSlots isl(TB + (U == 4 ? 2 : 1));
  if (active) {
    // every load (and its scale) in flight before the first LDS write
    uint4 ld[E / U];
    float scl[E / U];
#pragma unroll
    for (int it = 0; it < E / U; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * (uint32_t)U;
      const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
      const uint64_t slot_i = scale_slot(tile_offset((uint32_t)(it * tpt) * (uint32_t)U, a.lo_bits, a.win_lo), a.in_map);
      scl[it] = sin[slot_t | slot_i];
      if constexpr (U == 4) {
        ld[it] = *reinterpret_cast<const uint4*>(Bw + g);
      } else {
        const uint2 w = *reinterpret_cast<const uint2*>(Bw + g);
        ld[it] = make_uint4(w.x, w.y, 0u, 0u);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int it = 0; it < E / U; ++it) {
      const float sc = scl[it];
      const uint32_t si = isl.of(it) ^ st;  // swz(i); swz(i + 2) = si ^ 2
      const uint4 w = ld[it];
      const float2 e0 = unpack16<S>(w.x, sc), e1 = unpack16<S>(w.y, sc);
      *reinterpret_cast<float4*>(region + pair_slot(si)) =
          pair_order(make_float4(e0.x, e0.y, e1.x, e1.y), pair_swapped(si));
      if constexpr (U == 4) {
        const float2 e2 = unpack16<S>(w.z, sc), e3 = unpack16<S>(w.w, sc);
        *reinterpret_cast<float4*>(region + pair_slot(si ^ 2u)) =
            pair_order(make_float4(e2.x, e2.y, e3.x, e3.y), pair_swapped(si));
      }
    }
  }
  __syncthreads();

  PhaseCtx<R> ctx;
  ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
  ctx.tb = 0;
  ctx.uniform = WU;
  for (int p = 0; p < a.n_phases; ++p) {
    const DevPhase P = load_phase(a.phases, p);
    phase_dispatch<R, WU, KIND>(reinterpret_cast<char*>(lds), lds_address(lds) | ((uint32_t)tile_in_block << (T + 3)), P,
                          (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx, tt, TB,
                          a.fmats + (size_t)p * kFusedWords);
    __syncthreads();
  }

  // largest component of each scale block of the tile (the blocks are the
  // tile's highest local bits, so a thread's entries fall in the block of
  // their iteration part: one running maximum per block)
  if (active) {
    float m[4] = {0.f, 0.f, 0.f, 0.f};
    const uint32_t st2 = swz(tt * 2u);
    const IterSlots isl2(TB + 1);
#pragma unroll
    for (int it = 0; it < E / 2; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * 2u;
      const float4 v = *reinterpret_cast<const float4*>(region + pair_slot(isl2.of(it) ^ st2));  // order irrelevant
      const float am = fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w)));
      const uint32_t q = (i >> blk_bits) & 3u;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (q == (uint32_t)c) m[c] = fmaxf(m[c], am);
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (c < nblk && m[c] > 0.f) atomicMax(&smax[nblk * tile_in_block + c], __float_as_uint(m[c]));
  }
  __syncthreads();
  if (active) {
    float inv[4];
#pragma unroll
    for (int c = 0; c < 4; ++c)
      inv[c] = c < nblk ? ldexpf(1.f, -block_exponent(__uint_as_float(smax[nblk * tile_in_block + c]))) : 1.f;
#pragma unroll
    for (int it = 0; it < E / U; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * (uint32_t)U;
      const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
      const uint32_t q = (i >> blk_bits) & 3u;
      const float iv = q == 0 ? inv[0] : q == 1 ? inv[1] : q == 2 ? inv[2] : inv[3];
      const uint32_t si = isl.of(it) ^ st;
      const float4 v0 = pair_order(*reinterpret_cast<const float4*>(region + pair_slot(si)), pair_swapped(si));
      if constexpr (U == 4) {
        const float4 v1 = pair_order(*reinterpret_cast<const float4*>(region + pair_slot(si ^ 2u)), pair_swapped(si));
        *reinterpret_cast<uint4*>(Bw + g) = make_uint4(pack16<S>(v0.x, v0.y, iv), pack16<S>(v0.z, v0.w, iv),
                                                       pack16<S>(v1.x, v1.y, iv), pack16<S>(v1.z, v1.w, iv));
      } else {
        *reinterpret_cast<uint2*>(Bw + g) = make_uint2(pack16<S>(v0.x, v0.y, iv), pack16<S>(v0.z, v0.w, iv));
      }
    }
    if (tt < (uint32_t)nblk) {
      float* sout = a.scale_out + batch * a.scale_stride + ((long long)blk << (T - blk_bits));
      sout[tt] = ldexpf(1.f, block_exponent(__uint_as_float(smax[nblk * tile_in_block + tt])));
    }
  }
}

// ---------------------------------------------------------------------------
// Launch records.

template <class A>
static void set_arg(Launch* L, const A& a) {
  static_assert(sizeof(A) <= kMaxArgBytes, "kernel argument too large for a launch record");
  std::memset(L->arg, 0, sizeof(L->arg));
  std::memcpy(L->arg, &a, sizeof(A));
  L->arg_bytes = (uint32_t)sizeof(A);
  L->seg_stride = (uint32_t)sizeof(Seg<A>);
}

static hipError_t set_shape(Launch* L, long long blocks_x, unsigned blocks_y, unsigned threads, size_t shmem) {
  if (blocks_x <= 0 || blocks_x > 0x7fffffffLL || blocks_y == 0 || blocks_y > 65535) return hipErrorInvalidValue;
  L->grid = dim3((unsigned)blocks_x, blocks_y, 1);
  L->block = dim3(threads, 1, 1);
  L->shmem = (uint32_t)shmem;
  return hipSuccess;
}

hipError_t record_init(const InitArgs& a, Launch* L) {
  *L = Launch();
  L->cls = 0;
  if (a.store == STORE_C64) {
    if (a.m0 - 1 > 64) return hipErrorInvalidValue;
    const long long threads = a.h < 11 ? ((long long)a.n_batches << a.h) : (((long long)a.n_batches << a.h) >> 5);
    L->fn = reinterpret_cast<const void*>(&k_init);
    L->gfn = reinterpret_cast<const void*>(&k_init_g);
    set_arg(L, a);
    return set_shape(L, (threads + kBlock - 1) / kBlock, 1, kBlock, 0);
  }
  if (a.m0 - 1 > 64 || a.blk_bits > 12 || a.blk_bits < 0 || a.blk_bits > a.h) return hipErrorInvalidValue;
  if (a.store == STORE_F16) L->fn = reinterpret_cast<const void*>(&k_init16<STORE_F16>);
  else if (a.store == STORE_BF16) L->fn = reinterpret_cast<const void*>(&k_init16<STORE_BF16>);
  else return hipErrorInvalidValue;
  set_arg(L, a);
  return set_shape(L, (long long)a.n_batches << (a.h - a.blk_bits), 1, kBlock, 0);
}

hipError_t record_resolve(const ResolveArgs& a, Launch* L) {
  *L = Launch();
  L->cls = 0;
  const long long total = (long long)a.n_batches * a.n_ops;
  if (total <= 0) return hipErrorInvalidValue;
  L->fn = reinterpret_cast<const void*>(&k_resolve);
  L->gfn = reinterpret_cast<const void*>(&k_resolve_g);
  set_arg(L, a);
  return set_shape(L, (total + kBlock - 1) / kBlock, 1, kBlock, 0);
}

template <int R, int NT, bool MULTI, bool WU>
static void pick_pass(Launch* L, int kind) {
  if (kind == 1) {
    L->fn = reinterpret_cast<const void*>(&k_pass<R, MULTI, WU, NT, 1>);
    L->gfn = reinterpret_cast<const void*>(&k_pass_g<R, MULTI, WU, NT, 1>);
  } else {
    L->fn = reinterpret_cast<const void*>(&k_pass<R, MULTI, WU, NT, 0>);
    L->gfn = reinterpret_cast<const void*>(&k_pass_g<R, MULTI, WU, NT, 0>);
  }
}

template <int R, int NT, bool MULTI, bool WU>
static void pick_pass16(Launch* L, int store, int kind) {
  if (kind == 1) {
    if (store == STORE_F16) L->fn = reinterpret_cast<const void*>(&k_pass16<R, MULTI, STORE_F16, WU, NT, 1>);
    else L->fn = reinterpret_cast<const void*>(&k_pass16<R, MULTI, STORE_BF16, WU, NT, 1>);
  } else {
    if (store == STORE_F16) L->fn = reinterpret_cast<const void*>(&k_pass16<R, MULTI, STORE_F16, WU, NT, 0>);
    else L->fn = reinterpret_cast<const void*>(&k_pass16<R, MULTI, STORE_BF16, WU, NT, 0>);
  }
}

// Block shape of a pass: one 2^(R+9)-entry tile per 512-thread block, one
// 2^(R+8)-entry tile per 256-thread block, or several smaller tiles per
// 256-thread block (their waves lie inside one tile when T - R >= 6).
template <int R>
static hipError_t record_pass_r(const PassArgs& a, Launch* L) {
  const int TB = a.T - R;
  if (TB < 0 || TB > 9) return hipErrorInvalidValue;
  const bool s16 = a.store == STORE_F16 || a.store == STORE_BF16;
  if (!s16 && a.store != STORE_C64) return hipErrorInvalidValue;
  const int NT = TB == 9 ? 512 : kBlock;
  const bool multi = TB < 8;
  const int tiles_per_block = multi ? (kBlock >> TB) : 1;
  const long long blocks = ((long long)a.n_tiles + tiles_per_block - 1) / tiles_per_block;
  size_t lds = (size_t)tiles_per_block << (a.T + 3);
  if (s16) lds += (size_t)4 * NT;  // per-tile block maxima
  if (a.kind != 0 && a.kind != 1) return hipErrorInvalidValue;
  if (TB == 9) {
    if (s16) pick_pass16<R, 512, false, true>(L, a.store, a.kind);
    else pick_pass<R, 512, false, true>(L, a.kind);
  } else if (!multi) {
    if (s16) pick_pass16<R, kBlock, false, true>(L, a.store, a.kind);
    else pick_pass<R, kBlock, false, true>(L, a.kind);
  } else if (TB >= 6) {
    if (s16) pick_pass16<R, kBlock, true, true>(L, a.store, a.kind);
    else pick_pass<R, kBlock, true, true>(L, a.kind);
  } else {
    if (s16) pick_pass16<R, kBlock, true, false>(L, a.store, a.kind);
    else pick_pass<R, kBlock, true, false>(L, a.kind);
  }
  set_arg(L, a);
  return set_shape(L, blocks, 1, NT, lds);
}

hipError_t record_pass(const PassArgs& a, int R, Launch* L) {
  *L = Launch();
  L->cls = 1;
  switch (R) {
    case 1: return record_pass_r<1>(a, L);
    case 2: return record_pass_r<2>(a, L);
    case 3: return record_pass_r<3>(a, L);
    case 4: return record_pass_r<4>(a, L);
    case 5: return record_pass_r<5>(a, L);
    default: return hipErrorInvalidValue;
  }
}

hipError_t issue(const Launch& L, hipStream_t s) {
  void* args[1] = {const_cast<unsigned char*>(L.arg)};
  return hipLaunchKernel(L.fn, L.grid, L.block, args, L.shmem, s);
}

hipError_t graph_add(const Launch& L, hipGraph_t g, hipGraphNode_t* node, const hipGraphNode_t* dep, size_t n_dep) {
  hipKernelNodeParams kp;
  std::memset(&kp, 0, sizeof(kp));
  void* args[1] = {const_cast<unsigned char*>(L.arg)};
  kp.func = const_cast<void*>(L.fn);
  kp.gridDim = L.grid;
  kp.blockDim = L.block;
  kp.sharedMemBytes = L.shmem;
  kp.kernelParams = args;
  kp.extra = nullptr;
  return hipGraphAddKernelNode(node, g, dep, n_dep, &kp);
}

bool groupable(const Launch& a, const Launch& b) {
  return a.gfn && a.fn == b.fn && a.gfn == b.gfn && a.block.x == b.block.x && a.seg_stride == b.seg_stride;
}

size_t write_segments(const Launch* const* members, int n, unsigned char* dst) {
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    const Launch& L = *members[i];
    std::memset(dst + off, 0, L.seg_stride);
    const uint32_t g[2] = {L.grid.x, L.grid.y};
    std::memcpy(dst + off, g, sizeof(g));
    std::memcpy(dst + off + kSegHeader, L.arg, L.arg_bytes);
    off += L.seg_stride;
  }
  return off;
}

hipError_t issue_grouped(const Launch* const* members, int n, const void* d_segs, hipStream_t s) {
  if (n < 1 || n > 65535 || !d_segs) return hipErrorInvalidValue;
  const Launch& L0 = *members[0];
  unsigned gx = 0, gy = 0;
  uint32_t shmem = 0;
  for (int i = 0; i < n; ++i) {
    if (!groupable(L0, *members[i])) return hipErrorInvalidValue;
    gx = std::max(gx, members[i]->grid.x);
    gy = std::max(gy, members[i]->grid.y);
    shmem = std::max(shmem, members[i]->shmem);
  }
  void* args[1] = {(void*)&d_segs};
  return hipLaunchKernel(L0.gfn, dim3(gx, gy, (unsigned)n), L0.block, args, shmem, s);
}

// Host emulation of a fused phase, wave by wave, with the lane layout of
// phase_tri: D[4 g + r][j] = sum_k A[4 g + r][k] B[k][j], A[i][k] from the
// operand table of lane i + 16 (k % 4) at step k / 4, B[k][j] the step-(k/4)
// value of lane 16 (k % 4) + j.  FP32 sums in step order.
template <int R>
static void emulate_tri(char* region, const DevPhase& P, const uint32_t* po, const float4* F, const float* rm, int TB) {
  constexpr int E = 1 << R;
  constexpr int G = E / 2;
  const int tpt = 1 << TB;
  auto comp = [](const float4& q, int st) { return st == 0 ? q.x : st == 1 ? q.y : st == 2 ? q.z : q.w; };
  for (int w0 = 0; w0 < tpt; w0 += 64) {
    static thread_local float vx[64][E], vy[64][E];
    uint32_t off[64][E];
    for (int l = 0; l < 64; ++l) {
      const uint32_t tt = (uint32_t)(w0 + l);
      uint32_t vb = 0;
      for (int t = 0; t < TB; ++t)
        if ((tt >> t) & 1u) vb ^= po[kPhaseEntries + t];
      for (int i = 0; i < E; ++i) {
        off[l][i] = vb ^ po[i];
        const float2 x = *reinterpret_cast<const float2*>(region + off[l][i]);
        vx[l][i] = x.x;
        vy[l][i] = x.y;
      }
    }
    for (int j = 0; j < G; ++j) {
      const float4* A = F + (j >= G / 2 ? 64 : 0);
      float out[64][4];
      for (int l = 0; l < 64; ++l) {
        const int g = l / 16, jj = l % 16;
        for (int r = 0; r < 4; ++r) {
          const int i = 4 * g + r;
          float d = 0.f;
          for (int st = 0; st < 4; ++st)
            for (int gg = 0; gg < 4; ++gg) {
              const int src = 16 * gg + jj;
              const float b = st == 0 ? vx[src][2 * j] : st == 1 ? vy[src][2 * j] : st == 2 ? vx[src][2 * j + 1]
                                                                                         : vy[src][2 * j + 1];
              d = std::fma(comp(A[i + 16 * gg], st), b, d);
            }
          out[l][r] = d;
        }
      }
      for (int l = 0; l < 64; ++l) {
        vx[l][2 * j] = out[l][0];
        vy[l][2 * j] = out[l][1];
        vx[l][2 * j + 1] = out[l][2];
        vy[l][2 * j + 1] = out[l][3];
      }
    }
    // the staircase tail (a unit phase: the next step's 4x4s), lane by lane
    for (int l = 0; l < 64; ++l) {
      Regs<R> v;
      for (int i = 0; i < E; ++i) {
        v.x[i] = vx[l][i];
        v.y[i] = vy[l][i];
      }
      if (P.pad == 3) {
        if (P.n_ops == 8) {
          v = op_dense<R, 1, 2>(v, rm + (size_t)(P.op_begin + 4) * 16);
          v = op_dense<R, 0, 2>(v, rm + (size_t)(P.op_begin + 6) * 16);
        }
        for (int i = 0; i < E; ++i) {
          vx[l][i] = v.x[i];
          vy[l][i] = v.y[i];
        }
        continue;
      }
      if (P.n_ops >= 4) v = op_sel<R, 1>(v, rm + (size_t)(P.op_begin + 3) * 16 + 8 * ((l >> 5) & 1));
      if (P.n_ops >= 5) v = op_reg<R, 2, 1>(v, (const TNC_TBL float*)(rm + (size_t)(P.op_begin + 4) * 16));
      if constexpr (R >= 4) {
        if (P.n_ops >= 6) v = op_reg<R, 3, 2>(v, (const TNC_TBL float*)(rm + (size_t)(P.op_begin + 5) * 16));
      }
      if constexpr (R >= 5) {
        if (P.n_ops >= 7) v = op_reg<R, 4, 3>(v, (const TNC_TBL float*)(rm + (size_t)(P.op_begin + 6) * 16));
      }
      for (int i = 0; i < E; ++i) {
        vx[l][i] = v.x[i];
        vy[l][i] = v.y[i];
      }
    }
    for (int l = 0; l < 64; ++l)
      for (int i = 0; i < E; ++i) *reinterpret_cast<float2*>(region + off[l][i]) = make_float2(vx[l][i], vy[l][i]);
  }
}

// Host emulation with the same helpers and the same LDS placement.
template <int R>
static void emulate_pass_r(const PassArgs& a) {
  constexpr int E = 1 << R;
  const int T = a.T, TB = T - R;
  const int tpt = 1 << TB;
  const int tbits = a.h - T;
  std::vector<float2> lds((size_t)1 << T);
  char* region = reinterpret_cast<char*>(lds.data());
  const bool s16 = a.store == STORE_F16 || a.store == STORE_BF16;
  auto dec = [&](uint32_t w, float sc) {
    return a.store == STORE_F16 ? unpack16<STORE_F16>(w, sc) : unpack16<STORE_BF16>(w, sc);
  };
  auto enc = [&](float2 v, float inv) {
    return a.store == STORE_F16 ? pack16<STORE_F16>(v.x, v.y, inv) : pack16<STORE_BF16>(v.x, v.y, inv);
  };
  const int blk_bits = T < 12 ? T : 12;
  for (long long tile = 0; tile < a.n_tiles; ++tile) {
    const long long batch = tile >> tbits;
    const unsigned long long blk = (unsigned long long)tile & ((1ull << tbits) - 1ull);
    const uint64_t boff = block_offset(blk, a.lo_bits, a.win_lo, a.win_len);
    float2* Bt = a.B + (batch << a.h) + boff;
    uint32_t* Bw = reinterpret_cast<uint32_t*>(a.B) + (batch << a.h);
    for (int tt = 0; tt < tpt; ++tt)
      for (int it = 0; it < E / 2; ++it) {
        const uint32_t i = (uint32_t)(it * tpt + tt) * 2u;
        if (s16) {
          const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
          const float sc = a.scale_in[batch * a.scale_stride + (long long)scale_slot(g, a.in_map)];
          lds[swz(i)] = dec(Bw[g], sc);
          lds[swz(i + 1u)] = dec(Bw[g + 1], sc);
        } else {
          const float2* src = Bt + tile_offset(i, a.lo_bits, a.win_lo);
          lds[swz(i)] = src[0];
          lds[swz(i + 1u)] = src[1];
        }
      }
    PhaseCtx<R> ctx;
    ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
    ctx.tb = 0;
    ctx.uniform = false;
    for (int p = 0; p < a.n_phases; ++p) {
      const DevPhase P = load_phase(a.phases, p);
      if (P.pad == 1 || P.pad == 3) {
        if constexpr (R >= 3)
          emulate_tri<R>(region, P, a.poffs + p * kPhaseOffs, a.fmats + (size_t)p * kFusedWords,
                         a.rmats + (size_t)batch * a.rstride, TB);
        continue;
      }
      for (int tt = 0; tt < tpt; ++tt)
        if (a.kind == 1)
          phase_dispatch<R, false, 1>(region, 0u, P, (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx,
                                      (uint32_t)tt, TB);
        else
          phase_dispatch<R, false, 0>(region, 0u, P, (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx,
                                      (uint32_t)tt, TB);
    }
    if (s16) {
      const int nblk = 1 << (T - blk_bits);
      float amax[4] = {0.f, 0.f, 0.f, 0.f};
      for (uint32_t i = 0; i < (1u << T); ++i) {
        const float2 v = lds[swz(i)];
        float& m = amax[(i >> blk_bits) & 3u];
        m = std::max(m, std::max(std::fabs(v.x), std::fabs(v.y)));
      }
      int ex[4];
      for (int c = 0; c < 4; ++c) ex[c] = block_exponent(amax[c]);
      for (uint32_t i = 0; i < (1u << T); ++i) {
        const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
        Bw[g] = enc(lds[swz(i)], std::ldexp(1.f, -ex[(i >> blk_bits) & 3u]));
      }
      float* sout = a.scale_out + batch * a.scale_stride + ((long long)blk << (T - blk_bits));
      for (int c = 0; c < nblk; ++c) sout[c] = std::ldexp(1.f, ex[c]);
      continue;
    }
    for (int tt = 0; tt < tpt; ++tt)
      for (int it = 0; it < E / 2; ++it) {
        const uint32_t i = (uint32_t)(it * tpt + tt) * 2u;
        float2* dst = Bt + tile_offset(i, a.lo_bits, a.win_lo);
        dst[0] = lds[swz(i)];
        dst[1] = lds[swz(i + 1u)];
      }
  }
}

void emulate_pass_host(const PassArgs& a, int R) {
  switch (R) {
    case 1: emulate_pass_r<1>(a); break;
    case 2: emulate_pass_r<2>(a); break;
    case 3: emulate_pass_r<3>(a); break;
    case 4: emulate_pass_r<4>(a); break;
    case 5: emulate_pass_r<5>(a); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Late phase: out[b][r][c] = sum_kk in[b][r][kk] * J[var][kk][c] in FP64.
// J folds, on the host, the early-region tensor Z_early (first launch), the
// late layers' one- and two-qubit gates and the removal of the crossing
// bonds between the fixed rows and the open band (Alg. 2).  Tiled 64 x 64
// per block, K in steps of 16, 4 x 4 complex accumulators per thread.
__device__ inline double2 to_d2(float2 v) { return make_double2((double)v.x, (double)v.y); }
__device__ inline double2 to_d2(double2 v) { return v; }

// Entry g of batch b of the first late launch's input, in FP64.
template <typename TIn, int S>
__device__ inline double2 late_in(const LateArgs& a, const TIn* __restrict__ in, int b, uint64_t g) {
  if constexpr (S == STORE_F16 || S == STORE_BF16) {
    const float sc = a.scale_in[(long long)b * a.scale_stride + (long long)scale_slot(g, a.in_map)];
    return to_d2(unpack16<S>(in[g], sc));
  } else {
    return to_d2(in[g]);
  }
}

template <typename TIn, int S>
__device__ __attribute__((always_inline)) inline void late_body(const LateArgs& a, uint32_t bx, uint32_t by) {
  __shared__ double2 As[16][65];
  __shared__ double2 Bs[16][65];
  const int b = by;
  const int tilesN = (a.N + 63) / 64;
  const int tilesM = (a.M + 63) / 64;
  // Consecutive block ids go to different XCDs (round robin over 8); the
  // tilesN column blocks of one row tile are given ids that land on the
  // same XCD, so they share its L2 for the row tile.
  const int xcd = bx & 7;
  const int g = bx >> 3;
  const int bn = g % tilesN;
  const int bm = (g / tilesN) * 8 + xcd;
  if (bm >= tilesM) return;
  const int row0 = bm * 64, col0 = bn * 64;
  const int var = a.xrow >= 0 ? (int)a.bits[(size_t)b * a.n + a.xrow] : 0;
  const double2* __restrict__ J = a.J + (size_t)var * a.K * a.N;
  const TIn* __restrict__ in = reinterpret_cast<const TIn*>(a.in) + (size_t)b * a.in_batch_stride;
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  double2 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = make_double2(0.0, 0.0);
  for (int k0 = 0; k0 < a.K; k0 += 16) {
    for (int e = tid; e < 1024; e += kBlock) {
      const int r = e >> 4, kk = e & 15;
      const int row = row0 + r;
      double2 val = make_double2(0.0, 0.0);
      if (row < a.M && k0 + kk < a.K) val = late_in<TIn, S>(a, in, b, (uint64_t)row * a.K + k0 + kk);
      As[kk][r] = val;
    }
    for (int e = tid; e < 1024; e += kBlock) {
      const int kk = e >> 6, c = e & 63;
      const int col = col0 + c;
      double2 val = make_double2(0.0, 0.0);
      if (col < a.N && k0 + kk < a.K) val = J[(size_t)(k0 + kk) * a.N + col];
      Bs[kk][c] = val;
    }
    __syncthreads();
#pragma unroll 4
    for (int kk = 0; kk < 16; ++kk) {
      double2 av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][tr * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tc * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j].x += av[i].x * bv[j].x - av[i].y * bv[j].y;
          acc[i][j].y += av[i].x * bv[j].y + av[i].y * bv[j].x;
        }
    }
    __syncthreads();
  }
  double2* out = a.out + (size_t)b * a.out_batch_stride;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + tr * 4 + i;
    if (row >= a.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = col0 + tc * 4 + j;
      if (col < a.N) out[(size_t)row * a.N + col] = acc[i][j];
    }
  }
}

template <typename TIn, int S>
__global__ __launch_bounds__(kBlock) void k_late(LateArgs a) { late_body<TIn, S>(a, blockIdx.x, blockIdx.y); }

template <typename TIn, int S>
__global__ __launch_bounds__(kBlock) void k_late_g(const Seg<LateArgs>* __restrict__ segs) {
  const Seg<LateArgs>* s = group_seg(segs);
  if (!s) return;
  const LateArgs a = s->a;
  late_body<TIn, S>(a, blockIdx.x, blockIdx.y);
}

// The same contraction on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
// a 64 x 64 output tile per 256-thread block, 32 x 32 (2 x 2 MFMA tiles)
// per wave; the complex product takes four real MFMAs per tile and k-step
// (re += ar*br - ai*bi, im += ar*bi + ai*br).  Lane l supplies A[l%16][k]
// and B[k][l%16] with k = l/16 and receives D[l/16 + 4q][l%16], q < 4.
typedef double tnc_d4 __attribute__((ext_vector_type(4)));

template <typename TIn, int S>
__device__ __attribute__((always_inline)) inline void late_mf_body(const LateArgs& a, uint32_t bx, uint32_t by) {
  __shared__ double2 As[16][65];
  __shared__ double2 Bs[16][65];
  const int b = by;
  const int tilesN = (a.N + 63) / 64;
  const int tilesM = (a.M + 63) / 64;
  const int xcd = bx & 7;
  const int g = bx >> 3;
  const int bn = g % tilesN;
  const int bm = (g / tilesN) * 8 + xcd;
  if (bm >= tilesM) return;
  const int row0 = bm * 64, col0 = bn * 64;
  const int var = a.xrow >= 0 ? (int)a.bits[(size_t)b * a.n + a.xrow] : 0;
  const double2* __restrict__ J = a.J + (size_t)var * a.K * a.N;
  const TIn* __restrict__ in = reinterpret_cast<const TIn*>(a.in) + (size_t)b * a.in_batch_stride;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int li = lane & 15, lk = lane >> 4;
  tnc_d4 cr[2][2], ci[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = tnc_d4{0.0, 0.0, 0.0, 0.0};
      ci[i][j] = tnc_d4{0.0, 0.0, 0.0, 0.0};
    }
  // the next k-slice of A and B is loaded into registers while the current
  // one is multiplied from LDS (kBlock = 256 threads: 4 elements each)
  double2 pa[4], pb[4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * kBlock;
      const int r = e >> 4, kk = e & 15;
      const int row = row0 + r;
      pa[q] = make_double2(0.0, 0.0);
      if (row < a.M && k0 + kk < a.K) pa[q] = late_in<TIn, S>(a, in, b, (uint64_t)row * a.K + k0 + kk);
      const int kb = e >> 6, c = e & 63;
      const int col = col0 + c;
      pb[q] = make_double2(0.0, 0.0);
      if (col < a.N && k0 + kb < a.K) pb[q] = J[(size_t)(k0 + kb) * a.N + col];
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < a.K; k0 += 16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * kBlock;
      As[e & 15][e >> 4] = pa[q];
      Bs[e >> 6][e & 63] = pb[q];
    }
    __syncthreads();
    if (k0 + 16 < a.K) fetch(k0 + 16);
#pragma unroll
    for (int kc = 0; kc < 4; ++kc) {
      const int kk = kc * 4 + lk;
      double2 av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[kk][wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[kk][wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].x, cr[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-av[i].y, bv[j].y, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].x, bv[j].y, ci[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i].y, bv[j].x, ci[i][j], 0, 0, 0);
        }
    }
    __syncthreads();
  }
  double2* out = a.out + (size_t)b * a.out_batch_stride;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = row0 + wr + 16 * i + lk + 4 * q;
        const int col = col0 + wc + 16 * j + li;
        if (row < a.M && col < a.N) out[(size_t)row * a.N + col] = make_double2(cr[i][j][q], ci[i][j][q]);
      }
}

template <typename TIn, int S>
__global__ __launch_bounds__(kBlock) void k_late_mf(LateArgs a) { late_mf_body<TIn, S>(a, blockIdx.x, blockIdx.y); }

template <typename TIn, int S>
__global__ __launch_bounds__(kBlock) void k_late_mf_g(const Seg<LateArgs>* __restrict__ segs) {
  const Seg<LateArgs>* s = group_seg(segs);
  if (!s) return;
  const LateArgs a = s->a;
  late_mf_body<TIn, S>(a, blockIdx.x, blockIdx.y);
}

hipError_t record_late(const LateArgs& a, bool in_c64, Launch* L) {
  *L = Launch();
  L->cls = 2;
  const long long tilesM8 = ((long long)(a.M + 63) / 64 + 7) / 8 * 8;
  const long long tiles = tilesM8 * ((a.N + 63) / 64);
  // matrix cores for contractions large enough to fill their 16 x 16 tiles
  const bool mf = in_c64 && a.N >= 32 && a.K >= 16 && a.M >= 64;
  if (!in_c64) {
    L->fn = reinterpret_cast<const void*>(&k_late<double2, STORE_C64>);
    L->gfn = reinterpret_cast<const void*>(&k_late_g<double2, STORE_C64>);
  } else if (a.store == STORE_F16) {
    L->fn = mf ? reinterpret_cast<const void*>(&k_late_mf<uint32_t, STORE_F16>)
               : reinterpret_cast<const void*>(&k_late<uint32_t, STORE_F16>);
  } else if (a.store == STORE_BF16) {
    L->fn = mf ? reinterpret_cast<const void*>(&k_late_mf<uint32_t, STORE_BF16>)
               : reinterpret_cast<const void*>(&k_late<uint32_t, STORE_BF16>);
  } else if (a.store == STORE_C64) {
    L->fn = mf ? reinterpret_cast<const void*>(&k_late_mf<float2, STORE_C64>)
               : reinterpret_cast<const void*>(&k_late<float2, STORE_C64>);
    L->gfn = mf ? reinterpret_cast<const void*>(&k_late_mf_g<float2, STORE_C64>)
                : reinterpret_cast<const void*>(&k_late_g<float2, STORE_C64>);
  } else {
    return hipErrorInvalidValue;
  }
  set_arg(L, a);
  if (a.n_batches < 1) return hipErrorInvalidValue;
  return set_shape(L, tiles, (unsigned)a.n_batches, kBlock, 0);
}

// ---------------------------------------------------------------------------
// Late program on the shrinking tensor, FP64.  A block loads 2^j consecutive
// rows of 2^s state entries into LDS; one- and two-qubit gates act on the
// state bits of every live row, a removal sums the lowest remaining row bit
// against C_u on state bit 0 (Alg. 2, the late ContractLayer steps).  After
// l removals the live rows are those whose low l row bits are zero.
__device__ inline double2 zfma2(double2 m0, double2 x0, double2 m1, double2 x1) {
  return make_double2(m0.x * x0.x - m0.y * x0.y + m1.x * x1.x - m1.y * x1.y,
                      m0.x * x0.y + m0.y * x0.x + m1.x * x1.y + m1.y * x1.x);
}

__device__ inline int insert_zero(int x, int bit) {
  const int lo = x & ((1 << bit) - 1);
  return ((x - lo) << 1) | lo;
}

__device__ __attribute__((always_inline)) inline void late_ops_body(const LateOpsArgs& a, double2* st, uint32_t bx,
                                                                    uint32_t by) {
  const long long row_out = bx;
  const int b = by;
  const int sb = a.s;
  const int total = 1 << (sb + a.j);
  const double2* in = a.in + (size_t)b * a.in_batch_stride + ((size_t)row_out << (a.j + sb));
  for (int i = threadIdx.x; i < total; i += blockDim.x) st[i] = in[i];
  __syncthreads();
  int l = 0;
  for (int o = 0; o < a.n_prog; ++o) {
    const LateOpDev& op = a.prog[o];
    const int live = a.j - l;
    if (op.kind == 1) {
      const int items = (1 << live) << (sb - 1);
      for (int w = threadIdx.x; w < items; w += blockDim.x) {
        const int r = (w >> (sb - 1)) << l;
        const int t0 = insert_zero(w & ((1 << (sb - 1)) - 1), op.a);
        const int i0 = (r << sb) | t0, i1 = i0 | (1 << op.a);
        const double2 x0 = st[i0], x1 = st[i1];
        st[i0] = zfma2(op.m[0], x0, op.m[1], x1);
        st[i1] = zfma2(op.m[2], x0, op.m[3], x1);
      }
    } else if (op.kind == 2) {
      const int items = (1 << live) << (sb - 2);
      for (int w = threadIdx.x; w < items; w += blockDim.x) {
        const int r = (w >> (sb - 2)) << l;
        const int t0 = insert_zero(insert_zero(w & ((1 << (sb - 2)) - 1), op.a), op.a + 1);
        const int base = (r << sb) | t0;
        const int idx[4] = {base, base | (1 << (op.a + 1)), base | (1 << op.a), base | (3 << op.a)};
        double2 x[4], y[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = st[idx[u]];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double2 p0 = zfma2(op.m[4 * q + 0], x[0], op.m[4 * q + 1], x[1]);
          const double2 p1 = zfma2(op.m[4 * q + 2], x[2], op.m[4 * q + 3], x[3]);
          y[q] = make_double2(p0.x + p1.x, p0.y + p1.y);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) st[idx[u]] = y[u];
      }
    } else if (op.kind == 3) {
      // an output-bit variant (xrow >= 0) takes the second set of matrices
      const double2* m = op.m + ((op.xrow >= 0 && (a.bits[(size_t)b * a.n + op.xrow] & 1)) ? 8 : 0);
      const int items = (1 << (live - 1)) << (sb - 1);
      for (int w = threadIdx.x; w < items; w += blockDim.x) {
        const int ra = (w >> (sb - 1)) << (l + 1);
        const int rb = ra | (1 << l);
        const int t0 = (w & ((1 << (sb - 1)) - 1)) << 1;
        const int ia = (ra << sb) | t0, ib = (rb << sb) | t0;
        const double2 x0 = st[ia], x1 = st[ia | 1], y0 = st[ib], y1 = st[ib | 1];
        const double2 o0a = zfma2(m[0], x0, m[1], x1), o0b = zfma2(m[4], y0, m[5], y1);
        const double2 o1a = zfma2(m[2], x0, m[3], x1), o1b = zfma2(m[6], y0, m[7], y1);
        st[ia] = make_double2(o0a.x + o0b.x, o0a.y + o0b.y);
        st[ia | 1] = make_double2(o1a.x + o1b.x, o1a.y + o1b.y);
      }
      ++l;
    } else if (op.kind == 6) {
      // two slots (l, l+1) at once: row u = bit l + 2 bit (l+1) takes C_u
      const int items = (1 << (live - 2)) << (sb - 1);
      for (int w = threadIdx.x; w < items; w += blockDim.x) {
        const int r0 = (w >> (sb - 1)) << (l + 2);
        const int t0 = (w & ((1 << (sb - 1)) - 1)) << 1;
        double2 o0 = make_double2(0.0, 0.0), o1 = make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int iu = ((r0 | (u << l)) << sb) | t0;
          const double2 x0 = st[iu], x1 = st[iu | 1];
          const double2 p0 = zfma2(op.m[4 * u], x0, op.m[4 * u + 1], x1);
          const double2 p1 = zfma2(op.m[4 * u + 2], x0, op.m[4 * u + 3], x1);
          o0 = make_double2(o0.x + p0.x, o0.y + p0.y);
          o1 = make_double2(o1.x + p1.x, o1.y + p1.y);
        }
        const int i0 = (r0 << sb) | t0;
        st[i0] = o0;
        st[i0 | 1] = o1;
      }
      l += 2;
    }
    __syncthreads();
  }
  double2* out = a.out + (size_t)b * a.out_batch_stride;
  if (a.final_kind == 5) {
    for (int bb = threadIdx.x; bb < (1 << a.k); bb += blockDim.x) {
      int t = 0;
      for (int q = 0; q < a.k; ++q) t |= ((bb >> (a.k - 1 - q)) & 1) << q;
      out[bb] = st[t];
    }
  } else if (a.final_kind == 4) {
    if (threadIdx.x == 0) {
      const int x = a.bits[(size_t)b * a.n + a.final_xrow];
      out[0] = zfma2(a.dot[x][0], st[0], a.dot[x][1], st[1]);
    }
  } else {
    for (int t = threadIdx.x; t < (1 << sb); t += blockDim.x) out[((size_t)row_out << sb) + t] = st[t];
  }
}

__global__ __launch_bounds__(kBlock) void k_late_ops(LateOpsArgs a) {
  extern __shared__ double2 st[];
  late_ops_body(a, st, blockIdx.x, blockIdx.y);
}

__global__ __launch_bounds__(kBlock) void k_late_ops_g(const Seg<LateOpsArgs>* __restrict__ segs) {
  extern __shared__ double2 st[];
  const Seg<LateOpsArgs>* s = group_seg(segs);
  if (!s) return;
  const LateOpsArgs a = s->a;
  late_ops_body(a, st, blockIdx.x, blockIdx.y);
}

hipError_t record_late_ops(const LateOpsArgs& a, Launch* L) {
  *L = Launch();
  L->cls = 2;
  if (a.s + a.j > 12 || a.n_batches < 1) return hipErrorInvalidValue;
  L->fn = reinterpret_cast<const void*>(&k_late_ops);
  L->gfn = reinterpret_cast<const void*>(&k_late_ops_g);
  set_arg(L, a);
  return set_shape(L, a.rows_out, (unsigned)a.n_batches, kBlock, sizeof(double2) << (a.s + a.j));
}

// ---------------------------------------------------------------------------
// The complex128 reference sweep: the same product initialisation as k_init
// kept in FP64, then every update of the sweep as its own launch, each
// thread one pair of entries.  A test path (the paper's precision study
// compares complex64 with complex128 runs, Sec. 5.1), not tuned.
__global__ __launch_bounds__(kBlock) void k_init64(InitArgs a) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long total = (long long)a.n_batches << a.h;
  if (gid >= total) return;
  const long long batch = gid >> a.h;
  const unsigned long long i = (unsigned long long)gid & ((1ull << a.h) - 1ull);
  double2* out = reinterpret_cast<double2*>(a.B) + gid;
  const int m = a.m0;
  if (i >> m) {
    *out = make_double2(0.0, 0.0);
    return;
  }
  const int x0 = a.bits[batch * a.n];
  double2 val = a.v[i & 1ull];
  for (int j = 1; j < m; ++j) {
    const int aj = (int)((i >> j) & 1ull), ajm = (int)((i >> (j - 1)) & 1ull);
    val = zmul(val, a.seg[4 * (j - 1) + 2 * aj + ajm]);
  }
  *out = zmul(val, a.f[x0][(i >> (m - 1)) & 1ull]);
}

__global__ __launch_bounds__(kBlock) void k_op64(Op64Args a) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long pairs = (long long)a.n_batches << (a.h - 1);
  if (gid >= pairs) return;
  const Op64 op = *a.op;
  const long long batch = gid >> (a.h - 1);
  const unsigned long long p = (unsigned long long)gid & ((1ull << (a.h - 1)) - 1ull);
  const unsigned long long ts = 1ull << op.target;
  const unsigned long long lo = p & (ts - 1ull);
  const unsigned long long i0 = ((p - lo) << 1) | lo, i1 = i0 | ts;
  double2* B = a.B + (batch << a.h);
  if (op.kind == 1) {
    B[i1] = B[i0];
    return;
  }
  const uint8_t* x = a.bits + (size_t)batch * a.n;
  const int var = (op.xrow0 >= 0 ? 2 * (x[op.xrow0] & 1) : 0) + (op.xrow1 >= 0 ? (x[op.xrow1] & 1) : 0);
  const int c = op.control >= 0 ? (int)((i0 >> op.control) & 1ull) : 0;
  const double2* m = op.m[var][c];
  const double2 b0 = B[i0], b1 = B[i1];
  const double2 p0 = zmul(m[0], b0), q0 = zmul(m[1], b1), p1 = zmul(m[2], b0), q1 = zmul(m[3], b1);
  B[i0] = make_double2(p0.x + q0.x, p0.y + q0.y);
  B[i1] = make_double2(p1.x + q1.x, p1.y + q1.y);
}

hipError_t launch_init64(const InitArgs& a, hipStream_t s) {
  if (a.m0 - 1 > 64 || a.h < 1) return hipErrorInvalidValue;
  const long long blocks = (((long long)a.n_batches << a.h) + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL || blocks < 1) return hipErrorInvalidValue;
  InitArgs b = a;
  return hipLaunchKernel(reinterpret_cast<const void*>(&k_init64), dim3((unsigned)blocks), dim3(kBlock),
                         std::array<void*, 1>{&b}.data(), 0, s);
}

hipError_t launch_op64(const Op64Args& a, hipStream_t s) {
  if (a.h < 1) return hipErrorInvalidValue;
  const long long blocks = (((long long)a.n_batches << (a.h - 1)) + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL || blocks < 1) return hipErrorInvalidValue;
  Op64Args b = a;
  return hipLaunchKernel(reinterpret_cast<const void*>(&k_op64), dim3((unsigned)blocks), dim3(kBlock),
                         std::array<void*, 1>{&b}.data(), 0, s);
}

// ---------------------------------------------------------------------------
// FP64 complex fill and sum (the ring's sum over slices).
__global__ __launch_bounds__(kBlock) void k_fill_zero(double2* out, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = make_double2(0.0, 0.0);
}

// A launch whose status is its own (hipGetLastError after a launch would
// also return, and clear, an error the caller had pending).  The arguments
// are the kernel's parameters by value, in order.
template <class... A>
static hipError_t launch_direct(const void* fn, dim3 grid, dim3 block, hipStream_t s, A... args) {
  void* argv[] = {static_cast<void*>(&args)...};
  return hipLaunchKernel(fn, grid, block, argv, 0, s);
}

hipError_t launch_fill_zero(double2* out, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  return launch_direct(reinterpret_cast<const void*>(&k_fill_zero), dim3((unsigned)((count + kBlock - 1) / kBlock)),
                       dim3(kBlock), s, out, count);
}

// out[i] += in[r * stride + i] for r = 0..rows-1 in order (FP64).
__global__ __launch_bounds__(kBlock) void k_accumulate_rows(double2* out, const double2* in, long long stride,
                                                           int rows, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  double2 acc = out[i];
  for (int r = 0; r < rows; ++r) {
    const double2 v = in[(long long)r * stride + i];
    acc.x += v.x;
    acc.y += v.y;
  }
  out[i] = acc;
}

hipError_t launch_accumulate_rows(double2* out, const double2* in, long long stride, int rows, long long count,
                                  hipStream_t s) {
  if (count <= 0 || rows <= 0) return hipSuccess;
  return launch_direct(reinterpret_cast<const void*>(&k_accumulate_rows),
                       dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), s, out, in, stride, rows, count);
}


// Batched sampling (Sec. 4.2, steps 3-4): one block per batch.  Thread t
// holds entries [t E, t E + E) of the batch's 2^k (E = 2^k / 256 or 1),
// their probabilities |Z|^2 in FP64 and their sum; a block scan of those
// sums gives every entry's inclusive prefix; the suffix is the smallest b
// whose prefix exceeds u Q_a (the last suffix if rounding leaves none).
__global__ __launch_bounds__(kBlock) void k_sample_batched(const double2* amps, int k, const double* u, int32_t* bout,
                                                           double* qout) {
  __shared__ double scan[kBlock];
  __shared__ int best;
  const long long batch = blockIdx.x;
  const int B = 1 << k;
  const int E = B > kBlock ? B / kBlock : 1;
  const int t = threadIdx.x;
  const int first = t * E;
  const double2* z = amps + batch * (long long)B;
  double p[kMaxSampleEntries];
  double local = 0.0;
#pragma unroll
  for (int e = 0; e < kMaxSampleEntries; ++e) {
    p[e] = 0.0;
    if (e < E && first + e < B) {
      const double2 v = z[first + e];
      p[e] = v.x * v.x + v.y * v.y;
      local += p[e];
    }
  }
  if (t == 0) best = B - 1;
  scan[t] = local;
  __syncthreads();
  // inclusive Hillis-Steele scan over the thread sums
  for (int off = 1; off < kBlock; off <<= 1) {
    const double add = t >= off ? scan[t - off] : 0.0;
    __syncthreads();
    scan[t] += add;
    __syncthreads();
  }
  const double q = scan[kBlock - 1];
  const double target = u[batch] * q;
  double run = scan[t] - local;  // exclusive prefix of this thread's entries
#pragma unroll
  for (int e = 0; e < kMaxSampleEntries; ++e) {
    if (e < E && first + e < B) {
      run += p[e];
      if (run > target) {
        atomicMin(&best, first + e);
        break;
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    bout[batch] = best;
    qout[batch] = q;
  }
}

// Frugal rejection (Sec. 4.1, steps 2-3): z = 2^n |amp|^2, accepted when
// u < min(1, z / M).
__global__ __launch_bounds__(kBlock) void k_frugal_accept(const double2* amps, long long count, int n, double M,
                                                          const double* u, uint8_t* accept, double* zout) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double2 v = amps[i];
  const double z = ldexp(v.x * v.x + v.y * v.y, n);
  zout[i] = z;
  accept[i] = u[i] < fmin(1.0, z / M) ? 1 : 0;
}

hipError_t launch_sample_batched(const double2* amps, int n_batches, int k, const double* u, int32_t* b, double* q,
                                 hipStream_t s) {
  if (n_batches <= 0) return hipSuccess;
  return launch_direct(reinterpret_cast<const void*>(&k_sample_batched), dim3((unsigned)n_batches), dim3(kBlock), s,
                       amps, k, u, b, q);
}

hipError_t launch_frugal_accept(const double2* amps, long long count, int n, double M, const double* u,
                                uint8_t* accept, double* z, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const long long blocks = (count + kBlock - 1) / kBlock;
  return launch_direct(reinterpret_cast<const void*>(&k_frugal_accept), dim3((unsigned)blocks), dim3(kBlock), s, amps,
                       count, n, M, u, accept, z);
}

// log-XEB (Sec. 5.2): F = gamma + n ln 2 + mean_i ln p_i with p_i = |amp|^2
// of the selected component of each batch (sel == nullptr: every component).
// One block, FP64 throughout.  result = {F, SE, F - 1.96 SE, F + 1.96 SE, N}.
__global__ __launch_bounds__(kBlock) void k_logxeb(const double2* amps, int n_batches, int k,
                                                   const int32_t* sel, int n_qubits, double* result) {
  __shared__ double s1[kBlock], s2[kBlock];
  const long long per = 1ll << k;
  const long long total = sel ? (long long)n_batches : (long long)n_batches * per;
  double a1 = 0.0, a2 = 0.0;
  for (long long i = threadIdx.x; i < total; i += blockDim.x) {
    const long long idx = sel ? (i * per + sel[i]) : i;
    const double2 z = amps[idx];
    const double lp = log(z.x * z.x + z.y * z.y);
    a1 += lp;
    a2 += lp * lp;
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s1[threadIdx.x] += s1[threadIdx.x + off];
      s2[threadIdx.x] += s2[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double N = (double)total;
    const double mean = s1[0] / N;
    const double var = N > 1 ? (s2[0] - N * mean * mean) / (N - 1.0) : 0.0;
    const double se = N > 1 ? sqrt(var > 0 ? var : 0.0) / sqrt(N) : 0.0;
    const double gamma = 0.57721566490153286060651209008240243;
    const double F = gamma + (double)n_qubits * 0.69314718055994530941723212145817657 + mean;
    result[0] = F;
    result[1] = se;
    result[2] = F - 1.96 * se;
    result[3] = F + 1.96 * se;
    result[4] = N;
  }
}

hipError_t launch_logxeb(const double2* amps, int n_batches, int k, const int32_t* sel, int n_qubits,
                         double* result, hipStream_t s) {
  return launch_direct(reinterpret_cast<const void*>(&k_logxeb), dim3(1), dim3(kBlock), s, amps, n_batches, k, sel,
                       n_qubits, result);
}

}  // namespace tnc
