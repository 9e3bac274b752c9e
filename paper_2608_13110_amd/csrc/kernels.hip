// HIP kernels for gfx950 (CDNA4) of the temporal-boundary contraction.
//
//  k_init   row-0 build-up of the boundary tensor (one write pass)
//  k_pass   one fused window of staircase updates over every tile of the
//           boundary tensor (the hot loop); in place, HBM-streaming
//  k_late   the folded late-phase contraction: the Alg. 2 join and the late
//           layers, FP64 accumulation
//  k_logxeb FP64 log-XEB reduction
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <vector>

#include "kernels.hpp"

namespace tnc {

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

__global__ __launch_bounds__(kBlock) void k_init(InitArgs a) {
  __shared__ double2 seg[4 * 64];
  const int nseg = a.m0 - 1;
  for (int i = threadIdx.x; i < 4 * nseg; i += blockDim.x) seg[i] = a.seg[i];
  __syncthreads();
  const int m = a.m0;
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
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

hipError_t launch_init(const InitArgs& a, hipStream_t s) {
  if (a.m0 - 1 > 64) return hipErrorInvalidValue;
  const long long threads = a.h < 11 ? ((long long)a.n_batches << a.h) : (((long long)a.n_batches << a.h) >> 5);
  const long long blocks = (threads + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_init, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
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

hipError_t launch_init16(const InitArgs& a, hipStream_t s) {
  if (a.m0 - 1 > 64 || a.blk_bits > 12 || a.blk_bits < 0 || a.blk_bits > a.h) return hipErrorInvalidValue;
  const long long blocks = (long long)a.n_batches << (a.h - a.blk_bits);
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  if (a.store == STORE_F16) hipLaunchKernelGGL(k_init16<STORE_F16>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  else if (a.store == STORE_BF16) hipLaunchKernelGGL(k_init16<STORE_BF16>, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Variant resolution: every op's matrix pair for each batch of the group,
// picked once from the batch's output bits, so the pass kernels read their
// matrices at addresses that depend on the op only.
__global__ __launch_bounds__(kBlock) void k_resolve(ResolveArgs a) {
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
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
  if (a.rmrows) {
    const float4* rs = a.mrows + ((size_t)op.mat * 4 + var) * 8;
    float4* rd = a.rmrows + (size_t)b * a.rmstride + (size_t)o * 8;
#pragma unroll
    for (int q = 0; q < 8; ++q) rd[q] = rs[q];
  }
}

hipError_t launch_resolve(const ResolveArgs& a, hipStream_t s) {
  const long long total = (long long)a.n_batches * a.n_ops;
  if (total <= 0) return hipSuccess;
  const long long blocks = (total + kBlock - 1) / kBlock;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_resolve, dim3((unsigned)blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// The pass kernel.  A tile is 2^T entries of one batch's boundary tensor: the
// global slots [0, lo_bits) and [win_lo, win_lo + win_len).  A block holds
// one tile (T - R >= 8 thread bits) or several small ones.  Data path:
//   HBM -> LDS with 16-byte accesses along the contiguous low slots,
//   per phase: LDS -> registers (2^R entries per thread, the phase's target
//   slots as register bits), the phase's updates in registers, registers ->
//   LDS,
//   LDS -> HBM, in place.
// WU: every wave lies inside one tile (one tile per block, or T - R >= 6),
// so the batch and everything read through it are wave-uniform.
// NT: threads per block (256; 512 for one 2^(R+9)-entry tile per block).
// Resident waves per SIMD the register allocation must allow: LDS admits
// five 2^12-entry (32 KiB) single-tile blocks per CU, so 16-entry phases in
// 256-thread blocks ask for five.
template <int R, bool MF, int NT>
constexpr int pass_waves_per_eu() {
  return MF ? 2 : (R == 4 && NT == 256 ? 5 : 1);
}

template <int R, bool MULTI, bool MF, bool WU, int NT = kBlock>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(pass_waves_per_eu<R, MF, NT>()))) void k_pass(
    PassArgs a) {
  extern __shared__ float2 lds[];
  constexpr int E = 1 << R;
  const int T = a.T;
  const int TB = T - R;
  const int tid = threadIdx.x;
  const int tile_in_block = MULTI ? (tid >> TB) : 0;
  const uint32_t tt = MULTI ? (uint32_t)(tid & ((1 << TB) - 1)) : (uint32_t)tid;
  const int tiles_per_block = MULTI ? (NT >> TB) : 1;
  // Blocks are dispatched round-robin over the 8 XCDs; each XCD takes a
  // contiguous range of tiles instead, so the blocks in flight on one XCD
  // read and write neighbouring runs (measured: 3.7 % more bandwidth on the
  // loads and stores alone, about 1 % per pass).
  const unsigned nb = gridDim.x;
  const unsigned lb = (nb & 7u) == 0u ? (blockIdx.x & 7u) * (nb >> 3) + (blockIdx.x >> 3) : blockIdx.x;
  const long long tile = (long long)lb * tiles_per_block + tile_in_block;
  const bool active = tile < a.n_tiles;
  const int tbits = a.h - T;
  long long batch = active ? (tile >> tbits) : 0;
  if constexpr (WU) batch = __builtin_amdgcn_readfirstlane((int)batch);
  const unsigned long long blk = active ? ((unsigned long long)tile & ((1ull << tbits) - 1ull)) : 0ull;
  float2* __restrict__ Bt = a.B + (batch << a.h) + block_offset(blk, a.lo_bits, a.win_lo, a.win_len);
  char* region = reinterpret_cast<char*>(lds) + ((size_t)tile_in_block << (T + 3));
  const int tpt = 1 << TB;

  if (active) {
#pragma unroll
    for (int it = 0; it < E / 2; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * 2u;
      const float4 val = *reinterpret_cast<const float4*>(Bt + tile_offset(i, a.lo_bits, a.win_lo));
      *reinterpret_cast<float4*>(region + ((size_t)swz(i) << 3)) = val;
    }
  }
  __syncthreads();

  const uint32_t tmask = (1u << T) - 1u;
  PhaseCtx<R, MF> ctx;
  ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
  ctx.rmr = a.rmrows ? a.rmrows + (size_t)batch * a.rmstride : nullptr;
  ctx.bits = a.bits;
  ctx.xpos = (size_t)batch * a.n;
  ctx.tb = 0;
  ctx.lane = tid & 63;
  ctx.uniform = WU;
  const uint32_t rbase = (uint32_t)tile_in_block << (T + 3);
  for (int p = 0; p < a.n_phases; ++p) {
    const DevPhase P = load_phase(a.phases, p);
    phase_dispatch<R, MF, WU && !MF>(reinterpret_cast<char*>(lds), rbase, P,
                                     (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx, tt, tmask,
                                     a.fmats + (size_t)p * kFusedWords, TB);
    __syncthreads();
  }

  if (active) {
#pragma unroll
    for (int it = 0; it < E / 2; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * 2u;
      const float4 val = *reinterpret_cast<const float4*>(region + ((size_t)swz(i) << 3));
      *reinterpret_cast<float4*>(Bt + tile_offset(i, a.lo_bits, a.win_lo)) = val;
    }
  }
}

// The pass kernel on 16-bit block-scaled storage: the same tiles and
// phases as k_pass, with the entries decoded (value = stored x block scale
// of the previous writer) on the way into LDS, and re-encoded on the way out
// with a fresh power-of-two scale per block of this pass's tiles (taken from
// the block's largest component after the pass).  4 entries (16 bytes) per
// HBM access, 2 when a thread holds only 2 entries.
template <int R, bool MULTI, int S, bool WU>
__global__ __launch_bounds__(kBlock) void k_pass16(PassArgs a) {
  extern __shared__ float2 lds[];
  constexpr int E = 1 << R;
  constexpr int U = E >= 4 ? 4 : 2;
  const int T = a.T;
  const int TB = T - R;
  const int tid = threadIdx.x;
  const int tile_in_block = MULTI ? (tid >> TB) : 0;
  const uint32_t tt = MULTI ? (uint32_t)(tid & ((1 << TB) - 1)) : (uint32_t)tid;
  const int tiles_per_block = MULTI ? (kBlock >> TB) : 1;
  const long long tile = (long long)blockIdx.x * tiles_per_block + tile_in_block;
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
  const bool two = T > blk_bits;
  if (tid < 2 * tiles_per_block) smax[tid] = 0u;

  // A scale slot gathers bit fields of the entry index, and the block part
  // (boff), the thread part (tt) and the iteration part (it) of an entry's
  // index occupy disjoint bits, so its slot is the OR of the three parts'
  // slots; the iteration part is the same for every thread (scalar work).
  const uint64_t slot_t = scale_slot(boff, a.in_map) |
                          scale_slot(tile_offset(tt * (uint32_t)U, a.lo_bits, a.win_lo), a.in_map);
  if (active) {
#pragma unroll
    for (int it = 0; it < E / U; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * (uint32_t)U;
      const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
      const uint64_t slot_i = scale_slot(tile_offset((uint32_t)(it * tpt) * (uint32_t)U, a.lo_bits, a.win_lo), a.in_map);
      const float sc = sin[slot_t | slot_i];
      if constexpr (U == 4) {
        const uint4 w = *reinterpret_cast<const uint4*>(Bw + g);
        const float2 e0 = unpack16<S>(w.x, sc), e1 = unpack16<S>(w.y, sc);
        const float2 e2 = unpack16<S>(w.z, sc), e3 = unpack16<S>(w.w, sc);
        *reinterpret_cast<float4*>(region + ((size_t)swz(i) << 3)) = make_float4(e0.x, e0.y, e1.x, e1.y);
        *reinterpret_cast<float4*>(region + ((size_t)swz(i + 2u) << 3)) = make_float4(e2.x, e2.y, e3.x, e3.y);
      } else {
        const uint2 w = *reinterpret_cast<const uint2*>(Bw + g);
        const float2 e0 = unpack16<S>(w.x, sc), e1 = unpack16<S>(w.y, sc);
        *reinterpret_cast<float4*>(region + ((size_t)swz(i) << 3)) = make_float4(e0.x, e0.y, e1.x, e1.y);
      }
    }
  }
  __syncthreads();

  const uint32_t tmask = (1u << T) - 1u;
  PhaseCtx<R, false> ctx;
  ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
  ctx.rmr = a.rmrows ? a.rmrows + (size_t)batch * a.rmstride : nullptr;
  ctx.bits = a.bits;
  ctx.xpos = (size_t)batch * a.n;
  ctx.tb = 0;
  ctx.lane = tid & 63;
  ctx.uniform = WU;
  for (int p = 0; p < a.n_phases; ++p) {
    const DevPhase P = load_phase(a.phases, p);
    phase_dispatch<R, false, WU>(reinterpret_cast<char*>(lds), (uint32_t)tile_in_block << (T + 3), P,
                                 (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx, tt, tmask,
                                 a.fmats + (size_t)p * kFusedWords, TB);
    __syncthreads();
  }

  // largest component of each block of the tile
  if (active) {
    float m0 = 0.f, m1 = 0.f;
#pragma unroll
    for (int it = 0; it < E / 2; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * 2u;
      const float4 v = *reinterpret_cast<const float4*>(region + ((size_t)swz(i) << 3));
      const float am = fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w)));
      if ((i >> blk_bits) & 1u) m1 = fmaxf(m1, am);
      else m0 = fmaxf(m0, am);
    }
    if (m0 > 0.f) atomicMax(&smax[2 * tile_in_block], __float_as_uint(m0));
    if (m1 > 0.f) atomicMax(&smax[2 * tile_in_block + 1], __float_as_uint(m1));
  }
  __syncthreads();
  if (active) {
    const int x0 = block_exponent(__uint_as_float(smax[2 * tile_in_block]));
    const int x1 = block_exponent(__uint_as_float(smax[2 * tile_in_block + 1]));
    const float inv0 = ldexpf(1.f, -x0), inv1 = ldexpf(1.f, -x1);
#pragma unroll
    for (int it = 0; it < E / U; ++it) {
      const uint32_t i = (uint32_t)(it * tpt + (int)tt) * (uint32_t)U;
      const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
      const float inv = ((i >> blk_bits) & 1u) ? inv1 : inv0;
      const float4 v0 = *reinterpret_cast<const float4*>(region + ((size_t)swz(i) << 3));
      if constexpr (U == 4) {
        const float4 v1 = *reinterpret_cast<const float4*>(region + ((size_t)swz(i + 2u) << 3));
        *reinterpret_cast<uint4*>(Bw + g) = make_uint4(pack16<S>(v0.x, v0.y, inv), pack16<S>(v0.z, v0.w, inv),
                                                       pack16<S>(v1.x, v1.y, inv), pack16<S>(v1.z, v1.w, inv));
      } else {
        *reinterpret_cast<uint2*>(Bw + g) = make_uint2(pack16<S>(v0.x, v0.y, inv), pack16<S>(v0.z, v0.w, inv));
      }
    }
    if (tt == 0) {
      float* sout = a.scale_out + batch * a.scale_stride + ((long long)blk << (T - blk_bits));
      sout[0] = ldexpf(1.f, x0);
      if (two) sout[1] = ldexpf(1.f, x1);
    }
  }
}

// Waits for outstanding vector-memory operations only (vmcnt <= n; gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at
// their maxima), and the LDS-only wait used before raw barriers.
#define TNC_WAIT_VMCNT0() __builtin_amdgcn_s_waitcnt(0x0F70)
// vmcnt <= n for n < 16 (vector-memory operations retire in issue order)
#define TNC_WAIT_VMCNT(n) __builtin_amdgcn_s_waitcnt(0x0F70 | ((n) & 15))
#define TNC_WAIT_LGKM0() __builtin_amdgcn_s_waitcnt(0xC07F)

// Workgroup barrier for LDS only: waits for this wave's LDS operations,
// not for vector-memory ones (a prefetch in flight stays in flight; the
// plain __syncthreads() would wait for it).  The empty asm statements keep
// the compiler from moving memory accesses across.
__device__ __attribute__((always_inline)) inline void tnc_lds_barrier() {
  asm volatile("" ::: "memory");
  TNC_WAIT_LGKM0();
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Persistent, software-pipelined form of the pass for one 2^T-entry tile
// per NT-thread block (T - R = 8 with 256 threads, 9 with 512): each block
// walks tiles blockIdx.x, blockIdx.x + gridDim.x, ...; the next tile's HBM
// loads are issued right after the current tile has been staged in LDS, so
// they are in flight while the current tile's register phases run (the
// phase barriers wait for LDS only).
template <int R, bool MF, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(2))) void k_pass_pipe(PassArgs a) {
  extern __shared__ float2 lds[];
  constexpr int E = 1 << R;
  constexpr int HALF = E / 2;
  const int T = a.T;
  const int tid = threadIdx.x;
  const uint32_t tt = (uint32_t)tid;
  const int tbits = a.h - T;
  char* region = reinterpret_cast<char*>(lds);
  const uint32_t tmask = (1u << T) - 1u;
  auto tile_base = [&](long long tile) -> float2* {
    const long long batch = tile >> tbits;
    const unsigned long long blk = (unsigned long long)tile & ((1ull << tbits) - 1ull);
    return a.B + (batch << a.h) + block_offset(blk, a.lo_bits, a.win_lo, a.win_len);
  };
  // prefetch buffer as plain floats (arrays of HIP vector types can be kept
  // out of registers)
  float p0[HALF], p1[HALF], p2[HALF], p3[HALF];
  auto prefetch = [&](long long t) {
    const float2* src = tile_base(t);
#pragma unroll
    for (int it = 0; it < HALF; ++it) {
      const uint32_t i = (uint32_t)(it * NT + tid) * 2u;
      const float4 q = *reinterpret_cast<const float4*>(src + tile_offset(i, a.lo_bits, a.win_lo));
      p0[it] = q.x;
      p1[it] = q.y;
      p2[it] = q.z;
      p3[it] = q.w;
    }
  };
  long long tile = blockIdx.x;
  if (tile < a.n_tiles) prefetch(tile);
  for (; tile < a.n_tiles; tile += gridDim.x) {
    const long long batch = tile >> tbits;
#pragma unroll
    for (int it = 0; it < HALF; ++it) {
      const uint32_t i = (uint32_t)(it * NT + tid) * 2u;
      *reinterpret_cast<float4*>(region + ((size_t)swz(i) << 3)) = make_float4(p0[it], p1[it], p2[it], p3[it]);
    }
    tnc_lds_barrier();
    const long long next = tile + gridDim.x;
    if (next < a.n_tiles) prefetch(next);
    PhaseCtx<R, MF> ctx;
    ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
    ctx.rmr = a.rmrows ? a.rmrows + (size_t)batch * a.rmstride : nullptr;
    ctx.bits = a.bits;
    ctx.xpos = (size_t)batch * a.n;
    ctx.tb = 0;
    ctx.lane = tid & 63;
    ctx.uniform = true;
    for (int p = 0; p < a.n_phases; ++p) {
      const DevPhase P = load_phase(a.phases, p);
      phase_dispatch<R, MF, !MF>(region, 0u, P, (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx, tt, tmask,
                                 a.fmats + (size_t)p * kFusedWords, T - R);
      tnc_lds_barrier();
    }
    float2* dst = tile_base(tile);
#pragma unroll
    for (int it = 0; it < HALF; ++it) {
      const uint32_t i = (uint32_t)(it * NT + tid) * 2u;
      const float4 val = *reinterpret_cast<const float4*>(region + ((size_t)swz(i) << 3));
      *reinterpret_cast<float4*>(dst + tile_offset(i, a.lo_bits, a.win_lo)) = val;
    }
    tnc_lds_barrier();
  }
}

typedef __attribute__((address_space(3))) void lds_void_t;

// Persistent pass with double-buffered LDS tiles: the next tile is fetched
// by direct global->LDS loads (global_load_lds_dwordx4, no VGPRs) while the
// current tile's register phases run.  Slot pair p of a buffer holds tile
// entries swz(p), swz(p)+1 (swz is an involution that keeps pairs), so the
// register phases use the same placement as the other pass kernels.  Phase
// barriers wait for LDS only, leaving the prefetch in flight.
// One block per CU (two 2^T-entry LDS tiles): 4 or 8 waves per CU.
template <int R, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT / 256, NT / 256))) void k_pass_dma(PassArgs a) {
  constexpr int E = 1 << R;
  constexpr int HALF = E / 2;
  constexpr int T = R + (NT == 512 ? 9 : 8);
  // two statically distinct buffers: the compiler can see that the phases
  // never read the buffer the DMA is writing, so it adds no memory waits
  __shared__ float2 ping[1 << T];
  __shared__ float2 pong[1 << T];
  const int tid = threadIdx.x;
  const uint32_t tt = (uint32_t)tid;
  const int tbits = a.h - T;
  constexpr uint32_t tmask = (1u << T) - 1u;
  const int wave = tid >> 6;
  auto tile_base = [&](long long tile) -> float2* {
    const long long batch = tile >> tbits;
    const unsigned long long blk = (unsigned long long)tile & ((1ull << tbits) - 1ull);
    return a.B + (batch << a.h) + block_offset(blk, a.lo_bits, a.win_lo, a.win_len);
  };
  auto fetch = [&](long long tile, float2* dst) {
    const float2* src = tile_base(tile);
#pragma unroll
    for (int it = 0; it < HALF; ++it) {
      const uint32_t p = (uint32_t)(it * NT + tid) * 2u;
      const float2* g = src + tile_offset(swz(p), a.lo_bits, a.win_lo);
      __builtin_amdgcn_global_load_lds(reinterpret_cast<const void*>(g),
                                       (lds_void_t*)(reinterpret_cast<char*>(dst) + ((size_t)(it * NT + wave * 64) << 4)),
                                       16, 0, 0);
    }
  };
  // one tile: wait for its prefetch, start the next tile's, run the phases,
  // store
  auto process = [&](long long tile, float2* cur, float2* nxt) {
    const long long batch = tile >> tbits;
    // this tile's prefetch was issued before the previous tile's HALF
    // stores, and vector-memory operations retire in issue order
    TNC_WAIT_VMCNT(HALF);
    TNC_WAIT_LGKM0();
    __builtin_amdgcn_s_barrier();
    const long long next = tile + gridDim.x;
    if (next < a.n_tiles) fetch(next, nxt);
    char* region = reinterpret_cast<char*>(cur);
    PhaseCtx<R, false> ctx;
    ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
    ctx.rmr = nullptr;
    ctx.bits = a.bits;
    ctx.xpos = (size_t)batch * a.n;
    ctx.tb = 0;
    ctx.lane = tid & 63;
    ctx.uniform = true;
    for (int p = 0; p < a.n_phases; ++p) {
      const DevPhase P = load_phase(a.phases, p);
      phase_dispatch<R, false>(region, 0u, P, (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx, tt, tmask);
      TNC_WAIT_LGKM0();
      __builtin_amdgcn_s_barrier();
    }
    float2* dst = tile_base(tile);
#pragma unroll
    for (int it = 0; it < HALF; ++it) {
      const uint32_t i = (uint32_t)(it * NT + tid) * 2u;
      const float4 val = *reinterpret_cast<const float4*>(region + ((size_t)swz(i) << 3));
      *reinterpret_cast<float4*>(dst + tile_offset(i, a.lo_bits, a.win_lo)) = val;
    }
  };
  long long tile = blockIdx.x;
  if (tile >= a.n_tiles) return;
  fetch(tile, ping);
  // the first tile has no stores queued behind its loads: wait for all
  TNC_WAIT_VMCNT0();
  for (;;) {
    process(tile, ping, pong);
    tile += gridDim.x;
    if (tile >= a.n_tiles) break;
    process(tile, pong, ping);
    tile += gridDim.x;
    if (tile >= a.n_tiles) break;
  }
}

static int pipe_blocks_per_cu(const void* fn, int nt, size_t lds) {
  int blocks = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, fn, nt, lds) != hipSuccess || blocks < 1) blocks = 1;
  return blocks;
}

static int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  }
  return cus;
}

template <int R, int NT>
static hipError_t launch_pass_dma(const PassArgs& a, hipStream_t s) {
  static int bpc = 0;
  if (bpc == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&bpc, reinterpret_cast<const void*>(&k_pass_dma<R, NT>), NT, 0) !=
            hipSuccess ||
        bpc < 1)
      bpc = 1;
  }
  const long long grid = std::min<long long>(a.n_tiles, (long long)bpc * device_cus());
  hipLaunchKernelGGL((k_pass_dma<R, NT>), dim3((unsigned)grid), dim3(NT), 0, s, a);
  return hipGetLastError();
}

template <int R, int S>
static hipError_t launch_pass16_rs(const PassArgs& a, hipStream_t s) {
  const int TB = a.T - R;
  if (TB < 0 || TB > 8) return hipErrorInvalidValue;
  const bool multi = TB < 8;
  const int tiles_per_block = multi ? (kBlock >> TB) : 1;
  const long long blocks = ((long long)a.n_tiles + tiles_per_block - 1) / tiles_per_block;
  const size_t lds = ((size_t)tiles_per_block << (a.T + 3)) + 2 * sizeof(uint32_t) * (size_t)kBlock;
  if (multi && TB >= 6) hipLaunchKernelGGL((k_pass16<R, true, S, true>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
  else if (multi) hipLaunchKernelGGL((k_pass16<R, true, S, false>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
  else hipLaunchKernelGGL((k_pass16<R, false, S, true>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

template <int R>
static hipError_t launch_pass_r(const PassArgs& a, hipStream_t s) {
  if (a.store == STORE_F16) return launch_pass16_rs<R, STORE_F16>(a, s);
  if (a.store == STORE_BF16) return launch_pass16_rs<R, STORE_BF16>(a, s);
  const int TB = a.T - R;
  const bool dma_ok = a.pipeline == 1 && !a.mfma;
  if constexpr (R >= 4) {
    if (dma_ok && TB == 8) return launch_pass_dma<R, 256>(a, s);
  }
  if constexpr (R == 4) {
    if (dma_ok && TB == 9) return launch_pass_dma<R, 512>(a, s);
  }
  if (TB == 9 && !a.mfma) {
    // one 2^(R+9)-entry tile per 512-thread block
    const size_t lds9 = (size_t)512 * (1 << R) * sizeof(float2);
    if (a.pipeline == 2) {
      static int bpc9[8] = {0};
      if (bpc9[R] == 0) bpc9[R] = pipe_blocks_per_cu(reinterpret_cast<const void*>(&k_pass_pipe<R, false, 512>), 512, lds9);
      const long long grid = std::min<long long>(a.n_tiles, (long long)bpc9[R] * device_cus());
      hipLaunchKernelGGL((k_pass_pipe<R, false, 512>), dim3((unsigned)grid), dim3(512), lds9, s, a);
      return hipGetLastError();
    }
    hipLaunchKernelGGL((k_pass<R, false, false, true, 512>), dim3((unsigned)a.n_tiles), dim3(512), lds9, s, a);
    return hipGetLastError();
  }
  if (TB < 0 || TB > 8) return hipErrorInvalidValue;
  const bool multi = TB < 8;
  const int tiles_per_block = multi ? (kBlock >> TB) : 1;
  const long long blocks = ((long long)a.n_tiles + tiles_per_block - 1) / tiles_per_block;
  const size_t lds = (size_t)kBlock * (1 << R) * sizeof(float2);
  // matrix-core updates need the four lanes of an MFMA block in one tile
  const bool mf = a.mfma && TB >= 2 && a.rmrows != nullptr;
  // persistent blocks with the next tile prefetched into registers
  // (pipeline = 2; the matrix-core form uses them for pipeline = 1 too)
  if (!multi && (a.pipeline == 2 || (a.pipeline && mf))) {
    const void* fn = mf ? reinterpret_cast<const void*>(&k_pass_pipe<R, true, kBlock>)
                        : reinterpret_cast<const void*>(&k_pass_pipe<R, false, kBlock>);
    static int per_cu[2][8] = {{0}};
    int& bpc = per_cu[mf ? 1 : 0][R];
    if (bpc == 0) bpc = pipe_blocks_per_cu(fn, kBlock, lds);
    const long long resident = (long long)bpc * device_cus();
    const long long grid = std::min<long long>(a.n_tiles, resident);
    if (mf) hipLaunchKernelGGL((k_pass_pipe<R, true, kBlock>), dim3((unsigned)grid), dim3(kBlock), lds, s, a);
    else hipLaunchKernelGGL((k_pass_pipe<R, false, kBlock>), dim3((unsigned)grid), dim3(kBlock), lds, s, a);
    return hipGetLastError();
  }
  if (multi) {
    if (mf) hipLaunchKernelGGL((k_pass<R, true, true, false>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    else if (TB >= 6) hipLaunchKernelGGL((k_pass<R, true, false, true>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    else hipLaunchKernelGGL((k_pass<R, true, false, false>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
  } else {
    if (mf) hipLaunchKernelGGL((k_pass<R, false, true, true>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
    else hipLaunchKernelGGL((k_pass<R, false, false, true>), dim3((unsigned)blocks), dim3(kBlock), lds, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_pass(const PassArgs& a, int R, hipStream_t s) {
  switch (R) {
    case 1: return launch_pass_r<1>(a, s);
    case 2: return launch_pass_r<2>(a, s);
    case 3: return launch_pass_r<3>(a, s);
    case 4: return launch_pass_r<4>(a, s);
    case 5: return launch_pass_r<5>(a, s);
    default: return hipErrorInvalidValue;
  }
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
    // the staircase tail, lane by lane
    for (int l = 0; l < 64; ++l) {
      Regs<R> v;
      for (int i = 0; i < E; ++i) {
        v.x[i] = vx[l][i];
        v.y[i] = vy[l][i];
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
  const uint32_t tmask = (1u << T) - 1u;
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
        float2* dst = reinterpret_cast<float2*>(region + ((size_t)swz(i) << 3));
        if (s16) {
          const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
          const float sc = a.scale_in[batch * a.scale_stride + (long long)scale_slot(g, a.in_map)];
          dst[0] = dec(Bw[g], sc);
          dst[1] = dec(Bw[g + 1], sc);
        } else {
          const float2* src = Bt + tile_offset(i, a.lo_bits, a.win_lo);
          dst[0] = src[0];
          dst[1] = src[1];
        }
      }
    PhaseCtx<R, false> ctx;
    ctx.rm = (const TNC_TBL float*)(a.rmats + (size_t)batch * a.rstride);
    ctx.rmr = a.rmrows ? a.rmrows + (size_t)batch * a.rmstride : nullptr;
    ctx.bits = a.bits;
    ctx.xpos = (size_t)batch * a.n;
    ctx.tb = 0;
    ctx.lane = 0;
    ctx.uniform = false;
    for (int p = 0; p < a.n_phases; ++p) {
      const DevPhase P = load_phase(a.phases, p);
      if (P.pad) {
        if constexpr (R >= 3)
          emulate_tri<R>(region, P, a.poffs + p * kPhaseOffs, a.fmats + (size_t)p * kFusedWords,
                         a.rmats + (size_t)batch * a.rstride, TB);
        continue;
      }
      for (int tt = 0; tt < tpt; ++tt)
        phase_dispatch<R, false>(region, 0u, P, (const TNC_TBL uint32_t*)a.poffs + p * kPhaseOffs, ctx, (uint32_t)tt, tmask);
    }
    if (s16) {
      float amax[2] = {0.f, 0.f};
      for (uint32_t i = 0; i < (1u << T); ++i) {
        const float2 v = lds[swz(i)];
        float& m = amax[(i >> blk_bits) & 1u];
        m = std::max(m, std::max(std::fabs(v.x), std::fabs(v.y)));
      }
      const int x0 = block_exponent(amax[0]), x1 = block_exponent(amax[1]);
      for (uint32_t i = 0; i < (1u << T); ++i) {
        const uint64_t g = boff + tile_offset(i, a.lo_bits, a.win_lo);
        Bw[g] = enc(lds[swz(i)], std::ldexp(1.f, -(((i >> blk_bits) & 1u) ? x1 : x0)));
      }
      float* sout = a.scale_out + batch * a.scale_stride + ((long long)blk << (T - blk_bits));
      sout[0] = std::ldexp(1.f, x0);
      if (T > blk_bits) sout[1] = std::ldexp(1.f, x1);
      continue;
    }
    for (int tt = 0; tt < tpt; ++tt)
      for (int it = 0; it < E / 2; ++it) {
        const uint32_t i = (uint32_t)(it * tpt + tt) * 2u;
        const float2* src = reinterpret_cast<const float2*>(region + ((size_t)swz(i) << 3));
        float2* dst = Bt + tile_offset(i, a.lo_bits, a.win_lo);
        dst[0] = src[0];
        dst[1] = src[1];
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
__global__ __launch_bounds__(kBlock) void k_late(LateArgs a) {
  __shared__ double2 As[16][65];
  __shared__ double2 Bs[16][65];
  const int b = blockIdx.y;
  const int tilesN = (a.N + 63) / 64;
  const int tilesM = (a.M + 63) / 64;
  // Consecutive block ids go to different XCDs (round robin over 8); the
  // tilesN column blocks of one row tile are given ids that land on the
  // same XCD, so they share its L2 for the row tile.
  const int xcd = blockIdx.x & 7;
  const int g = blockIdx.x >> 3;
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

// The same contraction on the FP64 matrix cores (v_mfma_f64_16x16x4f64):
// a 64 x 64 output tile per 256-thread block, 32 x 32 (2 x 2 MFMA tiles)
// per wave; the complex product takes four real MFMAs per tile and k-step
// (re += ar*br - ai*bi, im += ar*bi + ai*br).  Lane l supplies A[l%16][k]
// and B[k][l%16] with k = l/16 and receives D[l/16 + 4q][l%16], q < 4.
typedef double tnc_d4 __attribute__((ext_vector_type(4)));

template <typename TIn, int S>
__global__ __launch_bounds__(kBlock) void k_late_mf(LateArgs a) {
  __shared__ double2 As[16][65];
  __shared__ double2 Bs[16][65];
  const int b = blockIdx.y;
  const int tilesN = (a.N + 63) / 64;
  const int tilesM = (a.M + 63) / 64;
  const int xcd = blockIdx.x & 7;
  const int g = blockIdx.x >> 3;
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

hipError_t launch_late(const LateArgs& a, bool in_c64, hipStream_t s) {
  const long long tilesM8 = ((long long)(a.M + 63) / 64 + 7) / 8 * 8;
  const long long tiles = tilesM8 * ((a.N + 63) / 64);
  if (tiles > 0x7fffffffLL || a.n_batches > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)tiles, (unsigned)a.n_batches);
  // matrix cores for contractions large enough to fill their 16 x 16 tiles
  if (in_c64 && a.N >= 32 && a.K >= 16 && a.M >= 64) {
    if (a.store == STORE_F16) hipLaunchKernelGGL((k_late_mf<uint32_t, STORE_F16>), grid, dim3(kBlock), 0, s, a);
    else if (a.store == STORE_BF16) hipLaunchKernelGGL((k_late_mf<uint32_t, STORE_BF16>), grid, dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((k_late_mf<float2, STORE_C64>), grid, dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
  if (!in_c64) hipLaunchKernelGGL((k_late<double2, STORE_C64>), grid, dim3(kBlock), 0, s, a);
  else if (a.store == STORE_F16) hipLaunchKernelGGL((k_late<uint32_t, STORE_F16>), grid, dim3(kBlock), 0, s, a);
  else if (a.store == STORE_BF16) hipLaunchKernelGGL((k_late<uint32_t, STORE_BF16>), grid, dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((k_late<float2, STORE_C64>), grid, dim3(kBlock), 0, s, a);
  return hipGetLastError();
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

__global__ __launch_bounds__(kBlock) void k_late_ops(LateOpsArgs a) {
  extern __shared__ double2 st[];
  const long long row_out = blockIdx.x;
  const int b = blockIdx.y;
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
      const int items = (1 << (live - 1)) << (sb - 1);
      for (int w = threadIdx.x; w < items; w += blockDim.x) {
        const int ra = (w >> (sb - 1)) << (l + 1);
        const int rb = ra | (1 << l);
        const int t0 = (w & ((1 << (sb - 1)) - 1)) << 1;
        const int ia = (ra << sb) | t0, ib = (rb << sb) | t0;
        const double2 x0 = st[ia], x1 = st[ia | 1], y0 = st[ib], y1 = st[ib | 1];
        const double2 o0a = zfma2(op.m[0], x0, op.m[1], x1), o0b = zfma2(op.m[4], y0, op.m[5], y1);
        const double2 o1a = zfma2(op.m[2], x0, op.m[3], x1), o1b = zfma2(op.m[6], y0, op.m[7], y1);
        st[ia] = make_double2(o0a.x + o0b.x, o0a.y + o0b.y);
        st[ia | 1] = make_double2(o1a.x + o1b.x, o1a.y + o1b.y);
      }
      ++l;
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

hipError_t launch_late_ops(const LateOpsArgs& a, hipStream_t s) {
  if (a.s + a.j > 12 || a.rows_out > 0x7fffffffLL || a.n_batches > 65535) return hipErrorInvalidValue;
  const size_t lds = sizeof(double2) << (a.s + a.j);
  hipLaunchKernelGGL(k_late_ops, dim3((unsigned)a.rows_out, (unsigned)a.n_batches), dim3(kBlock), lds, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// log-XEB (Sec. 5.2): F = gamma + n ln 2 + mean_i ln p_i with p_i = |amp|^2
// of the selected component of each batch (sel == nullptr: every component).
// One block, FP64 throughout.  result = {F, SE, F - 1.96 SE, F + 1.96 SE, N}.
// FP64 complex fill and sum (the ring's sum over slices).
__global__ __launch_bounds__(kBlock) void k_fill_zero(double2* out, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = make_double2(0.0, 0.0);
}

__global__ __launch_bounds__(kBlock) void k_accumulate(double2* out, const double2* in, long long count) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) {
    const double2 a = out[i], b = in[i];
    out[i] = make_double2(a.x + b.x, a.y + b.y);
  }
}

hipError_t launch_fill_zero(double2* out, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, out, count);
  return hipGetLastError();
}

hipError_t launch_accumulate(double2* out, const double2* in, long long count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_accumulate, dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, out, in,
                     count);
  return hipGetLastError();
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
  hipLaunchKernelGGL(k_sample_batched, dim3((unsigned)n_batches), dim3(kBlock), 0, s, amps, k, u, b, q);
  return hipGetLastError();
}

hipError_t launch_frugal_accept(const double2* amps, long long count, int n, double M, const double* u,
                                uint8_t* accept, double* z, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  const long long blocks = (count + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_frugal_accept, dim3((unsigned)blocks), dim3(kBlock), 0, s, amps, count, n, M, u, accept, z);
  return hipGetLastError();
}

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
  hipLaunchKernelGGL(k_logxeb, dim3(1), dim3(kBlock), 0, s, amps, n_batches, k, sel, n_qubits, result);
  return hipGetLastError();
}

}  // namespace tnc
