// LDS placement of a pass tile, and the table of dense phase forms, shared
// by the kernels (kernels.hpp) and the host planner (plan.cpp), which places
// each phase's lane bits and cuts each dense phase by them.
#pragma once

#include <cstdint>

#if defined(__HIPCC__)
#define TNC_LDS_HD __host__ __device__ __attribute__((always_inline))
#else
#define TNC_LDS_HD
#endif

namespace tnc {

// Tile entry i (8 bytes) sits in LDS slot swz(i).  A bank cycle of an
// 8-byte access serves the slots of 16 (or 32) lanes; lanes whose slots are
// equal modulo 16 (32) conflict.  swz adds to each tile bit p >= 4 a mask of
// lower slot bits (bits 0..4), so that each slot direction has several
// sources: direction q < 4 comes from tile bit q, from tile bit q + 6 (with
// direction 4 added) and from one of the tile bits 4, 11..13; direction 4
// from tile bits 5 and 10 (and, with direction 3, tile bit 4).  The planner
// puts the low lane bits of a register phase on tile bits whose directions
// are independent (lane_slot_dir), choosing among the sources of each
// direction around the bits the phase holds in registers.  Every tile bit
// only adds lower bits, so the map is linear over GF(2), unitriangular
// (invertible), keeps [0, 2^T), and keeps swz(1) = 1: the entry pair
// (2j, 2j + 1) shares one aligned 16-byte slot, in either order
// (pair_swapped).
TNC_LDS_HD inline uint32_t swz(uint32_t i) {
  // slot-bit masks of tile bits 4..13
  constexpr uint32_t kMask[10] = {8u, 16u, 17u, 18u, 20u, 24u, 16u, 1u, 2u, 12u};
  uint32_t m = 0;
#pragma unroll
  for (int b = 0; b < 10; ++b) m ^= (0u - ((i >> (4 + b)) & 1u)) & kMask[b];
  return i ^ m;
}

// Slot bits 0..4 of tile bit p alone: the bank direction a lane bit placed
// on tile bit p moves its lane's slot in.
TNC_LDS_HD inline uint32_t lane_slot_dir(int p) { return swz(1u << p) & 31u; }

// For the entry pair (i, i + 1), i even, with s = swz(i): the byte offset of
// its aligned 16-byte slot, and whether entry i + 1 is the first of the two.
// (swz is linear: for disjoint bit sets, swz(a | b) = swz(a) ^ swz(b).)
TNC_LDS_HD inline uint32_t pair_slot(uint32_t s) { return (s & ~1u) << 3; }
TNC_LDS_HD inline bool pair_swapped(uint32_t s) { return (s & 1u) != 0u; }

// Register-bit pairs (A, B), A < B < 5, numbered in lexicographic order:
// the codes of a dense phase's updates.
TNC_LDS_HD constexpr int dense_pair_code(int a, int b) {
  return a == 0 ? b - 1 : a == 1 ? 2 + b : a == 2 ? 4 + b : 9;
}

// The dense phase forms: G updates whose codes (4 bits each, update 0 in the
// low bits) are one of the register-bit patterns the planner produces, each
// compiled as straight-line code: a wavefront step of two rows is (0,1)
// (1,2), then (3,4) (0,4); a row alone is (0,1) (2,3).  The planner cuts a
// phase to its longest prefix that has a form.
TNC_LDS_HD constexpr bool dense_form_exists(int R, int G, uint32_t codes) {
  return (G == 1 && codes == 0x0u && R >= 2) || (G == 2 && codes == 0x40u && R >= 3) ||
         (G == 2 && codes == 0x70u && R >= 4) || (G == 3 && codes == 0x940u && R >= 5) ||
         (G == 4 && codes == 0x3940u && R >= 5);
}

}  // namespace tnc
