// XCD-aware block numbering.  The 256 CUs of the chip sit in 8 XCDs with an
// L2 each, and workgroups are handed out round-robin over the XCDs, so
// consecutive block ids never share an L2.  Renumbering the blocks so that
// XCD k runs one contiguous eighth of the grid puts neighbouring blocks
// (which share cache lines: overlapping tile windows and window slabs)
// in the same L2.
#pragma once
#include <hip/hip_runtime.h>

namespace pm {

constexpr unsigned kXcds = 8;

// block id lid of total (dispatch order) -> the id whose work it does
__device__ __forceinline__ unsigned xcd_block(unsigned lid, unsigned total) {
  if (total % kXcds) return lid;
  return (lid % kXcds) * (total / kXcds) + lid / kXcds;
}

// pairs of neighbouring blocks on one XCD at about the same time, the grid
// order otherwise kept: within every 16 dispatch ids, XCD k runs blocks 2k and
// 2k + 1 (dispatched 8 ids apart)
__device__ __forceinline__ unsigned xcd_pair(unsigned lid, unsigned total) {
  if (total % (2 * kXcds)) return lid;
  const unsigned g = lid / (2 * kXcds), r = lid % (2 * kXcds);
  return g * (2 * kXcds) + (r % kXcds) * 2 + r / kXcds;
}

}  // namespace pm
