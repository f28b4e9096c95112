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

}  // namespace pm
