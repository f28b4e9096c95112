// Tile windows: the mesh is cut into (n/T)^3 tiles of T^3 cells; the window
// of a tile covers the tile plus R cells beyond each face (W = T + 2R per
// axis, z fastest) and lives in a slab [slot][tile][W^3] of int64 partial
// sums.  A cell's value is the sum of the windows that cover it: along each
// axis the own tile at local l + R, the previous tile at l + T + R when
// l < R, the next one at l - T + R when l >= T - R (indices periodic).
#pragma once
#include <hip/hip_runtime.h>

namespace pm {

struct WinCover {
  int t[3], l[3], n;  // covering tiles and local coordinates along one axis
};

__device__ __forceinline__ WinCover win_cover(int x, int T, int R, int log2T, int ntm) {
  WinCover w;
  const int tc = x >> log2T, l = x & (T - 1);
  int k = 0;
  w.t[k] = tc; w.l[k] = l + R; ++k;
  if (l < R) { w.t[k] = (tc - 1) & ntm; w.l[k] = l + T + R; ++k; }
  if (l >= T - R) { w.t[k] = (tc + 1) & ntm; w.l[k] = l - T + R; ++k; }
  w.n = k;
  return w;
}

// sum of the windows covering the cell whose x and y covers are cx, cy
__device__ __forceinline__ long long win_sum(const long long* __restrict__ slab, const WinCover& cx,
                                             const WinCover& cy, const WinCover& cz, int W, int log2nt) {
  const long long W3 = (long long)W * W * W;
  long long acc = 0;
  for (int p = 0; p < cx.n; ++p)
    for (int q = 0; q < cy.n; ++q)
      for (int r = 0; r < cz.n; ++r) {
        const long long t = ((long long)cx.t[p] << (2 * log2nt)) | (cy.t[q] << log2nt) | cz.t[r];
        acc += slab[t * W3 + ((long long)cx.l[p] * W + cy.l[q]) * W + cz.l[r]];
      }
  return acc;
}

// the same cover when T > 2R: the own tile and at most one neighbour, in
// scalars (no dynamically indexed arrays, so nothing spills to scratch)
struct Cover2 {
  int t0, l0, t1, l1;
  bool two;
};

__device__ __forceinline__ Cover2 cover2(int x, int T, int R, int log2T, int ntm) {
  Cover2 c;
  const int tc = x >> log2T, l = x & (T - 1);
  c.t0 = tc;
  c.l0 = l + R;
  c.two = l < R || l >= T - R;
  c.t1 = (l < R ? tc - 1 : tc + 1) & ntm;
  c.l1 = l < R ? l + T + R : l - T + R;
  return c;
}

}  // namespace pm
