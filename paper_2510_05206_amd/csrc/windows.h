// Tile windows: the mesh is cut into (n/T)^3 tiles of T^3 cells (nt per
// axis); the window of a tile covers the tile plus Rlo cells below and Rhi
// cells above each axis (W = T + Rlo + Rhi) and holds int64 partial sums.
// The halo is asymmetric where the stencil is: a width-6 kernel anchored at
// floor(u) reaches 2 nodes below and 3 above.  In the slab of one slot the
// windows are stored row-major over the mesh: the window row (lx, ly) of
// tile (tx, ty, tz) is W values at
//   ((((tx nt + ty) W + lx) W + ly) nt + tz) W,
// so the rows of all tz at fixed (tx, ty, lx, ly) are one contiguous run of
// nt W values.  A cell's value is the sum of the windows that cover it:
// along each axis the own tile at local l + Rlo, the previous tile at
// l + T + Rlo when l < Rhi, the next one at l - T + Rlo when l >= T - Rlo
// (indices periodic).
#pragma once
#include <hip/hip_runtime.h>

namespace pm {

struct WinCover {
  int t[3], l[3], n;  // covering tiles and local coordinates along one axis
};

__device__ __forceinline__ WinCover win_cover(int x, int T, int Rlo, int Rhi, int log2T, int ntm) {
  WinCover w;
  const int tc = x >> log2T, l = x & (T - 1);
  int k = 0;
  w.t[k] = tc; w.l[k] = l + Rlo; ++k;
  if (l < Rhi) { w.t[k] = (tc - 1) & ntm; w.l[k] = l + T + Rlo; ++k; }
  if (l >= T - Rlo) { w.t[k] = (tc + 1) & ntm; w.l[k] = l - T + Rlo; ++k; }
  w.n = k;
  return w;
}

// offset of window row (lx, ly) of tile (tx, ty, tz) in a slot's slab
__device__ __forceinline__ long long slab_row(int tx, int ty, int tz, int lx, int ly, int W, int nt) {
  return (((((long long)tx * nt + ty) * W + lx) * W + ly) * nt + tz) * W;
}

// sum of the windows covering a cell with covers cx, cy, cz
template <class V>
__device__ __forceinline__ V win_sum(const V* __restrict__ slab, const WinCover& cx, const WinCover& cy,
                                     const WinCover& cz, int W, int nt) {
  V acc = 0;
  for (int p = 0; p < cx.n; ++p)
    for (int q = 0; q < cy.n; ++q)
      for (int r = 0; r < cz.n; ++r) acc += slab[slab_row(cx.t[p], cy.t[q], cz.t[r], cx.l[p], cy.l[q], W, nt) + cz.l[r]];
  return acc;
}

// store an LDS window (z fastest, W <= 32) of tile t into the slot's slab:
// the block's groups of 32 lanes take rows r = lx W + ly in turn, one lane
// per z.  slab_row(tx, ty, tz, lx, ly) = slab_row(tx, ty, tz, 0, 0) +
// r nt W, so the addresses advance by a constant (no division by W per row)
template <class V>
__device__ __forceinline__ void store_window(const V* win, V* slab, int t, int W, int log2nt) {
  const int nt = 1 << log2nt, m = nt - 1;
  const int tx = t >> (2 * log2nt), ty = (t >> log2nt) & m, tz = t & m;
  const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5, W2 = W * W, ng = blockDim.x >> 5;
  if (lane >= W) return;
  const long long ntW = (long long)nt * W;
  long long o = slab_row(tx, ty, tz, 0, 0, W, nt) + grp * ntW + lane;
  for (int r = grp; r < W2; r += ng, o += ng * ntW) slab[o] = win[r * W + lane];
}

// the same with the int64 window converted to FP32 partial sums (value
// times scale) on the way out
__device__ __forceinline__ void store_window_f32(const unsigned long long* win, float* slab, int t, int W, int log2nt,
                                                 double scale) {
  const int nt = 1 << log2nt, m = nt - 1;
  const int tx = t >> (2 * log2nt), ty = (t >> log2nt) & m, tz = t & m;
  const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5, W2 = W * W, ng = blockDim.x >> 5;
  if (lane >= W) return;
  const long long ntW = (long long)nt * W;
  long long o = slab_row(tx, ty, tz, 0, 0, W, nt) + grp * ntW + lane;
  for (int r = grp; r < W2; r += ng, o += ng * ntW) slab[o] = (float)((double)(long long)win[r * W + lane] * scale);
}

// the same cover when Rlo + Rhi <= T: the own tile and at most one
// neighbour, in scalars (no dynamically indexed arrays, so nothing spills)
struct Cover2 {
  int t0, l0, t1, l1;
  bool two;
};

__device__ __forceinline__ Cover2 cover2(int x, int T, int Rlo, int Rhi, int log2T, int ntm) {
  Cover2 c;
  const int tc = x >> log2T, l = x & (T - 1);
  c.t0 = tc;
  c.l0 = l + Rlo;
  c.two = l < Rhi || l >= T - Rlo;
  c.t1 = (l < Rhi ? tc - 1 : tc + 1) & ntm;
  c.l1 = l < Rhi ? l + T + Rlo : l - T + Rlo;
  return c;
}

}  // namespace pm
