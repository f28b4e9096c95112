// Tile-binned particle <-> mesh kernels (no global atomics on the mesh).
//
// Once per force evaluation the particles are counting-sorted by the
// 16^3-cell tile that holds their home node (k_bin_count / k_bin_scan /
// k_bin_scatter).  Each later kernel runs one workgroup per tile over that
// tile's particles:
//   k_tile_deposit   accumulates the fixed-point CIC/TSC mass in an int64 LDS
//                    window (tile + 1 cell each side) and writes the whole
//                    window to a scratch slab;
//   k_assemble_run   sums, for every cell, the window values of the (up to 8)
//                    tiles whose window covers it (int64: order-free; the FP32
//                    partial sums of the ES force chains in a fixed order),
//                    one z-run of cells per block (k_assemble: small meshes);
//   k_tile_kick      stages the potential over the tile + stencil reach in LDS
//                    and does the FD-gradient gather, kick and drift;
//   k_tile_adj_kick  the same gather with the position gradient for the
//                    adjoint kick, writing u = beta V_bar in sorted order;
//   k_tile_dipole    scatters u through the transposed gather (kernel x FD
//                    stencil) into an int64 LDS window, in fixed point with a
//                    scale set by max|u| (deterministic);
//   k_tile_adj_drift gradient gather of the mesh cotangent and reverse drifts;
//   k_tile_es_*      the same roles with the width-6 ES kernel of the NUFFT
//                    force (deposit, kick, adjoint kick, gradient spread,
//                    adjoint drift), further down.
// The windows make each HBM access coalesced and each particle's stencil an
// LDS access; the mesh is written once per pass.
#include <type_traits>

#include "mak.h"
#include "windows.h"
#include "xcd.h"

namespace pm {

constexpr int kTileMax = 16;
// threads per workgroup of the PM transposed gather: its int64 LDS window
// (85 KB at FD4) allows one workgroup per CU, so more threads per workgroup
// means more waves per CU
constexpr int kPmDipoleThreads = 1024;
constexpr int kPmDepositThreads = 256;

struct TileGeo {
  int T, log2T, log2nt, n_tiles;
  long long ts;  // ints per slot of count/offset
};

__device__ __forceinline__ void tile_origin(int t, const TileGeo& tg, int o[3]) {
  const int m = (1 << tg.log2nt) - 1;
  o[2] = (t & m) << tg.log2T;
  o[1] = ((t >> tg.log2nt) & m) << tg.log2T;
  o[0] = (t >> (2 * tg.log2nt)) << tg.log2T;
}

// ------------------------------------------------------------- binning

// The kick V' = alpha V + beta A and the drift X' = X + tau V with one fixed
// rounding in every kernel and path: whether a b + c d is contracted into a
// fused multiply-add, and which product it keeps, depends on the code around
// it, and the forward ES kick takes a particle through one of two paths by
// its rank in the tile list (which the binning's atomics set), so an implicit
// contraction would make runs differ in the last bit.
__device__ __forceinline__ float kick_v(float al, float v, float be, float A) { return fmaf(be, A, al * v); }
__device__ __forceinline__ float drift_x(float x, float tp, float v) { return fmaf(tp, v, x); }

template <int P>
__global__ void __launch_bounds__(256) k_bin_count(BinArgs a) {
  const int slot = blockIdx.y;
  if (!slot_on(a.g.gate, a.active, slot)) return;
  const long long N = a.g.N;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const bool valid = i < N;
  const long long ps = slot * a.g.part_stride;
  int tile = -1;
  if (valid) {
    float p[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
    if (a.vel) {  // merged first drift X += tau V, written back (every load before the stores)
      const float t = slot_f(a.g.gate, a.g.sched, a.g.sched_steps, a.tau, slot, kSchTau1);
      float v[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) v[c] = a.vel[ps + c * N + i];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        p[c] = drift_x(p[c], t, v[c]);
        a.disp[ps + c * N + i] = p[c];
      }
    }
    long long j[3];
    lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
    const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
    const int nm = a.g.n_g - 1;
    int h[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      h[c] = (home_node<P>((fixed_coord(j[c], p[c], a.g.log2_r, umask) + a.g.ushift) & umask, nm) - a.home_shift) & nm;
    tile = (((h[0] >> a.log2T) << a.log2nt | (h[1] >> a.log2T)) << a.log2nt) | (h[2] >> a.log2T);
  }
  // wave-aggregated counting: one atomic per distinct tile in the wave
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(valid);
  int rank = 0;
  while (pending) {
    const int leader = __builtin_ctzll(pending);
    const int lt = __shfl(tile, leader);
    const unsigned long long m = __ballot(valid && tile == lt) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd(a.count + slot * a.ts + lt, (int)__popcll(m));
    base = __shfl(base, leader);
    if ((m >> lane) & 1ull) rank = base + (int)__popcll(m & ((1ull << lane) - 1ull));
    pending &= ~m;
  }
  if (valid) {
    a.key[slot * N + i] = tile;
    a.rank[slot * N + i] = rank;
  }
}

// exclusive scan of the tile counts in three short passes: each 1024-tile
// block scans its counts and records its total, one block per slot scans the
// totals (writing the grand total after the last tile), then every block adds
// its base
__device__ __forceinline__ int block_scan_1024(int v, int* wsum, int& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int w = lane < 16 ? wsum[lane] : 0;
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
      const int y = __shfl_up(w, o, 64);
      if (lane >= o) w += y;
    }
    if (lane < 16) wsum[lane] = w;  // inclusive over waves
  }
  __syncthreads();
  total = wsum[15];
  return x - v + (wave ? wsum[wave - 1] : 0);  // exclusive
}

__global__ void __launch_bounds__(1024) k_bin_scan_blocks(const int32_t* count, int32_t* offset, int32_t* partial,
                                                          int n_tiles, long long ts, int np) {
  __shared__ int wsum[16];
  const int slot = blockIdx.y, b = blockIdx.x;
  const int i = b * 1024 + threadIdx.x;
  const int v = i < n_tiles ? count[slot * ts + i] : 0;
  int total;
  const int ex = block_scan_1024(v, wsum, total);
  if (i < n_tiles) offset[slot * ts + i] = ex;
  if (threadIdx.x == 0) partial[slot * np + b] = total;
}

__global__ void __launch_bounds__(1024) k_bin_scan_partials(int32_t* partial, int32_t* offset, int n_tiles,
                                                            long long ts, int nb, int np) {
  __shared__ int wsum[16];
  const int slot = blockIdx.x;
  int run = 0;
  for (int b0 = 0; b0 < nb; b0 += 1024) {  // nb <= np partials, 1024 at a time
    const int b = b0 + threadIdx.x;
    const int v = b < nb ? partial[slot * np + b] : 0;
    int total;
    const int ex = block_scan_1024(v, wsum, total);
    __syncthreads();  // wsum is reused by the next round
    if (b < nb) partial[slot * np + b] = run + ex;
    run += total;
  }
  if (threadIdx.x == 0) offset[slot * ts + n_tiles] = run;
}

__global__ void __launch_bounds__(1024) k_bin_scan_add(const int32_t* partial, int32_t* offset, int n_tiles,
                                                       long long ts, int np) {
  const int slot = blockIdx.y, b = blockIdx.x;
  const int i = b * 1024 + threadIdx.x;
  if (b > 0 && i < n_tiles) offset[slot * ts + i] += partial[slot * np + b];
}

__global__ void __launch_bounds__(256) k_bin_scatter(BinArgs a) {
  const int slot = blockIdx.y;
  if (!slot_on(a.g.gate, a.active, slot)) return;
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= a.g.N) return;
  const long long N = a.g.N;
  const int t = a.key[slot * N + i];
  a.sorted[slot * N + a.offset[slot * a.ts + t] + a.rank[slot * N + i]] = (int32_t)i;
}

// ------------------------------------------------------------- deposit

template <int P>
__global__ void __launch_bounds__(kPmDepositThreads) k_tile_deposit(TileArgs a) {
  constexpr int NT = kPmDepositThreads, KR = kernel_reach<P>();
  __shared__ unsigned long long win[(kTileMax + 2 * KR) * (kTileMax + 2 * KR) * (kTileMax + 2 * KR)];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!slot_on(a.g.gate, a.active, slot)) return;
  const int T = a.T, W = T + 2 * KR, W3 = W * W * W;
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  // the first particle's loads are in flight while the window is cleared;
  // later ones are fetched while the current one scatters
  int p = beg + threadIdx.x;
  long long i = 0;
  float x[3] = {0.f, 0.f, 0.f};
  if (p < end) {
    i = a.sorted[slot * N + p];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[c] = a.disp[ps + c * N + i];
  }
  for (int e = threadIdx.x; e < W3; e += NT) win[e] = 0ull;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  __syncthreads();
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  constexpr int shift = 3 * kWeightBits - kMassBits;
  for (; p < end; p += NT) {
    long long j[3];
    lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
    int w[3][P], l0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      long long U = (fixed_coord(j[c], x[c], a.g.log2_r, umask) + a.g.ushift) & umask;
      weights1d<P>(U, w[c]);
      // local index of the first stencil node in the window (home at h - o + 1)
      l0[c] = home_node<P>(U, nm) - o[c] + KR + first_node<P>();
    }
    if (p + NT < end) {
      i = a.sorted[slot * N + p + NT];
#pragma unroll
      for (int c = 0; c < 3; ++c) x[c] = a.disp[ps + c * N + i];
    }
    // node masses once; the remainder to 2^32 goes to the largest weight
    unsigned long long v[P * P * P], sum = 0, best = 0;
    int home = 0;
#pragma unroll
    for (int xx = 0; xx < P; ++xx)
#pragma unroll
      for (int y = 0; y < P; ++y) {
        unsigned long long wxy = (unsigned long long)w[0][xx] * (unsigned)w[1][y];
#pragma unroll
        for (int z = 0; z < P; ++z) {
          const int k = (xx * P + y) * P + z;
          unsigned long long q = wxy * (unsigned)w[2][z];
          v[k] = rne_shift(q, shift);
          sum += v[k];
          if (q > best) { best = q; home = k; }
        }
      }
    const unsigned long long rem = (1ull << kMassBits) - sum;
#pragma unroll
    for (int xx = 0; xx < P; ++xx)
#pragma unroll
      for (int y = 0; y < P; ++y) {
        const int bxy = ((l0[0] + xx) * W + l0[1] + y) * W + l0[2];
#pragma unroll
        for (int z = 0; z < P; ++z) {
          const int k = (xx * P + y) * P + z;
          atomicAdd(&win[bxy + z], v[k] + (k == home ? rem : 0ull));
        }
      }
  }
  __syncthreads();
  store_window(win, reinterpret_cast<unsigned long long*>(a.scratch) + (long long)slot * a.n_tiles * W3, t, W,
               a.log2nt);
}

// sum of the windows covering one cell (windows.h), in a fixed order
template <class V>
__device__ __forceinline__ V assemble_cell(const AssembleArgs& a, const V* __restrict__ slab, int x, int y, int z) {
  const int T = a.T, Rlo = a.Rlo, Rhi = a.Rhi, W = T + Rlo + Rhi;
  const int ntm = (1 << a.log2nt) - 1;
  return win_sum(slab, win_cover(x, T, Rlo, Rhi, a.log2T, ntm), win_cover(y, T, Rlo, Rhi, a.log2T, ntm),
                 win_cover(z, T, Rlo, Rhi, a.log2T, ntm), W, 1 << a.log2nt);
}

// z-runs of one block (n >= 256): the x and y covers are block-uniform, so
// the window-row bases are scalar and each thread only adds its z offsets.
// NX x NY covering rows (a block-uniform case); every load of the thread's
// CPT cells is issued before the sums: the second z cover is read for every
// cell (clamped to the first where the cell has one) and masked
// arithmetically, since a load under a per-lane branch is waited for inside
// it, which serialises a thread's loads.  The sums run in the order of
// win_sum (rows by x cover, then y cover; z covers in order).
__device__ __forceinline__ float keep_if(float v, bool k) { return v * (k ? 1.f : 0.f); }
__device__ __forceinline__ long long keep_if(long long v, bool k) { return v & -(long long)k; }

template <int NX, int NY, int CPT, class V>
__device__ __forceinline__ void assemble_runs(const AssembleArgs& a, const V* __restrict__ slab, const Cover2& cx,
                                              const Cover2& cy, long long e0, V (&acc)[CPT]) {
  const int T = a.T, Rlo = a.Rlo, Rhi = a.Rhi, W = T + Rlo + Rhi;
  const int nt = 1 << a.log2nt, ntm = nt - 1, nm = a.g.n_g - 1;
  constexpr int NR = NX * NY;
  const V* row[NR];
#pragma unroll
  for (int p = 0; p < NX; ++p)
#pragma unroll
    for (int q = 0; q < NY; ++q)
      row[p * NY + q] =
          slab + slab_row(p ? cx.t1 : cx.t0, q ? cy.t1 : cy.t0, 0, p ? cx.l1 : cx.l0, q ? cy.l1 : cy.l0, W, nt);
  V v0[CPT][NR], v1[CPT][NR];
  bool two[CPT];
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    const Cover2 cz = cover2((int)((e0 + threadIdx.x + 256 * k) & nm), T, Rlo, Rhi, a.log2T, ntm);
    // offsets within a row run of nt W values
    const int oz0 = cz.t0 * W + cz.l0, oz1 = cz.two ? cz.t1 * W + cz.l1 : oz0;
    two[k] = cz.two;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      v0[k][r] = row[r][oz0];
      v1[k][r] = row[r][oz1];
    }
  }
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    acc[k] = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      acc[k] += v0[k][r];
      acc[k] += keep_if(v1[k][r], two[k]);
    }
  }
}

template <bool OUT_F32>
__device__ __forceinline__ auto assemble_out(const AssembleArgs& a, int slot, long long acc) {
  if constexpr (OUT_F32)
    return (float)(a.inv_scale ? (double)acc * a.inv_scale[slot] : (double)acc * a.scale - a.shift);
  else
    return acc;
}

// One cell per thread, any mesh and halo, in a fixed order.  OUT_F32
// converts the int64 sums with inv_scale (or scale and shift); with an FP32
// slab the partial sums add in FP32 and the shift follows.
template <bool OUT_F32>
__global__ void __launch_bounds__(256) k_assemble(AssembleArgs a) {
  const int slot = blockIdx.y;
  if (!slot_on(a.g.gate, a.active, slot)) return;
  const int L = a.g.log2_ng, nm = a.g.n_g - 1;
  const long long e = (long long)xcd_block(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (e >= a.g.M) return;
  const int W = a.T + a.Rlo + a.Rhi;
  const long long sl = (long long)slot * a.n_tiles * W * W * W;
  const int x = (int)(e >> (2 * L)), y = (int)((e >> L) & nm), z = (int)(e & nm);
  using V = typename std::conditional<OUT_F32, float, long long>::type;
  V out;
  if constexpr (OUT_F32) {
    if (a.slab_f32)
      out = assemble_cell(a, reinterpret_cast<const float*>(a.scratch) + sl, x, y, z) - (float)a.shift;
    else
      out = assemble_out<true>(a, slot, assemble_cell(a, reinterpret_cast<const long long*>(a.scratch) + sl, x, y, z));
  } else {
    out = assemble_cell(a, reinterpret_cast<const long long*>(a.scratch) + sl, x, y, z);
  }
  reinterpret_cast<V*>(a.out)[slot * a.g.mesh_stride + e] = out;
}

// z-runs: with n >= 256 CPT and Rlo + Rhi <= T a block of 256 threads sums
// 256 CPT consecutive cells of one (x, y) row (scalar x and y covers), CPT
// per thread, every load issued before the sums.  SLAB_F32: the windows are
// FP32 partial sums (out = sum - shift).
template <bool OUT_F32, bool SLAB_F32, int CPT>
__global__ void __launch_bounds__(256) k_assemble_run(AssembleArgs a) {
  const int slot = blockIdx.y;
  if (!slot_on(a.g.gate, a.active, slot)) return;
  const int L = a.g.log2_ng, nm = a.g.n_g - 1;
  const long long e0 = (long long)xcd_block(blockIdx.x, gridDim.x) * (256 * CPT);
  const int W = a.T + a.Rlo + a.Rhi;
  const long long sl = (long long)slot * a.n_tiles * W * W * W;
  const int x = (int)(e0 >> (2 * L)), y = (int)((e0 >> L) & nm);
  using S = typename std::conditional<SLAB_F32, float, long long>::type;
  using V = typename std::conditional<OUT_F32, float, long long>::type;
  const S* slab = reinterpret_cast<const S*>(a.scratch) + sl;
  const int ntm = (1 << a.log2nt) - 1;
  const Cover2 cx = cover2(x, a.T, a.Rlo, a.Rhi, a.log2T, ntm), cy = cover2(y, a.T, a.Rlo, a.Rhi, a.log2T, ntm);
  S acc[CPT];
  if (cx.two) {
    if (cy.two) assemble_runs<2, 2>(a, slab, cx, cy, e0, acc);
    else assemble_runs<2, 1>(a, slab, cx, cy, e0, acc);
  } else {
    if (cy.two) assemble_runs<1, 2>(a, slab, cx, cy, e0, acc);
    else assemble_runs<1, 1>(a, slab, cx, cy, e0, acc);
  }
  V* o = reinterpret_cast<V*>(a.out) + slot * a.g.mesh_stride + e0 + threadIdx.x;
#pragma unroll
  for (int k = 0; k < CPT; ++k) {
    if constexpr (SLAB_F32)
      o[256 * k] = acc[k] - (float)a.shift;
    else
      o[256 * k] = assemble_out<OUT_F32>(a, slot, acc[k]);
  }
}

// ----------------------------------------------------- windowed gathers

// stage mesh values over the tile + Rlo cells below / Rhi above into LDS
// Rows of W <= 32 consecutive z values: 8 groups of 32 lanes take rows
// (lx, ly) in turn, each lane one z; 8 rows per group are loaded before any
// is stored, so every thread keeps 8 HBM reads in flight.
__device__ __forceinline__ void load_window(float* win, const float* mesh, const int o[3], int T, int Rlo,
                                            int Rhi, int L, int nm) {
  constexpr int U = 8;
  const int W = T + Rlo + Rhi, W2 = W * W;
  const int lane = threadIdx.x & 31, grp = threadIdx.x >> 5;
  const bool zok = lane < W;
  const unsigned gz = (unsigned)((o[2] - Rlo + lane) & nm);
  // rows r = lx W + ly step by 8 (one carry when W > 8), no division per
  // row; a mesh of at most 1024^3 cells indexes in 32 bits
  int lx = grp / W, ly = grp - lx * W;
  for (int r0 = grp; r0 < W2; r0 += 8 * U) {
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + 8 * u;
      v[u] = 0.f;
      if (zok && r < W2) {
        const unsigned gx = (unsigned)((o[0] - Rlo + lx) & nm), gy = (unsigned)((o[1] - Rlo + ly) & nm);
        v[u] = mesh[((gx << L | gy) << L) | gz];
      }
      ly += 8;
      while (ly >= W) {
        ly -= W;
        ++lx;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = r0 + 8 * u;
      if (zok && r < W2) win[r * W + lane] = v[u];
    }
  }
}

struct WinAcc {
  const float* w;
  int W;
  __device__ float operator()(int x, int y, int z) const { return w[(x * W + y) * W + z]; }
};

// kernel weights (float) and the window-local first node of each axis
template <int P>
__device__ __forceinline__ void tile_weights(const TileArgs& a, long long i, const float p[3], const int o[3],
                                             int R, float w[3][P], float dw[3][P], int l0[3]) {
  long long j[3];
  lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    long long U = (fixed_coord(j[c], p[c], a.g.log2_r, umask) + a.g.ushift) & umask;
    weights1d_f<P>(U, w[c], dw[c]);
    l0[c] = home_node<P>(U, nm) - o[c] + R + first_node<P>();
  }
}

// forward: A = gather(FD phi); V = alpha V + beta A; X += tau V (or A only)
template <int P, int ORD>
__global__ void __launch_bounds__(256) k_tile_kick(TileArgs a) {
  constexpr int R = kernel_reach<P>() + ORD / 2;
  __shared__ float win[(kTileMax + 2 * R) * (kTileMax + 2 * R) * (kTileMax + 2 * R)];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!slot_on(a.g.gate, a.active, slot)) return;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  load_window(win, a.mesh_in + slot * a.g.mesh_stride, o, a.T, R, R, a.g.log2_ng, a.g.n_g - 1);
  __syncthreads();
  const WinAcc acc{win, a.T + 2 * R};
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const float al = slot_f(a.g.gate, a.g.sched, a.g.sched_steps, a.alpha, slot, kSchAlpha);
  const float be = slot_f(a.g.gate, a.g.sched, a.g.sched_steps, a.beta, slot, kSchBeta);
  const float tp = slot_f(a.g.gate, a.g.sched, a.g.sched_steps, a.tau, slot, kSchTau2);
  for (int p = beg + threadIdx.x; p < end; p += 256) {
    const long long i = a.sorted[slot * N + p];
    float x[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
    float w[3][P], dw[3][P], A[3], dA[3][3];
    int l0[3];
    tile_weights<P>(a, i, x, o, R, w, dw, l0);
    fd_gather<P, ORD, false>(acc, l0, w, dw, A, dA);
    if (a.acc_in) {  // interlaced grids: the mean of the two gathers
#pragma unroll
      for (int c = 0; c < 3; ++c) A[c] = 0.5f * (A[c] + a.acc_in[ps + c * N + i]);
    }
    if (a.acc_out) {
#pragma unroll
      for (int c = 0; c < 3; ++c) a.acc_out[ps + c * N + i] = A[c];
      continue;
    }
    float v[3];  // every load before the stores, which the compiler cannot order past them
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = a.vel[ps + c * N + i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = kick_v(al, v[c], be, A[c]);
      a.vel[ps + c * N + i] = v[c];
      a.disp[ps + c * N + i] = drift_x(x[c], tp, v[c]);
    }
  }
}

// adjoint kick at X^{n-1/2}: V^{n-1} = (V^n - beta A)/alpha; X_bar += r sum_c
// u_c dA_c/du (u = beta V_bar); V_bar *= alpha; u stored in sorted order and
// max|u| reduced per slot (fixed-point scale of the scatter)
template <int P, int ORD>
__global__ void __launch_bounds__(256, 2) k_tile_adj_kick(TileArgs a) {  // <= 256 VGPRs (two workgroups per CU)
  constexpr int R = kernel_reach<P>() + ORD / 2;
  __shared__ float win[(kTileMax + 2 * R) * (kTileMax + 2 * R) * (kTileMax + 2 * R)];
  __shared__ float red[256];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  load_window(win, a.mesh_in + slot * a.g.mesh_stride, o, a.T, R, R, a.g.log2_ng, a.g.n_g - 1);
  __syncthreads();
  const WinAcc acc{win, a.T + 2 * R};
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const float al = a.alpha[slot], be = a.beta[slot];
  const float r = (float)(1 << a.g.log2_r);
  float umax = 0.f;
  for (int p = beg + threadIdx.x; p < end; p += 256) {
    const long long i = a.sorted[slot * N + p];
    float x[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
    float w[3][P], dw[3][P], A[3], dA[3][3];
    int l0[3];
    tile_weights<P>(a, i, x, o, R, w, dw, l0);
    fd_gather<P, ORD, true>(acc, l0, w, dw, A, dA);
    float vb[3], u[3], tx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vb[c] = a.vbar[ps + c * N + i];
      u[c] = be * vb[c];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) tx[d] = r * (u[0] * dA[0][d] + u[1] * dA[1][d] + u[2] * dA[2][d]);
    if (a.il_in) {  // interlaced grids: the mean of the two grids' force and direct term
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        A[c] = 0.5f * (A[c] + a.il_in[2 * ps + c * N + i]);
        tx[c] = 0.5f * (tx[c] + a.il_in[2 * ps + (3 + c) * N + i]);
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.u_sorted[ps + c * N + p] = u[c];
      umax = fmaxf(umax, fabsf(u[c]));
    }
    if (a.il_out) {  // the second grid: its terms only, the state untouched
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a.il_out[2 * ps + c * N + i] = A[c];
        a.il_out[2 * ps + (3 + c) * N + i] = tx[c];
      }
      continue;
    }
    float v[3], xb[3];  // every load before the stores
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = a.vel[ps + c * N + i];
      xb[c] = a.xbar[ps + c * N + i];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.vel[ps + c * N + i] = (v[c] - be * A[c]) / al;
      a.vbar[ps + c * N + i] = al * vb[c];
      a.xbar[ps + c * N + i] = xb[c] + tx[c];
    }
  }
  red[threadIdx.x] = umax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.f)
    atomicMax(reinterpret_cast<unsigned int*>(a.umax) + slot, __float_as_uint(red[0]));
}

// fixed-point scale of the cotangent scatter: every node sum is bounded by
// N max|u| sum|c_s| (times 3 components), kept below 2^61; with
// node_per_u > 0 every single node value (< node_per_u max|u|) is also kept
// below 2^31
__global__ void k_dipole_scale(const unsigned int* umax_bits, double* scale, double* inv_scale, double bound_per_u,
                               double node_per_u, int batch) {
  const int s = threadIdx.x;
  if (s >= batch) return;
  const double um = (double)__uint_as_float(umax_bits[s]);
  const double m = um * bound_per_u;
  int k = m > 0.0 ? 61 - (ilogb(m) + 1) : 200;
  if (node_per_u > 0.0) {  // FP32 scaling on the device: a finite float power of two
    if (um > 0.0) k = min(k, 31 - (ilogb(um * node_per_u) + 1));
    k = min(k, 120);
  }
  if (k > 200) k = 200;
  scale[s] = ldexp(1.0, k);
  inv_scale[s] = ldexp(1.0, -k);
}

// transposed FD gather (mesh cotangent of the force), into an int64 window
// covering the tile + R cells: phi_bar(node) += u_c G_c[t] w w, each node
// value rounded to an int32 at the slot's fixed-point scale (|value| <=
// max|u| sum|c_s| < 2^31 there)
template <int P, int ORD>
__global__ void __launch_bounds__(kPmDipoleThreads) k_tile_dipole(TileArgs a) {
  constexpr int NT = kPmDipoleThreads;
  constexpr int H = ORD / 2, R = kernel_reach<P>() + H, Q = P + 2 * H;
  extern __shared__ unsigned long long dwin[];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  const int W = a.T + 2 * R, W3 = W * W * W;
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  // the first particle's loads are in flight while the window is cleared;
  // later ones are fetched while the current one scatters
  int p = beg + (int)(((threadIdx.x % (NT / 16)) * 16) + threadIdx.x / (NT / 16));  // lanes 16 apart in the tile list
  long long i = 0;
  float x[3] = {0.f, 0.f, 0.f}, u[3] = {0.f, 0.f, 0.f};
  if (p < end) {
    i = a.sorted[slot * N + p];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = a.disp[ps + c * N + i];
      u[c] = a.u_sorted[ps + c * N + p];
    }
  }
  for (int e = threadIdx.x; e < W3; e += NT) dwin[e] = 0ull;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  __syncthreads();
  // fixed point: every node value is below 2^31 at this scale (a power of two)
  const float S = (float)a.scale[slot];
  for (; p < end; p += NT) {
    float w[3][P], dw[3][P];
    int l0[3];
    tile_weights<P>(a, i, x, o, R, w, dw, l0);
    const float us[3] = {u[0] * S, u[1] * S, u[2] * S};
    if (p + NT < end) {
      const int q = p + NT;
      i = a.sorted[slot * N + q];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        x[c] = a.disp[ps + c * N + i];
        u[c] = a.u_sorted[ps + c * N + q];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float G[Q];
#pragma unroll
      for (int tt = 0; tt < Q; ++tt) {
        float g = 0.f;
#pragma unroll
        for (int q = 0; q < P; ++q) {
          int s = tt - H - q;
          if (s >= -H && s <= H) g += w[c][q] * fd_coef<ORD>(s);
        }
        G[tt] = g * us[c];
      }
      const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
#pragma unroll
      for (int tt = 0; tt < Q; ++tt) {
        if (G[tt] == 0.f) continue;
#pragma unroll
        for (int q1 = 0; q1 < P; ++q1)
#pragma unroll
          for (int q2 = 0; q2 < P; ++q2) {
            int n3[3];
            n3[c] = l0[c] - H + tt;
            n3[a1] = l0[a1] + q1;
            n3[a2] = l0[a2] + q2;
            const int v = (int)rintf(G[tt] * w[a1][q1] * w[a2][q2]);
            atomicAdd(&dwin[(n3[0] * W + n3[1]) * W + n3[2]], (unsigned long long)(long long)v);
          }
      }
    }
  }
  __syncthreads();
  store_window(dwin, reinterpret_cast<unsigned long long*>(a.scratch) + (long long)slot * a.n_tiles * W3, t, W,
               a.log2nt);
}

// scatter-w.r.t.-positions: X_bar += coef r sum_j rho_bar_j dW_j/du, then the
// reverse drift X -= tau V, V_bar += tau X_bar
template <int P>
__global__ void __launch_bounds__(256) k_tile_adj_drift(TileArgs a) {
  constexpr int R = kernel_reach<P>();
  __shared__ float win[(kTileMax + 2 * R) * (kTileMax + 2 * R) * (kTileMax + 2 * R)];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  load_window(win, a.mesh_in + slot * a.g.mesh_stride, o, a.T, R, R, a.g.log2_ng, a.g.n_g - 1);
  __syncthreads();
  const int W = a.T + 2 * R;
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const float cf = a.coef[slot] * (float)(1 << a.g.log2_r), tau = a.tau[slot];
  for (int p = beg + threadIdx.x; p < end; p += 256) {
    const long long i = a.sorted[slot * N + p];
    float x[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
    float w[3][P], dw[3][P];
    int l0[3];
    tile_weights<P>(a, i, x, o, R, w, dw, l0);
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int xx = 0; xx < P; ++xx)
#pragma unroll
      for (int yy = 0; yy < P; ++yy) {
        const int b = ((l0[0] + xx) * W + l0[1] + yy) * W + l0[2];
#pragma unroll
        for (int zz = 0; zz < P; ++zz) {
          float f = win[b + zz];
          gx += f * dw[0][xx] * w[1][yy] * w[2][zz];
          gy += f * w[0][xx] * dw[1][yy] * w[2][zz];
          gz += f * w[0][xx] * w[1][yy] * dw[2][zz];
        }
      }
    float g[3] = {cf * gx, cf * gy, cf * gz};
    if (a.il_in) {  // interlaced grids: the mean of the two grids' scatter terms
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = 0.5f * (g[c] + a.il_in[2 * ps + c * N + i]);
    }
    if (a.il_out) {  // the first grid: its term only, the state untouched
#pragma unroll
      for (int c = 0; c < 3; ++c) a.il_out[2 * ps + c * N + i] = g[c];
      continue;
    }
    float xb[3], v[3], vb[3];  // every load before the stores
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xb[c] = a.xbar[ps + c * N + i] + g[c];
      v[c] = a.vel[ps + c * N + i];
      vb[c] = a.vbar[ps + c * N + i];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.disp[ps + c * N + i] = x[c] - tau * v[c];
      a.xbar[ps + c * N + i] = xb[c];
      a.vbar[ps + c * N + i] = vb[c] + tau * xb[c];
    }
  }
}

// ------------------------------------------- forward-mode tangents (PM)

// JVP of the deposit w.r.t. the positions (a scatter with the gradient
// kernel dotted with the tangent positions, held in xbar): node +=
// coef sum_c xdot_c dW/du_c, coef = r n_g^3 / N (the contrast's
// normalisation and dq -> mesh units), in int64 fixed point at the slot's
// scale (every node value of one particle is below 3 coef max|xdot| < 2^31
// there, as |W| <= 1 and |dW/du| <= 1 per cell for CIC, TSC and PCS)
template <int P>
__global__ void __launch_bounds__(256) k_tile_tan_spread(TileArgs a) {
  constexpr int R = kernel_reach<P>();
  __shared__ unsigned long long win[(kTileMax + 2 * R) * (kTileMax + 2 * R) * (kTileMax + 2 * R)];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  const int W = a.T + 2 * R, W3 = W * W * W;
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  for (int e = threadIdx.x; e < W3; e += 256) win[e] = 0ull;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  __syncthreads();
  const float S = (float)a.scale[slot] * a.coef[slot];
  for (int p = beg + threadIdx.x; p < end; p += 256) {
    const long long i = a.sorted[slot * N + p];
    const float x[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
    float w[3][P], dw[3][P];
    int l0[3];
    tile_weights<P>(a, i, x, o, R, w, dw, l0);
    const float td[3] = {a.xbar[ps + i] * S, a.xbar[ps + N + i] * S, a.xbar[ps + 2 * N + i] * S};
#pragma unroll
    for (int xx = 0; xx < P; ++xx)
#pragma unroll
      for (int yy = 0; yy < P; ++yy) {
        const float cx = td[0] * dw[0][xx] * w[1][yy], cy = td[1] * w[0][xx] * dw[1][yy],
                    cz = td[2] * w[0][xx] * w[1][yy];
        unsigned long long* row = win + ((l0[0] + xx) * W + l0[1] + yy) * W + l0[2];
#pragma unroll
        for (int zz = 0; zz < P; ++zz) {
          const float v = (cx + cy) * w[2][zz] + cz * dw[2][zz];
          atomicAdd(row + zz, (unsigned long long)(long long)(int)rintf(v));
        }
      }
  }
  __syncthreads();
  store_window(win, reinterpret_cast<unsigned long long*>(a.scratch) + (long long)slot * a.n_tiles * W3, t, W,
               a.log2nt);
}

// direct part of J_A xdot (the gather's JVP w.r.t. the positions, phi
// fixed): r sum_d dA_c/du_d xdot_d into acc_out
template <int P, int ORD>
__global__ void __launch_bounds__(256, 2) k_tile_tan_direct(TileArgs a) {
  constexpr int R = kernel_reach<P>() + ORD / 2;
  __shared__ float win[(kTileMax + 2 * R) * (kTileMax + 2 * R) * (kTileMax + 2 * R)];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  load_window(win, a.mesh_in + slot * a.g.mesh_stride, o, a.T, R, R, a.g.log2_ng, a.g.n_g - 1);
  __syncthreads();
  const WinAcc acc{win, a.T + 2 * R};
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const float r = (float)(1 << a.g.log2_r);
  for (int p = beg + threadIdx.x; p < end; p += 256) {
    const long long i = a.sorted[slot * N + p];
    const float x[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
    float w[3][P], dw[3][P], A[3], dA[3][3];
    int l0[3];
    tile_weights<P>(a, i, x, o, R, w, dw, l0);
    fd_gather<P, ORD, true>(acc, l0, w, dw, A, dA);
    const float td[3] = {a.xbar[ps + i], a.xbar[ps + N + i], a.xbar[ps + 2 * N + i]};
#pragma unroll
    for (int c = 0; c < 3; ++c)
      a.acc_out[ps + c * N + i] = r * (dA[c][0] * td[0] + dA[c][1] * td[1] + dA[c][2] * td[2]);
  }
}

// the tangent kick and drift: J = gather(FD grad of the tangent potential)
// + the direct part (acc_in); Vdot = alpha Vdot + beta J, Xdot += tau Vdot
// (Xdot in xbar, Vdot in vbar)
template <int P, int ORD>
__global__ void __launch_bounds__(256) k_tile_tan_kick(TileArgs a) {
  constexpr int R = kernel_reach<P>() + ORD / 2;
  __shared__ float win[(kTileMax + 2 * R) * (kTileMax + 2 * R) * (kTileMax + 2 * R)];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  load_window(win, a.mesh_in + slot * a.g.mesh_stride, o, a.T, R, R, a.g.log2_ng, a.g.n_g - 1);
  __syncthreads();
  const WinAcc acc{win, a.T + 2 * R};
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const float al = a.alpha[slot], be = a.beta[slot], tp = a.tau[slot];
  for (int p = beg + threadIdx.x; p < end; p += 256) {
    const long long i = a.sorted[slot * N + p];
    const float x[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
    float w[3][P], dw[3][P], A[3], dA[3][3];
    int l0[3];
    tile_weights<P>(a, i, x, o, R, w, dw, l0);
    fd_gather<P, ORD, false>(acc, l0, w, dw, A, dA);
    float J[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) J[c] = A[c] + a.acc_in[ps + c * N + i];
    if (a.il_in) {  // interlaced grids: the mean with the other grid's J ([B][3][N])
#pragma unroll
      for (int c = 0; c < 3; ++c) J[c] = 0.5f * (J[c] + a.il_in[ps + c * N + i]);
    }
    if (a.il_out) {  // interlaced grids: this grid's J only, the state untouched
#pragma unroll
      for (int c = 0; c < 3; ++c) a.il_out[ps + c * N + i] = J[c];
      continue;
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float v = kick_v(al, a.vbar[ps + c * N + i], be, J[c]);
      a.vbar[ps + c * N + i] = v;
      a.xbar[ps + c * N + i] = drift_x(a.xbar[ps + c * N + i], tp, v);
    }
  }
}

// ------------------------------------------------------------- launchers

hipError_t launch_binning(const BinArgs& a, int mak, hipStream_t s) {
  dim3 grid((unsigned)((a.g.N + 255) / 256), a.batch);
  if (mak == 2) k_bin_count<2><<<grid, 256, 0, s>>>(a);
  else if (mak == 3) k_bin_count<3><<<grid, 256, 0, s>>>(a);
  else k_bin_count<4><<<grid, 256, 0, s>>>(a);
  const int nb = (a.n_tiles + 1023) / 1024;
  if (nb > a.scan_np) return hipErrorInvalidValue;
  k_bin_scan_blocks<<<dim3((unsigned)nb, a.batch), 1024, 0, s>>>(a.count, a.offset, a.scan_partial, a.n_tiles, a.ts,
                                                                 a.scan_np);
  k_bin_scan_partials<<<a.batch, 1024, 0, s>>>(a.scan_partial, a.offset, a.n_tiles, a.ts, nb, a.scan_np);
  k_bin_scan_add<<<dim3((unsigned)nb, a.batch), 1024, 0, s>>>(a.scan_partial, a.offset, a.n_tiles, a.ts, a.scan_np);
  k_bin_scatter<<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_tile(const TileArgs& a, int kind, int mak, int ord, hipStream_t s) {
  dim3 grid((unsigned)a.n_tiles, a.batch);
#define PM_TILE_ORD(KER, P)                                                   \
  do {                                                                        \
    if (ord == 2) KER<P, 2><<<grid, 256, 0, s>>>(a);                          \
    else if (ord == 4) KER<P, 4><<<grid, 256, 0, s>>>(a);                     \
    else KER<P, 6><<<grid, 256, 0, s>>>(a);                                   \
  } while (0)
  // PCS windows with the order-6 stencil would exceed a workgroup's static
  // LDS: PCS runs with FD2 / FD4 (the context refuses FD6)
#define PM_TILE_ORD4(KER)                                                     \
  do {                                                                        \
    if (ord == 2) KER<4, 2><<<grid, 256, 0, s>>>(a);                          \
    else if (ord == 4) KER<4, 4><<<grid, 256, 0, s>>>(a);                     \
    else return hipErrorInvalidValue;                                         \
  } while (0)
  switch (kind) {
    case TK_DEPOSIT:
      if (mak == 2) k_tile_deposit<2><<<grid, kPmDepositThreads, 0, s>>>(a);
      else if (mak == 3) k_tile_deposit<3><<<grid, kPmDepositThreads, 0, s>>>(a);
      else k_tile_deposit<4><<<grid, kPmDepositThreads, 0, s>>>(a);
      break;
    case TK_KICK:
      if (mak == 2) PM_TILE_ORD(k_tile_kick, 2); else if (mak == 3) PM_TILE_ORD(k_tile_kick, 3);
      else PM_TILE_ORD4(k_tile_kick);
      break;
    case TK_ADJ_KICK:
      if (mak == 2) PM_TILE_ORD(k_tile_adj_kick, 2); else if (mak == 3) PM_TILE_ORD(k_tile_adj_kick, 3);
      else PM_TILE_ORD4(k_tile_adj_kick);
      break;
    case TK_TAN_SPREAD:
      if (mak == 2) k_tile_tan_spread<2><<<grid, 256, 0, s>>>(a);
      else if (mak == 3) k_tile_tan_spread<3><<<grid, 256, 0, s>>>(a);
      else k_tile_tan_spread<4><<<grid, 256, 0, s>>>(a);
      break;
    case TK_TAN_DIRECT:
      if (mak == 2) PM_TILE_ORD(k_tile_tan_direct, 2); else if (mak == 3) PM_TILE_ORD(k_tile_tan_direct, 3);
      else PM_TILE_ORD4(k_tile_tan_direct);
      break;
    case TK_TAN_KICK:
      if (mak == 2) PM_TILE_ORD(k_tile_tan_kick, 2); else if (mak == 3) PM_TILE_ORD(k_tile_tan_kick, 3);
      else PM_TILE_ORD4(k_tile_tan_kick);
      break;
    case TK_ADJ_DRIFT:
      if (mak == 2) k_tile_adj_drift<2><<<grid, 256, 0, s>>>(a);
      else if (mak == 3) k_tile_adj_drift<3><<<grid, 256, 0, s>>>(a);
      else k_tile_adj_drift<4><<<grid, 256, 0, s>>>(a);
      break;
    case TK_DIPOLE: {
      int R = (mak == 4 ? 2 : 1) + ord / 2, W = a.T + 2 * R;
      size_t lds = (size_t)W * W * W * sizeof(unsigned long long);
      // ORD 6 (and PCS with ORD 4) needs 110 KB of LDS: above the default
      // dynamic limit (raised once by configure_tile_kernels)
#define PM_DIPOLE(P, O) k_tile_dipole<P, O><<<grid, kPmDipoleThreads, lds, s>>>(a)
      if (mak == 2) {
        if (ord == 2) PM_DIPOLE(2, 2); else if (ord == 4) PM_DIPOLE(2, 4); else PM_DIPOLE(2, 6);
      } else if (mak == 3) {
        if (ord == 2) PM_DIPOLE(3, 2); else if (ord == 4) PM_DIPOLE(3, 4); else PM_DIPOLE(3, 6);
      } else {
        if (ord == 2) PM_DIPOLE(4, 2); else if (ord == 4) PM_DIPOLE(4, 4); else return hipErrorInvalidValue;
      }
#undef PM_DIPOLE
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
#undef PM_TILE_ORD
#undef PM_TILE_ORD4
  return hipGetLastError();
}

hipError_t launch_dipole_scale(const unsigned int* umax_bits, double* scale, double* inv_scale,
                               double bound_per_u, double node_per_u, int batch, hipStream_t s) {
  k_dipole_scale<<<1, 64, 0, s>>>(umax_bits, scale, inv_scale, bound_per_u, node_per_u, batch);
  return hipGetLastError();
}

hipError_t launch_assemble(const AssembleArgs& a, bool out_f32, hipStream_t s) {
  if (a.slab_f32 && !out_f32) return hipErrorInvalidValue;
  if (a.g.n_g >= 256 && a.Rlo + a.Rhi <= a.T) {
    // z-runs; four cells per thread (one 1024-cell row per block) from
    // n = 1024 on: fewer, longer blocks with four times the loads in flight
    if (a.g.n_g >= 1024) {
      dim3 grid((unsigned)(a.g.M / 1024), a.batch);
      if (a.slab_f32) k_assemble_run<true, true, 4><<<grid, 256, 0, s>>>(a);
      else if (out_f32) k_assemble_run<true, false, 4><<<grid, 256, 0, s>>>(a);
      else k_assemble_run<false, false, 4><<<grid, 256, 0, s>>>(a);
    } else {
      dim3 grid((unsigned)(a.g.M / 256), a.batch);
      if (a.slab_f32) k_assemble_run<true, true, 1><<<grid, 256, 0, s>>>(a);
      else if (out_f32) k_assemble_run<true, false, 1><<<grid, 256, 0, s>>>(a);
      else k_assemble_run<false, false, 1><<<grid, 256, 0, s>>>(a);
    }
  } else {
    dim3 grid((unsigned)((a.g.M + 255) / 256), a.batch);
    if (out_f32) k_assemble<true><<<grid, 256, 0, s>>>(a);
    else k_assemble<false><<<grid, 256, 0, s>>>(a);
  }
  return hipGetLastError();
}

// ============================================================ NUFFT (ES)
// Exponential-of-semicircle spreading and interpolation (Sec. "Force
// evaluation", NUFFT paragraphs): width 6 on the fine grid, 1D weights by
// integer linear interpolation in a table of phi at 4096 samples per cell
// (20-bit values), so spreading is bit-reproducible; the 3D weight of a node
// is formed in two truncating steps, floor(floor(w_x w_y / 2^17) w_z / 2^12),
// which puts 2^31 at the kernel's peak phi(0)^3 (no remainder: the ES kernel
// is not a partition of unity).  The particles are binned by their first stencil
// node floor(u) - 2, so the window starts at the tile origin and reaches 5
// cells beyond it: window rows then start on the tile's 64-byte boundary.
namespace {
constexpr int kEsW = 6, kEsLo = kEsHaloLo, kEsHi = kEsHaloHi;
constexpr int kEsSpreadThreads = 512;  // threads per ES spread workgroup (deposit, gradient spread): 16 waves per CU at two per CU
constexpr int kEsShift = kFracBits - 12;  // 4096 samples per cell
constexpr int kEsSub = (1 << kEsShift) - 1;

__device__ __forceinline__ int es_interp(int t0, int t1, int f) {
  return t0 + (((t1 - t0) * f + (1 << (kEsShift - 1))) >> kEsShift);
}

// Table rows of one axis.  With f = frac(u) in 2^-20 cells and g = 1 - f,
// node floor(u) - m (m = 0, 1, 2) lies m + f cells from u and node
// floor(u) + 1 + m lies m + g cells away; the host table's row k holds the
// sample pairs at k + 4096 m, so row (f >> 8) serves the three nodes below
// and row (g >> 8) the three above (g = 1 reads row 4096: exact 1, 2, 3
// cells; phi is 0 at 3 cells).
struct EsAxis {
  int4 a0, b0;
  int2 a1, b1;
  int fa, fb;  // in-sample fractions (8 bits)
  int f, g;    // distances of the nodes floor(u) and floor(u) + 1
};

__device__ __forceinline__ int es_axis(long long U, const int32_t* __restrict__ tab, EsAxis& e) {
  e.f = (int)(U & ((1 << kFracBits) - 1));
  e.g = (1 << kFracBits) - e.f;
  const int32_t* ra = tab + 8 * (e.f >> kEsShift);
  const int32_t* rb = tab + 8 * (e.g >> kEsShift);
  e.a0 = *reinterpret_cast<const int4*>(ra);
  e.a1 = *reinterpret_cast<const int2*>(ra + 4);
  e.b0 = *reinterpret_cast<const int4*>(rb);
  e.b1 = *reinterpret_cast<const int2*>(rb + 4);
  e.fa = e.f & kEsSub;
  e.fb = e.g & kEsSub;
  return (int)(U >> kFracBits);
}

// integer weights of the nodes floor(u) - 2 .. floor(u) + 3
__device__ __forceinline__ void es_int_weights(const EsAxis& e, int w[kEsW]) {
  w[0] = es_interp(e.a1.x, e.a1.y, e.fa);
  w[1] = es_interp(e.a0.z, e.a0.w, e.fa);
  w[2] = es_interp(e.a0.x, e.a0.y, e.fa);
  w[3] = es_interp(e.b0.x, e.b0.y, e.fb);
  w[4] = es_interp(e.b0.z, e.b0.w, e.fb);
  w[5] = es_interp(e.b1.x, e.b1.y, e.fb);
}

__device__ __forceinline__ int es_weights(long long U, const int32_t* tab, int w[kEsW]) {
  EsAxis e;
  const int h = es_axis(U, tab, e);
  es_int_weights(e, w);
  return h;
}

// float weight and d/du phi(u - node) of one node at distance dist (2^-20
// cells), from the kernel's closed form: with z = dist / 3 cells,
// d phi / d dist = -phi beta z / (3 sqrt(1 - z^2)); 1 - z = (3 - dist) / 3 is
// formed from the integer distance, so the edge of the support stays exact.
// below: the node lies below u (d dist / du = +1), else above (-1).
// Branch-free: a node is at most 3 cells away, where the table's phi is 0,
// and there 1 - z is clamped to its smallest nonzero value so that the
// derivative is 0 times a finite factor (a branch here would wait for the
// table row of the farthest node inside it).  The product under the square
// root is at least 2^-21, so the bare reciprocal square root needs no
// denormal scaling.
__device__ __forceinline__ void es_node_d(int wi, int dist, bool below, float beta, float& w, float& dw) {
  constexpr float inv = 1.0f / (float)(1 << kWeightBits);
  constexpr int kHalf = (kEsW / 2) << kFracBits;  // 3 cells
  constexpr float kInvHalf = 1.0f / (float)kHalf;
  const float phi = (float)wi * inv;
  w = phi;
  const float z = (float)dist * kInvHalf, omz = (float)max(kHalf - dist, 1) * kInvHalf;
  const float dphi = -phi * beta * z * (1.0f / (float)(kEsW / 2)) * __builtin_amdgcn_rsqf(omz * (1.f + z));
  dw = (below && dist > 0) ? dphi : -dphi;
}

// weights and derivatives from an axis' table rows
__device__ __forceinline__ void es_axis_weights_d(const EsAxis& e, float beta, float w[kEsW], float dw[kEsW]) {
  int wi[kEsW];
  es_int_weights(e, wi);
  constexpr int one = 1 << kFracBits;
  es_node_d(wi[0], 2 * one + e.f, true, beta, w[0], dw[0]);
  es_node_d(wi[1], one + e.f, true, beta, w[1], dw[1]);
  es_node_d(wi[2], e.f, true, beta, w[2], dw[2]);
  es_node_d(wi[3], e.g, false, beta, w[3], dw[3]);
  es_node_d(wi[4], one + e.g, false, beta, w[4], dw[4]);
  es_node_d(wi[5], 2 * one + e.g, false, beta, w[5], dw[5]);
}

__device__ __forceinline__ int es_weights_d(long long U, const int32_t* __restrict__ tab, float beta,
                                            float w[kEsW], float dw[kEsW]) {
  EsAxis e;
  const int h = es_axis(U, tab, e);
  es_axis_weights_d(e, beta, w, dw);
  return h;
}

// fixed-point weight of one node from A = floor(w_x w_y / 2^17) < 2^24 and
// the z weight c <= 2^20: floor(A c / 2^12) <= 2^31, the low 32 bits of a
// 24 x 24-bit product shifted (mul_u24, mul_hi_u24, one funnel shift)
__device__ __forceinline__ unsigned es_node_mass(unsigned A, unsigned c) {
  const unsigned long long p = (unsigned long long)(A & 0xffffffu) * (c & 0xffffffu);  // < 2^44
  return (unsigned)(p >> 12);
}

// The ES windows are (16 + 5)^3 (every NUFFT mesh has 16-cell tiles) and are
// loaded straight into LDS (global_load_lds_dword: lane l of a wave writes
// the dword at M0 + 4 l), element e = 256 k + 64 wave + lane, so no data
// passes through registers and every load of the window is in flight at
// once: one HBM round trip per window.  The LDS buffer is padded to whole
// rounds (kEsWinLds floats); lanes past the window re-read a valid cell into
// the padding.
constexpr int kEsWin = kTileMax + kEsLo + kEsHi;
constexpr int kEsWin3 = kEsWin * kEsWin * kEsWin;
constexpr int kEsWinLds = (kEsWin3 + 255) / 256 * 256;

__device__ __forceinline__ void load_window_es(float* win, const float* __restrict__ mesh, const int o[3], int L,
                                               int nm) {
  constexpr int W = kEsWin, W2 = W * W, NE = kEsWinLds / 256;
  const int lane = threadIdx.x & 63, wbase = threadIdx.x & ~63;
#pragma unroll 4
  for (int k = 0; k < NE; ++k) {
    const int e0 = 256 * k + wbase, e = min(e0 + lane, kEsWin3 - 1);
    const int lx = e / W2, r = e - lx * W2, ly = r / W, lz = r - ly * W;
    const int gx = (o[0] - kEsLo + lx) & nm, gy = (o[1] - kEsLo + ly) & nm, gz = (o[2] - kEsLo + lz) & nm;
    // (a mesh of at most 1024^3 cells: the cell index fits 32 bits)
    const float* src = mesh + ((((unsigned)gx << L | (unsigned)gy) << L) | (unsigned)gz);
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(win + e0), 4, 0, 0);
  }
  __builtin_amdgcn_s_waitcnt(0);  // this thread's window loads have landed (the caller's barrier does the rest)
}
}  // namespace

// Particle loads are software-pipelined: the next particle's index and
// coordinates are in flight while the current one scatters.  Lanes of a wave
// take consecutive entries of the tile's bank order (below), whose window
// bases mostly differ modulo 64: the int64 atomics of one instruction rarely
// share a bank or an address.
__global__ void __launch_bounds__(kEsSpreadThreads) k_tile_es_deposit(TileArgs a) {
  constexpr int NT = kEsSpreadThreads;
  extern __shared__ unsigned long long ewin[];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  constexpr int W = kEsWin, W3 = W * W * W;
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  int p = beg + (int)threadIdx.x;  // consecutive lanes of the bank order: window bases spread over the banks
  long long i = 0;
  float x0 = 0.f, x1 = 0.f, x2 = 0.f;
  if (p < end) {
    i = a.sorted[slot * N + a.bank[slot * N + p]];
    x0 = a.disp[ps + i];
    x1 = a.disp[ps + N + i];
    x2 = a.disp[ps + 2 * N + i];
  }
  for (int e = threadIdx.x; e < W3; e += NT) ewin[e] = 0ull;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  __syncthreads();
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  for (; p < end; p += NT) {
    long long j[3];
    lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
    const float xc[3] = {x0, x1, x2};
    int w[3][kEsW], l0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long U = fixed_coord(j[c], xc[c], a.g.log2_r, umask);
      l0[c] = ((es_weights(U, a.es_tab, w[c]) - kEsAnchor) & nm) - o[c];  // first node floor(u) - 2
    }
    if (p + NT < end) {
      i = a.sorted[slot * N + a.bank[slot * N + p + NT]];
      x0 = a.disp[ps + i];
      x1 = a.disp[ps + N + i];
      x2 = a.disp[ps + 2 * N + i];
    }
#pragma unroll
    for (int x = 0; x < kEsW; ++x)
#pragma unroll
      for (int y = 0; y < kEsW; ++y) {
        const unsigned long long ab =
            (unsigned long long)((unsigned)w[0][x] & 0xffffffu) * ((unsigned)w[1][y] & 0xffffffu);  // <= 2^40
        const unsigned A = (unsigned)(ab >> 17);                                                   // <= 2^23
        unsigned long long* row = ewin + ((l0[0] + x) * W + l0[1] + y) * W + l0[2];
#pragma unroll
        for (int z = 0; z < kEsW; ++z) atomicAdd(row + z, (unsigned long long)es_node_mass(A, (unsigned)w[2][z]));
      }
  }
  __syncthreads();
  if (a.win_f32)
    store_window_f32(ewin, reinterpret_cast<float*>(a.scratch) + (long long)slot * a.n_tiles * W3, t, W, a.log2nt,
                     a.win_scale != 0.0 ? a.win_scale : a.inv_scale[slot]);
  else
    store_window(ewin, reinterpret_cast<unsigned long long*>(a.scratch) + (long long)slot * a.n_tiles * W3, t, W,
                 a.log2nt);
}

// A_c = sum_j g_c(j) phi(u - j) from the three force meshes, then the kick
// and drift (or A only for the force hook).  The components take turns in
// one LDS window (V_c = alpha V_c + beta A_c is per component), so three
// workgroups fit on a CU; the drift follows once every V_c is updated.
__device__ __forceinline__ float es_contract(const float* __restrict__ win, int W, const int l0[3],
                                             const float (&w)[3][kEsW]) {
  float A = 0.f;
#pragma unroll
  for (int xx = 0; xx < kEsW; ++xx) {
    float sx = 0.f;
#pragma unroll
    for (int yy = 0; yy < kEsW; ++yy) {
      const int b = ((l0[0] + xx) * W + l0[1] + yy) * W + l0[2];
      float r = 0.f;
#pragma unroll
      for (int zz = 0; zz < kEsW; ++zz) r += w[2][zz] * win[b + zz];
      sx += w[1][yy] * r;
    }
    A += w[0][xx] * sx;
    __builtin_amdgcn_sched_barrier(0);  // one x plane of reads in flight at a time (register pressure)
  }
  return A;
}

// weights and window-local first nodes from given coordinates
__device__ __forceinline__ void es_particle_x(const TileArgs& a, long long i, const float x[3], const int o[3],
                                              long long umask, int nm, float (&w)[3][kEsW], int (&l0)[3]) {
  constexpr float inv = 1.0f / (float)(1 << kWeightBits);
  long long j[3];
  lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int wi[kEsW];
    long long U = fixed_coord(j[c], x[c], a.g.log2_r, umask);
    l0[c] = ((es_weights(U, a.es_tab, wi) - kEsAnchor) & nm) - o[c];
#pragma unroll
    for (int q = 0; q < kEsW; ++q) w[c][q] = (float)wi[q] * inv;
  }
}

__device__ __forceinline__ void es_particle(const TileArgs& a, long long i, const int o[3], long long umask, int nm,
                                            float (&w)[3][kEsW], int (&l0)[3]) {
  constexpr float inv = 1.0f / (float)(1 << kWeightBits);
  const long long N = a.g.N, ps = (long long)blockIdx.y * a.g.part_stride;
  long long j[3];
  lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    int wi[kEsW];
    long long U = fixed_coord(j[c], a.disp[ps + c * N + i], a.g.log2_r, umask);
    l0[c] = ((es_weights(U, a.es_tab, wi) - kEsAnchor) & nm) - o[c];
#pragma unroll
    for (int q = 0; q < kEsW; ++q) w[c][q] = (float)wi[q] * inv;
  }
}

// The first particle of every thread keeps its weights, position and
// velocity in registers over the three components, so its dependent loads
// (index, position, table rows) are paid once; the others (a tile holds 512
// particles on average) recompute them per component.  One cached particle
// at <= 128 VGPRs (four workgroups per CU) measured 5% faster than two at
// <= 168 (three per CU).
__global__ void __launch_bounds__(256, 4) k_tile_es_kick(TileArgs a) {  // <= 128 VGPRs: 4 waves per SIMD
  extern __shared__ float fwin[];  // one (T + 5)^3 window, the components in turn
  constexpr int K = 1;
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  const int W = a.T + kEsLo + kEsHi;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  const float al = a.alpha[slot], be = a.beta[slot], tp = a.tau[slot];
  const bool force_only = a.acc_out != nullptr;
  float wk[K][3][kEsW], xk[K][3], vk[K][3];
  int lk[K][3];
  long long ik[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int p = beg + threadIdx.x + 256 * k;
    ik[k] = p < end ? a.sorted[slot * N + p] : 0;
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool ok = beg + (int)threadIdx.x + 256 * k < end;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xk[k][c] = ok ? a.disp[ps + c * N + ik[k]] : 0.f;
      vk[k][c] = ok && !force_only ? a.vel[ps + c * N + ik[k]] : 0.f;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) es_particle_x(a, ik[k], xk[k], o, umask, nm, wk[k], lk[k]);
  for (int c = 0; c < 3; ++c) {
    if (c) __syncthreads();  // the previous component's reads are done
    load_window_es(fwin, a.mesh_in + slot * 3 * a.comp_stride + c * a.comp_stride, o, a.g.log2_ng, nm);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (beg + (int)threadIdx.x + 256 * k >= end) continue;
      const float A = es_contract(fwin, W, lk[k], wk[k]);
      if (force_only)
        a.acc_out[ps + c * N + ik[k]] = A;
      else
        vk[k][c] = kick_v(al, vk[k][c], be, A);
    }
    // the others: the table rows of the three axes together, the velocity
    // and the next particle's coordinates in flight during the contraction
    int p = beg + (int)threadIdx.x + 256 * K;
    long long i = 0;
    float x[3] = {0.f, 0.f, 0.f};
    if (p < end) {
      i = a.sorted[slot * N + p];
#pragma unroll
      for (int d = 0; d < 3; ++d) x[d] = a.disp[ps + d * N + i];
    }
    for (; p < end; p += 256) {
      float w[3][kEsW];
      int l0[3];
      {
        long long j[3];
        lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
        EsAxis e[3];
#pragma unroll
        for (int d = 0; d < 3; ++d)
          l0[d] = ((es_axis(fixed_coord(j[d], x[d], a.g.log2_r, umask), a.es_tab, e[d]) - kEsAnchor) & nm) - o[d];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          int wi[kEsW];
          es_int_weights(e[d], wi);
#pragma unroll
          for (int q = 0; q < kEsW; ++q) w[d][q] = (float)wi[q] * (1.0f / (float)(1 << kWeightBits));
        }
      }
      const float v = force_only ? 0.f : a.vel[ps + c * N + i];
      const long long in = a.sorted[slot * N + min(p + 256, end - 1)];  // (the last round reads its own)
#pragma unroll
      for (int d = 0; d < 3; ++d) x[d] = a.disp[ps + d * N + in];
      const float A = es_contract(fwin, W, l0, w);
      if (force_only)
        a.acc_out[ps + c * N + i] = A;
      else
        a.vel[ps + c * N + i] = kick_v(al, v, be, A);
      i = in;
    }
  }
  if (force_only) return;
#pragma unroll
  for (int k = 0; k < K; ++k) {  // drift
    if (beg + (int)threadIdx.x + 256 * k >= end) continue;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      a.vel[ps + c * N + ik[k]] = vk[k][c];
      a.disp[ps + c * N + ik[k]] = drift_x(xk[k][c], tp, vk[k][c]);
    }
  }
  for (int p = beg + threadIdx.x + 256 * K; p < end; p += 256) {  // this thread's own V writes
    const long long i = a.sorted[slot * N + p];
    float x[3], v[3];  // every load before the stores (which the compiler cannot order past them)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      x[c] = a.disp[ps + c * N + i];
      v[c] = a.vel[ps + c * N + i];
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) a.disp[ps + c * N + i] = drift_x(x[c], tp, v[c]);
  }
}

// ------------------------------------------------ NUFFT adjoint (ES kernel)

// reverse kick with the ES gather of the 3 force meshes and its position
// gradient: V = (V - beta A) / alpha, V_bar = alpha V_bar, u = beta V_bar,
// X_bar += r sum_c u_c dA_c/du; u kept in sorted order with max |u|
// separable contraction of a window with the weights and their gradient:
// A = sum w0 w1 w2 f, dA[d] = the same with w_d replaced by dw_d
__device__ __forceinline__ void es_contract_grad(const float* __restrict__ win, int W, const int l0[3],
                                                 const float (&w)[3][kEsW], const float (&dw)[3][kEsW], float& A,
                                                 float (&dA)[3]) {
  A = 0.f;
  dA[0] = dA[1] = dA[2] = 0.f;
#pragma unroll
  for (int xx = 0; xx < kEsW; ++xx) {
    float sww = 0.f, sdw = 0.f, swd = 0.f;
#pragma unroll
    for (int yy = 0; yy < kEsW; ++yy) {
      const int b = ((l0[0] + xx) * W + l0[1] + yy) * W + l0[2];
      float rw = 0.f, rd = 0.f;
#pragma unroll
      for (int zz = 0; zz < kEsW; ++zz) {
        const float f = win[b + zz];
        rw += w[2][zz] * f;
        rd += dw[2][zz] * f;
      }
      sww += w[1][yy] * rw;
      sdw += dw[1][yy] * rw;
      swd += w[1][yy] * rd;
    }
    A += w[0][xx] * sww;
    dA[0] += dw[0][xx] * sww;
    dA[1] += w[0][xx] * sdw;
    dA[2] += w[0][xx] * swd;
  }
}

__device__ __forceinline__ void es_particle_d(const TileArgs& a, long long i, const float x[3], const int o[3],
                                              long long umask, int nm, float (&w)[3][kEsW], float (&dw)[3][kEsW],
                                              int (&l0)[3]) {
  long long j[3];
  lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    long long U = fixed_coord(j[d], x[d], a.g.log2_r, umask);
    l0[d] = ((es_weights_d(U, a.es_tab, a.es_beta, w[d], dw[d]) - kEsAnchor) & nm) - o[d];
  }
}

// The weights are recomputed per component: keeping them in registers over
// the components costs more registers than the occupancy allows.  The
// particle loop keeps its dependent loads in flight together: the table rows
// of all three axes are issued at once, the particle's velocity and
// cotangents (read for the update) and the next particle's index and
// coordinates load during the weights and the contraction.
__global__ void __launch_bounds__(256) k_tile_es_adj_kick(TileArgs a) {
  extern __shared__ float fwin[];  // one (T + 5)^3 window, the components in turn
  __shared__ float red[256];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  const int W = a.T + kEsLo + kEsHi;  // (a runtime stride keeps the contraction compact)
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  const float al = a.alpha[slot], be = a.beta[slot];
  const float r = (float)(1 << a.g.log2_r);
  float umax = 0.f;
  for (int c = 0; c < 3; ++c) {
    if (c) __syncthreads();
    load_window_es(fwin, a.mesh_in + slot * 3 * a.comp_stride + c * a.comp_stride, o, a.g.log2_ng, nm);
    __syncthreads();
    int p = beg + (int)threadIdx.x;
    long long i = 0;
    float x[3] = {0.f, 0.f, 0.f};
    if (p < end) {
      i = a.sorted[slot * N + p];
#pragma unroll
      for (int d = 0; d < 3; ++d) x[d] = a.disp[ps + d * N + i];
    }
    for (; p < end; p += 256) {
      long long j[3];
      lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
      EsAxis e[3];
      int l0[3];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        l0[d] = ((es_axis(fixed_coord(j[d], x[d], a.g.log2_r, umask), a.es_tab, e[d]) - kEsAnchor) & nm) - o[d];
      const float v = a.vel[ps + c * N + i], vb = a.vbar[ps + c * N + i];
      float xb[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) xb[d] = a.xbar[ps + d * N + i];
      const long long in = a.sorted[slot * N + min(p + 256, end - 1)];  // (the last round reads its own)
      float w[3][kEsW], dw[3][kEsW];
#pragma unroll
      for (int d = 0; d < 3; ++d) es_axis_weights_d(e[d], a.es_beta, w[d], dw[d]);
      float xn[3];
#pragma unroll
      for (int d = 0; d < 3; ++d) xn[d] = a.disp[ps + d * N + in];
      float A, dA[3];
      es_contract_grad(fwin, W, l0, w, dw, A, dA);
      // reverse kick: V = (V - beta A) / alpha, V_bar = alpha V_bar, u = beta V_bar
      const float u = be * vb;
      a.vel[ps + c * N + i] = (v - be * A) / al;
      a.vbar[ps + c * N + i] = al * vb;
      a.u_sorted[ps + c * N + p] = u;
      umax = fmaxf(umax, fabsf(u));
#pragma unroll
      for (int d = 0; d < 3; ++d) a.xbar[ps + d * N + i] = xb[d] + r * u * dA[d];
      i = in;
#pragma unroll
      for (int d = 0; d < 3; ++d) x[d] = xn[d];
    }
  }
  red[threadIdx.x] = umax;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.f)
    atomicMax(reinterpret_cast<unsigned int*>(a.umax) + slot, __float_as_uint(red[0]));
}

// Spreading of d(j) = sum_c u_c d/du_c phi3(u - j) (the kernel's gradient
// along the cotangent u) for the adjoint's mesh term: the Fourier transform
// of the spread gradient is -i k_c times that of the spread of u_c, so one
// spread replaces the three per-component spreads and their transforms.
// Fixed point at the scale set from max |u|: each node value is below 2^31
// (|phi| <= 1, |phi'| < 1 per cell, so |d| < 3 max|u|), rounded half-even in
// FP32 and summed as int64 (order-free).
__global__ void __launch_bounds__(kEsSpreadThreads) k_tile_es_divspread(TileArgs a) {
  constexpr int NT = kEsSpreadThreads;
  extern __shared__ unsigned long long ewin[];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  constexpr int W = kEsWin, W3 = W * W * W;
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  int p = beg + (int)threadIdx.x;  // consecutive lanes of the bank order: window bases spread over the banks
  long long i = 0;
  float u0 = 0.f, u1 = 0.f, u2 = 0.f, x0 = 0.f, x1 = 0.f, x2 = 0.f;
  // forward mode (tan_xbar): the spread's tangent, u = coef Xdot from xbar
  const bool tan = a.tan_xbar != 0;
  const float tc = a.coef[slot];
  if (p < end) {
    const int q = a.bank[slot * N + p];
    i = a.sorted[slot * N + q];
    u0 = tan ? tc * a.xbar[ps + i] : a.u_sorted[ps + q];
    u1 = tan ? tc * a.xbar[ps + N + i] : a.u_sorted[ps + N + q];
    u2 = tan ? tc * a.xbar[ps + 2 * N + i] : a.u_sorted[ps + 2 * N + q];
    x0 = a.disp[ps + i];
    x1 = a.disp[ps + N + i];
    x2 = a.disp[ps + 2 * N + i];
  }
  for (int e = threadIdx.x; e < W3; e += NT) ewin[e] = 0ull;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  __syncthreads();
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  const float S = (float)a.scale[slot];  // a power of two
  for (; p < end; p += NT) {
    const bool any = u0 != 0.f || u1 != 0.f || u2 != 0.f;
    const float u[3] = {u0 * S, u1 * S, u2 * S};
    long long j[3];
    lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
    const float xc[3] = {x0, x1, x2};
    float w[3][kEsW], dw[3][kEsW];
    int l0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long U = fixed_coord(j[c], xc[c], a.g.log2_r, umask);
      l0[c] = ((es_weights_d(U, a.es_tab, a.es_beta, w[c], dw[c]) - kEsAnchor) & nm) - o[c];
    }
    if (p + NT < end) {
      const int q = a.bank[slot * N + p + NT];
      i = a.sorted[slot * N + q];
      u0 = tan ? tc * a.xbar[ps + i] : a.u_sorted[ps + q];
      u1 = tan ? tc * a.xbar[ps + N + i] : a.u_sorted[ps + N + q];
      u2 = tan ? tc * a.xbar[ps + 2 * N + i] : a.u_sorted[ps + 2 * N + q];
      x0 = a.disp[ps + i];
      x1 = a.disp[ps + N + i];
      x2 = a.disp[ps + 2 * N + i];
    }
    if (!any) continue;
#pragma unroll
    for (int x = 0; x < kEsW; ++x)
#pragma unroll
      for (int y = 0; y < kEsW; ++y) {
        // v(z) = (u_x w0' w1 + u_y w0 w1') w2(z) + u_z w0 w1 w2'(z)
        const float pa = u[0] * dw[0][x] * w[1][y] + u[1] * w[0][x] * dw[1][y];
        const float pb = u[2] * w[0][x] * w[1][y];
        unsigned long long* row = ewin + ((l0[0] + x) * W + l0[1] + y) * W + l0[2];
#pragma unroll
        for (int z = 0; z < kEsW; ++z) {
          const int v = (int)rintf(pa * w[2][z] + pb * dw[2][z]);
          atomicAdd(row + z, (unsigned long long)(long long)v);
        }
      }
  }
  __syncthreads();
  if (a.win_f32)
    store_window_f32(ewin, reinterpret_cast<float*>(a.scratch) + (long long)slot * a.n_tiles * W3, t, W, a.log2nt,
                     a.win_scale != 0.0 ? a.win_scale : a.inv_scale[slot]);
  else
    store_window(ewin, reinterpret_cast<unsigned long long*>(a.scratch) + (long long)slot * a.n_tiles * W3, t, W,
                 a.log2nt);
}

// X_bar += coef r sum_j b_bar_j d/du phi(u - j) (the spreading differentiated
// w.r.t. the positions), then the reverse drift X -= tau V, V_bar += tau X_bar
__global__ void __launch_bounds__(256) k_tile_es_adj_drift(TileArgs a) {
  extern __shared__ float bwin[];  // (T + 5)^3
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  const int W = a.T + kEsLo + kEsHi;  // (a runtime stride keeps the contraction compact)
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  load_window_es(bwin, a.mesh_in + slot * a.g.mesh_stride, o, a.g.log2_ng, a.g.n_g - 1);
  __syncthreads();
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  const float cf = a.coef[slot] * (float)(1 << a.g.log2_r), tau = a.tau[slot];
  // as in the adjoint kick: the table rows of the three axes together, the
  // update operands and the next particle's coordinates in flight during the
  // contraction
  int p = beg + (int)threadIdx.x;
  long long i = 0;
  float xv[3] = {0.f, 0.f, 0.f};
  if (p < end) {
    i = a.sorted[slot * N + p];
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[c] = a.disp[ps + c * N + i];
  }
  for (; p < end; p += 256) {
    const float x[3] = {xv[0], xv[1], xv[2]};
    long long j[3];
    lattice_of(i, a.g.log2_np, a.g.log2_pb, j);
    EsAxis e[3];
    int l0[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      l0[c] = ((es_axis(fixed_coord(j[c], x[c], a.g.log2_r, umask), a.es_tab, e[c]) - kEsAnchor) & nm) - o[c];
    float xb0[3], v0[3], vb0[3], il[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      xb0[c] = a.il_out ? 0.f : a.xbar[ps + c * N + i];
      v0[c] = a.il_out ? 0.f : a.vel[ps + c * N + i];
      vb0[c] = a.il_out ? 0.f : a.vbar[ps + c * N + i];
      il[c] = a.il_in ? a.il_in[2 * ps + c * N + i] : 0.f;
    }
    const long long in = a.sorted[slot * N + min(p + 256, end - 1)];  // (the last round reads its own)
    float w[3][kEsW], dw[3][kEsW];
#pragma unroll
    for (int c = 0; c < 3; ++c) es_axis_weights_d(e[c], a.es_beta, w[c], dw[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) xv[c] = a.disp[ps + c * N + in];
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int xx = 0; xx < kEsW; ++xx) {
      float sww = 0.f, sdw = 0.f, swd = 0.f;
#pragma unroll
      for (int yy = 0; yy < kEsW; ++yy) {
        const int b = ((l0[0] + xx) * W + l0[1] + yy) * W + l0[2];
        float rw = 0.f, rd = 0.f;
#pragma unroll
        for (int zz = 0; zz < kEsW; ++zz) {
          const float f = bwin[b + zz];
          rw += w[2][zz] * f;
          rd += dw[2][zz] * f;
        }
        sww += w[1][yy] * rw;
        sdw += dw[1][yy] * rw;
        swd += w[1][yy] * rd;
      }
      gx += dw[0][xx] * sww;
      gy += w[0][xx] * sdw;
      gz += w[0][xx] * swd;
    }
    float g[3] = {cf * gx, cf * gy, cf * gz};
    if (a.il_in) {  // interlaced grids: the mean of the two grids' scatter terms
#pragma unroll
      for (int c = 0; c < 3; ++c) g[c] = 0.5f * (g[c] + il[c]);
    }
    if (a.il_out) {  // the first grid: its term only, the state untouched
#pragma unroll
      for (int c = 0; c < 3; ++c) a.il_out[2 * ps + c * N + i] = g[c];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float xb = xb0[c] + g[c];
        a.disp[ps + c * N + i] = x[c] - tau * v0[c];
        a.xbar[ps + c * N + i] = xb;
        a.vbar[ps + c * N + i] = vb0[c] + tau * xb;
      }
    }
    i = in;
  }
}

// Forward-mode tangent kick with the ES kernel: per component, the direct
// part r sum_d dA_c/du_d Xdot_d from the primal force mesh (into acc_out,
// [B][3][N]), then the gather of the tangent force mesh (mesh_in2) and
// Vdot_c = alpha Vdot_c + beta (both); finally Xdot += tau Vdot (Xdot in
// xbar, Vdot in vbar)
__global__ void __launch_bounds__(256) k_tile_es_tan_kick(TileArgs a) {
  extern __shared__ float fwin[];  // one (T + 5)^3 window, the meshes in turn
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  const int W = a.T + kEsLo + kEsHi;
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  const float al = a.alpha[slot], be = a.beta[slot], tp = a.tau[slot];
  const float r = (float)(1 << a.g.log2_r);
  for (int c = 0; c < 3; ++c) {
    if (c) __syncthreads();
    load_window_es(fwin, a.mesh_in + slot * 3 * a.comp_stride + c * a.comp_stride, o, a.g.log2_ng, nm);
    __syncthreads();
    for (int p = beg + threadIdx.x; p < end; p += 256) {
      const long long i = a.sorted[slot * N + p];
      const float x[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
      float w[3][kEsW], dw[3][kEsW];
      int l0[3];
      es_particle_d(a, i, x, o, umask, nm, w, dw, l0);
      float A, dA[3];
      es_contract_grad(fwin, W, l0, w, dw, A, dA);
      a.acc_out[ps + c * N + i] =
          r * (dA[0] * a.xbar[ps + i] + dA[1] * a.xbar[ps + N + i] + dA[2] * a.xbar[ps + 2 * N + i]);
    }
    __syncthreads();
    load_window_es(fwin, a.mesh_in2 + slot * 3 * a.comp_stride + c * a.comp_stride, o, a.g.log2_ng, nm);
    __syncthreads();
    for (int p = beg + threadIdx.x; p < end; p += 256) {
      const long long i = a.sorted[slot * N + p];
      float w[3][kEsW];
      int l0[3];
      es_particle(a, i, o, umask, nm, w, l0);
      const float J = es_contract(fwin, W, l0, w) + a.acc_out[ps + c * N + i];
      a.vbar[ps + c * N + i] = kick_v(al, a.vbar[ps + c * N + i], be, J);
    }
  }
  for (int p = beg + threadIdx.x; p < end; p += 256) {  // this thread's own particles
    const long long i = a.sorted[slot * N + p];
#pragma unroll
    for (int c = 0; c < 3; ++c)
      a.xbar[ps + c * N + i] = drift_x(a.xbar[ps + c * N + i], tp, a.vbar[ps + c * N + i]);
  }
}


// raise the dynamic-LDS limit of every kernel that needs more than the
// default, to its largest window (16^3 tiles); called once per bind, outside
// any stream capture
hipError_t configure_tile_kernels() {
  constexpr int We = kTileMax + kEsLo + kEsHi;
  const int es64 = We * We * We * 8, es32 = kEsWinLds * 4;
  auto dip = [](int o, int kr) { int W = kTileMax + 2 * (kr + o / 2); return W * W * W * 8; };
  const hipFuncAttribute A = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipSuccess;
  auto set = [&](const void* f, int bytes) {
    hipError_t r = hipFuncSetAttribute(f, A, bytes);
    if (e == hipSuccess) e = r;
  };
  set((const void*)k_tile_dipole<2, 2>, dip(2, 1));
  set((const void*)k_tile_dipole<2, 4>, dip(4, 1));
  set((const void*)k_tile_dipole<2, 6>, dip(6, 1));
  set((const void*)k_tile_dipole<3, 2>, dip(2, 1));
  set((const void*)k_tile_dipole<3, 4>, dip(4, 1));
  set((const void*)k_tile_dipole<3, 6>, dip(6, 1));
  set((const void*)k_tile_dipole<4, 2>, dip(2, 2));
  set((const void*)k_tile_dipole<4, 4>, dip(4, 2));
  set((const void*)k_tile_es_deposit, es64);
  set((const void*)k_tile_es_kick, es32);
  set((const void*)k_tile_es_adj_kick, es32);
  set((const void*)k_tile_es_divspread, es64);
  set((const void*)k_tile_es_adj_drift, es32);
  set((const void*)k_tile_es_tan_kick, es32);
  return e;
}

// ------------------------------------------------ LDS bank order (ES)

// Every LDS access of an ES spread is a particle's window base plus an offset
// that all lanes of the instruction share (the unrolled 6^3 loop), so the
// bank conflicts of an instruction are set by the bases of the wave's
// particles.  The spreads' accesses are 8-byte atomics on int64 window
// cells, each on a pair of the 32 four-byte banks; they run without
// conflicts when every 16 consecutive lanes hold distinct bases mod 16 (a
// deal by base mod 16 that gives consecutive lanes the same class was 40%
// slower than one that steps through the classes).  For each tile this
// writes `bank`, an order of its entries in `sorted`, in chunks of
// kBankChunk: the entries are counted by base mod 16 and dealt round-robin,
// round r holding the r-th entry of every class that has one, in class
// order, so consecutive entries take distinct classes until the smaller
// classes run out.  The spreads take their particles in this order; their
// results are integer sums and do not depend on it.  The gathers keep the
// tile's lattice order, whose particle data is contiguous in memory.
constexpr int kBankChunk = 1024;
constexpr int kBankKeys = 16;

__global__ void __launch_bounds__(256) k_tile_es_bank_order(TileArgs a, int32_t* bank) {
  constexpr int KE = kBankChunk / 256;
  __shared__ int cnt[kBankKeys];
  const int slot = blockIdx.y, t = (int)xcd_block(blockIdx.x, gridDim.x);
  if (!((a.active >> slot) & 1ull)) return;
  constexpr int W = kEsWin;  // the spread windows' row stride
  int o[3];
  tile_origin(t, TileGeo{a.T, a.log2T, a.log2nt, a.n_tiles, a.ts}, o);
  const long long N = a.g.N, ps = slot * a.g.part_stride;
  const int beg = a.offset[slot * a.ts + t], end = a.offset[slot * a.ts + t + 1];
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  const int nm = a.g.n_g - 1;
  const int32_t* list = a.sorted + slot * N;
  int32_t* out = bank + slot * N;
  for (int c0 = beg; c0 < end; c0 += kBankChunk) {
    const int m = min(kBankChunk, end - c0);
    if (threadIdx.x < kBankKeys) cnt[threadIdx.x] = 0;
    __syncthreads();
    // every entry's index, then every coordinate, before any use (entries
    // past the chunk read its last one): loads under the per-entry branch
    // were waited for one after another
    int32_t id[KE];
    float xq[KE][3];
#pragma unroll
    for (int k = 0; k < KE; ++k) id[k] = list[c0 + min((int)threadIdx.x + 256 * k, m - 1)];
#pragma unroll
    for (int k = 0; k < KE; ++k)
#pragma unroll
      for (int c = 0; c < 3; ++c) xq[k][c] = a.disp[ps + c * N + id[k]];
    int res[KE], rank[KE];
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      res[k] = rank[k] = 0;
      if (e < m) {
        long long j[3];
        lattice_of(id[k], a.g.log2_np, a.g.log2_pb, j);
        int l0[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const long long U = fixed_coord(j[c], xq[k][c], a.g.log2_r, umask);
          l0[c] = (((int)(U >> kFracBits) - kEsAnchor) & nm) - o[c];
        }
        res[k] = ((l0[0] * W + l0[1]) * W + l0[2]) & (kBankKeys - 1);
        rank[k] = atomicAdd(&cnt[res[k]], 1);
      }
    }
    __syncthreads();  // every entry of the chunk is counted
    int cn[kBankKeys];
#pragma unroll
    for (int c = 0; c < kBankKeys; ++c) cn[c] = cnt[c];
    // entry r of class k: the rounds before r hold sum_c min(cn_c, r)
    // entries, and round r the classes below k that still have an r-th
#pragma unroll
    for (int k = 0; k < KE; ++k) {
      const int e = (int)threadIdx.x + 256 * k;
      if (e >= m) continue;
      const int r = rank[k];
      int pos = 0;
#pragma unroll
      for (int c = 0; c < kBankKeys; ++c) pos += min(cn[c], r) + (c < res[k] && cn[c] > r ? 1 : 0);
      out[c0 + pos] = c0 + e;
    }
    __syncthreads();  // the counters are read before the next chunk clears them
  }
}

hipError_t launch_es_bank_order(const TileArgs& a, int32_t* bank, hipStream_t s) {
  if (a.T != kTileMax) return hipErrorInvalidValue;
  k_tile_es_bank_order<<<dim3((unsigned)a.n_tiles, a.batch), 256, 0, s>>>(a, bank);
  return hipGetLastError();
}

hipError_t launch_tile_es(const TileArgs& a, int kind, hipStream_t s) {
  dim3 grid((unsigned)a.n_tiles, a.batch);
  if (a.T != kTileMax) return hipErrorInvalidValue;  // the ES kernels assume 16-cell tiles
  const int W = kEsWin;
  const size_t fl = (size_t)kEsWinLds * sizeof(float);  // gather windows (padded)
  if (kind == TK_ES_DEPOSIT) {
    size_t lds = (size_t)W * W * W * sizeof(unsigned long long);
    k_tile_es_deposit<<<grid, kEsSpreadThreads, lds, s>>>(a);
  } else if (kind == TK_ES_KICK) {
    k_tile_es_kick<<<grid, 256, fl, s>>>(a);
  } else if (kind == TK_ES_ADJ_KICK) {
    k_tile_es_adj_kick<<<grid, 256, fl, s>>>(a);
  } else if (kind == TK_ES_DIPOLE) {
    size_t lds = (size_t)W * W * W * sizeof(unsigned long long);
    k_tile_es_divspread<<<grid, kEsSpreadThreads, lds, s>>>(a);
  } else if (kind == TK_ES_ADJ_DRIFT) {
    k_tile_es_adj_drift<<<grid, 256, fl, s>>>(a);
  } else if (kind == TK_ES_TAN_KICK) {
    k_tile_es_tan_kick<<<grid, 256, fl, s>>>(a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pm
