// Register-resident column FFT: the four-step split L = P * E inside one
// workgroup.  C columns per workgroup, P = 256 / C threads per column, each
// thread holding E = L / P elements of its column.
//
//   input layout : thread n1 holds x[n1 + P n2], n2 = 0 .. E-1
//   pass A       : E-point DFT over n2 in registers, twiddle W_L^(n1 k2)
//   exchange     : through LDS
//   pass B       : the thread takes k2 = n1 + j P (j < E / P) and runs the
//                  P-point DFTs over n1 in registers
//   output layout: value j P + k1 of thread n1 is X[(n1 + j P) + E k1]
//
// X[k2 + E k1] = sum_n1 W_P^(n1 k1) W_L^(n1 k2) sum_n2 W_E^(n2 k2) x[n1 + P n2]
// is the DFT of length L.  One LDS round trip replaces the log2(L) LDS
// stages of a radix-2/4 Stockham pass.  The functions are host-callable so
// that the index algebra can be exercised by a CPU emulation of one block.
#pragma once
#include <hip/hip_runtime.h>

namespace pm {
namespace freg {

__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmulw(float2 a, float2 w) {
  return make_float2(a.x * w.x - a.y * w.y, a.x * w.y + a.y * w.x);
}

// exp(-2 pi i k / 32), k = 0 .. 15
struct Tw32 {
  static constexpr float re[16] = {1.000000000e+00f,  9.807852804e-01f,  9.238795325e-01f,  8.314696123e-01f,
                                   7.071067812e-01f,  5.555702330e-01f,  3.826834324e-01f,  1.950903220e-01f,
                                   0.0f,              -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
                                   -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f};
  static constexpr float im[16] = {0.0f,              -1.950903220e-01f, -3.826834324e-01f, -5.555702330e-01f,
                                   -7.071067812e-01f, -8.314696123e-01f, -9.238795325e-01f, -9.807852804e-01f,
                                   -1.000000000e+00f, -9.807852804e-01f, -9.238795325e-01f, -8.314696123e-01f,
                                   -7.071067812e-01f, -5.555702330e-01f, -3.826834324e-01f, -1.950903220e-01f};
};

// o * W_N^k (conjugate twiddle for the inverse); k is a compile-time
// constant after unrolling, so the trivial twiddles fold away
template <int N, bool INV>
__host__ __device__ __forceinline__ float2 twiddle(float2 o, int k) {
  if (k == 0) return o;
  if (4 * k == N) return INV ? make_float2(-o.y, o.x) : make_float2(o.y, -o.x);  // +-i
  const int s = k * (32 / N);
  const float wr = Tw32::re[s], wi = INV ? -Tw32::im[s] : Tw32::im[s];
  return make_float2(o.x * wr - o.y * wi, o.x * wi + o.y * wr);
}

// in-register DFT of length N (natural order in and out), radix-2
// decimation in time; N <= 32
template <int N, bool INV>
struct Dft {
  __host__ __device__ static __forceinline__ void run(float2* x) {
    float2 e[N / 2], o[N / 2];
#pragma unroll
    for (int i = 0; i < N / 2; ++i) {
      e[i] = x[2 * i];
      o[i] = x[2 * i + 1];
    }
    Dft<N / 2, INV>::run(e);
    Dft<N / 2, INV>::run(o);
#pragma unroll
    for (int k = 0; k < N / 2; ++k) {
      float2 t = twiddle<N, INV>(o[k], k);
      x[k] = cadd(e[k], t);
      x[k + N / 2] = csub(e[k], t);
    }
  }
};
template <bool INV>
struct Dft<1, INV> {
  __host__ __device__ static __forceinline__ void run(float2*) {}
};

// column passes: C columns per block, lanes run over columns first so that a
// wave reads C consecutive complex values of several rows
template <int L_, int C>
struct Shape {
  static constexpr int L = L_;
  static constexpr int P = 256 / C;   // threads per column
  static constexpr int E = L / P;     // elements per thread
  static constexpr int J = E / P;     // pass-B DFTs per thread
  static constexpr int PAD = 16;      // float2 of padding per k2 block (LDS banks)
  static constexpr int KS = P * C + PAD;
  static constexpr int LDS = (E * KS > L * C) ? E * KS : L * C;  // float2
  static_assert(P * C == 256, "256 threads per block");
  static_assert(E >= P && E % P == 0 && E <= 32 && P <= 32, "shape");
  __host__ __device__ static int lane_c(int tid) { return tid % C; }
  __host__ __device__ static int lane_n1(int tid) { return tid / C; }
  __host__ __device__ static int y_idx(int k2, int n1, int c) { return k2 * KS + n1 * C + c; }
  __host__ __device__ static int nat_idx(int t, int c) { return t * C + c; }
  __host__ __device__ static int t_in(int n1, int r) { return n1 + P * r; }
  __host__ __device__ static int t_out(int n1, int r) { return (n1 + (r / P) * P) + E * (r % P); }
};

// row passes: R contiguous rows per block of NT threads, lanes run along the
// row first so that a wave reads P consecutive values of each of 64 / P rows
template <int L_, int P_, int NT = 256>
struct RowShape {
  static constexpr int L = L_;
  static constexpr int P = P_;
  static constexpr int R = NT / P;    // rows per block
  static constexpr int E = L / P;
  static constexpr int J = E / P;
  static constexpr int PAD = 16;
  static constexpr int KS = P * R + PAD;
  static constexpr int RS = L + 1;    // natural row stride in LDS
  static constexpr int LDS = (E * KS > R * RS) ? E * KS : R * RS;
  static_assert(P * R == NT && NT % 64 == 0, "whole waves of whole rows");
  static_assert(E >= P && E % P == 0 && E <= 32 && P <= 32, "shape");
  __host__ __device__ static int lane_c(int tid) { return tid / P; }
  __host__ __device__ static int lane_n1(int tid) { return tid % P; }
  __host__ __device__ static int y_idx(int k2, int n1, int c) { return k2 * KS + c * P + n1; }
  __host__ __device__ static int nat_idx(int t, int c) { return c * RS + t; }
  __host__ __device__ static int t_in(int n1, int r) { return n1 + P * r; }
  __host__ __device__ static int t_out(int n1, int r) { return (n1 + (r / P) * P) + E * (r % P); }
};

// pass A in registers: DFT over n2, then the twiddle W_L^(n1 k2) from the
// table tw[t] = exp(-2 pi i t / Lmax), read with stride tws = Lmax / L
template <class S, bool INV>
__host__ __device__ __forceinline__ void pass_a(float2* v, int n1, const float2* tw, int tws) {
  Dft<S::E, INV>::run(v);
#pragma unroll
  for (int k2 = 1; k2 < S::E; ++k2) {
    float2 w = tw[(n1 * k2) * tws];  // n1 k2 < L
    if (INV) w.y = -w.y;
    v[k2] = cmulw(v[k2], w);
  }
}

template <class S>
__host__ __device__ __forceinline__ void store_y(const float2* v, float2* lds, int n1, int c) {
#pragma unroll
  for (int k2 = 0; k2 < S::E; ++k2) lds[S::y_idx(k2, n1, c)] = v[k2];
}

// pass B: P-point DFTs over n1 for k2 = n1 + j P; output layout
template <class S, bool INV>
__host__ __device__ __forceinline__ void pass_b(float2* v, const float2* lds, int n1, int c) {
#pragma unroll
  for (int j = 0; j < S::J; ++j) {
    const int k2 = n1 + j * S::P;
    float2 u[S::P];
#pragma unroll
    for (int m = 0; m < S::P; ++m) u[m] = lds[S::y_idx(k2, m, c)];
    Dft<S::P, INV>::run(u);
#pragma unroll
    for (int k1 = 0; k1 < S::P; ++k1) v[j * S::P + k1] = u[k1];
  }
}

// output layout -> natural order in LDS -> input layout (to chain a second
// transform on the same columns)
template <class S>
__host__ __device__ __forceinline__ void store_nat_out(const float2* v, float2* lds, int n1, int c) {
#pragma unroll
  for (int r = 0; r < S::E; ++r) lds[S::nat_idx(S::t_out(n1, r), c)] = v[r];
}
template <class S>
__host__ __device__ __forceinline__ void load_nat_in(float2* v, const float2* lds, int n1, int c) {
#pragma unroll
  for (int r = 0; r < S::E; ++r) v[r] = lds[S::nat_idx(S::t_in(n1, r), c)];
}

}  // namespace freg
}  // namespace pm
