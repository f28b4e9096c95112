// Device helpers of the mass-assignment kernels (tab. interpolation_kernels):
// fixed-point mesh coordinates, integer 1D weights, their float values and
// derivatives, and the finite-difference gradient stencils of
// tab. derivative_kernels.
#pragma once
#include "kernels.h"

namespace pm {

// U = j r 2^20 + rne(Psi r 2^20) mod n_g 2^20; exact from FP32 Psi (r = 2^k)
__device__ __forceinline__ long long fixed_coord(long long j, float psi, int log2_r, long long umask) {
  float t = psi * (float)(1 << (log2_r + kFracBits));
  long long f = (long long)rintf(t);  // round half to even
  return ((j << (log2_r + kFracBits)) + f) & umask;
}

__device__ __forceinline__ unsigned long long rne_shift(unsigned long long p, int s) {
  unsigned long long q = p >> s, rem = p & ((1ull << s) - 1), half = 1ull << (s - 1);
  return q + ((rem > half) || (rem == half && (q & 1ull)));
}

// home node of a particle on one axis (wrapped): CIC and PCS floor(u), TSC
// round(u); the stencil runs from home + first_node to home + first_node + P - 1
// and reaches kernel_reach nodes from the home node on either side
template <int P>
__device__ __forceinline__ int home_node(long long U, int nm) {
  if constexpr (P == 2 || P == 4) return (int)(U >> kFracBits) & nm;
  else return (int)((U + (1ll << (kFracBits - 1))) >> kFracBits) & nm;
}
template <int P>
constexpr int first_node() { return P == 2 ? 0 : -1; }
template <int P>
constexpr int kernel_reach() { return P == 4 ? 2 : 1; }

// round-half-even of p / d for a compile-time divisor (the PCS weights)
template <unsigned long long D>
__device__ __forceinline__ unsigned long long rne_div(unsigned long long p) {
  const unsigned long long q = p / D, rem = p - q * D;
  return q + ((2 * rem > D) || (2 * rem == D && (q & 1ull)));
}

// integer 1D weights (sum 2^20); returns the first node, unwrapped
template <int P>
__device__ __forceinline__ int weights1d(long long U, int w[P]) {
  constexpr long long one = 1ll << kFracBits;
  if constexpr (P == 2) {
    int f = (int)(U & (one - 1));
    w[0] = (int)one - f;
    w[1] = f;
    return (int)(U >> kFracBits);
  } else if constexpr (P == 3) {
    long long n = (U + (one >> 1)) >> kFracBits;
    long long X = U - (n << kFracBits);
    long long a = (one >> 1) - X, b = (one >> 1) + X;
    int wl = (int)rne_shift((unsigned long long)(a * a), 2 * kFracBits + 1 - kWeightBits);
    int wr = (int)rne_shift((unsigned long long)(b * b), 2 * kFracBits + 1 - kWeightBits);
    w[0] = wl;
    w[1] = (1 << kWeightBits) - wl - wr;
    w[2] = wr;
    return (int)n - 1;
  } else {
    // PCS (cubic B-spline) at F = frac(u) 2^20, G = 2^20 - F: G^3/6, F^3/6 and
    // (4 - 6f^2 + 3f^3)/6 rounded half-even from exact integers, the
    // remaining node takes the rest of 2^20
    static_assert(P == 4 && kWeightBits == kFracBits, "PCS weights in the position's fixed point");
    const unsigned long long F = (unsigned long long)(U & (one - 1)), G = (unsigned long long)one - F;
    constexpr unsigned long long D = 6ull << (2 * kFracBits);
    const int wa = (int)rne_div<D>(G * G * G);
    const int wd = (int)rne_div<D>(F * F * F);
    const int wb = (int)rne_div<D>((4ull << (3 * kFracBits)) + 3 * F * F * F - 6 * F * F * (unsigned long long)one);
    w[0] = wa;
    w[1] = wb;
    w[2] = (1 << kWeightBits) - wa - wb - wd;
    w[3] = wd;
    return (int)(U >> kFracBits) - 1;
  }
}

// float weights and d/du (u in mesh cells)
template <int P>
__device__ __forceinline__ int weights1d_f(long long U, float w[P], float dw[P]) {
  int wi[P];
  int i0 = weights1d<P>(U, wi);
  constexpr float inv = 1.0f / (float)(1 << kWeightBits);
#pragma unroll
  for (int a = 0; a < P; ++a) w[a] = (float)wi[a] * inv;
  if constexpr (P == 2) {
    dw[0] = -1.f;
    dw[1] = 1.f;
  } else if constexpr (P == 3) {
    constexpr long long one = 1ll << kFracBits;
    long long n = (U + (one >> 1)) >> kFracBits;
    float x = (float)(U - (n << kFracBits)) * (1.0f / (float)one);
    dw[0] = -(0.5f - x);
    dw[1] = -2.f * x;
    dw[2] = 0.5f + x;
  } else {
    // d/du of the PCS weights at f = frac(u), g = 1 - f
    constexpr long long one = 1ll << kFracBits;
    const float f = (float)(U & (one - 1)) * (1.0f / (float)one), g = 1.f - f;
    dw[0] = -0.5f * g * g;
    dw[1] = f * (1.5f * f - 2.f);
    dw[2] = g * (2.f - 1.5f * g);
    dw[3] = 0.5f * f * f;
  }
  return i0;
}

// Particle storage order: the lattice is cut into blocks of B = 2^b sites per
// axis (B^3 consecutive particles, z fastest inside a block, blocks in x-major
// order).  With B = tile edge / (n_g / n_p) an unperturbed block fills exactly
// one mesh tile, so the particles of a tile are a contiguous run.  b = log2
// n_p is plain row-major order.
__device__ __forceinline__ void lattice_of(long long i, int log2_np, int b, long long j[3]) {
  const int nb = log2_np - b;
  const long long bm = (1ll << b) - 1, nm = (1ll << nb) - 1;
  const long long loc = i & ((1ll << (3 * b)) - 1), blk = i >> (3 * b);
  j[2] = ((blk & nm) << b) | (loc & bm);
  j[1] = (((blk >> nb) & nm) << b) | ((loc >> b) & bm);
  j[0] = ((blk >> (2 * nb)) << b) | (loc >> (2 * b));
}

__host__ __device__ __forceinline__ long long blocked_index(long long x, long long y, long long z, int log2_np, int b) {
  const int nb = log2_np - b;
  const long long bm = (1ll << b) - 1;
  const long long blk = (((x >> b) << nb | (y >> b)) << nb) | (z >> b);
  return (blk << (3 * b)) | ((((x & bm) << b) | (y & bm)) << b) | (z & bm);
}

// finite-difference stencil c_s (s = -H..H) of d/dx
template <int ORD>
__device__ __forceinline__ float fd_coef(int s) {
  if constexpr (ORD == 2) {
    return s == 1 ? 0.5f : (s == -1 ? -0.5f : 0.f);
  } else if constexpr (ORD == 4) {
    const float c[5] = {1.f / 12, -8.f / 12, 0.f, 8.f / 12, -1.f / 12};
    return c[s + 2];
  } else {
    const float c[7] = {-1.f / 60, 9.f / 60, -45.f / 60, 0.f, 45.f / 60, -9.f / 60, 1.f / 60};
    return c[s + 3];
  }
}

// A_c = sum_j W_j (FD_c phi)_j and, when GRAD, dA_c/du_a, for a particle with
// P-point kernels starting at node i0 (per axis); `at(x, y, z)` loads phi at
// node offsets (which may run H below i0 and P-1+H above).  The c-axis
// weights are the kernel convolved with the stencil (P + 2H points).
template <int P, int ORD, bool GRAD, class Acc>
__device__ __forceinline__ void fd_gather(const Acc& at, const int i0[3], const float w[3][P],
                                          const float dw[3][P], float A[3], float dA[3][3]) {
  constexpr int H = ORD / 2;
  constexpr int Q = P + 2 * H;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float G[Q], dG[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      float g = 0.f, d = 0.f;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        int s = t - H - q;
        if (s >= -H && s <= H) {
          float cs = fd_coef<ORD>(s);
          g += w[c][q] * cs;
          d += dw[c][q] * cs;
        }
      }
      G[t] = g;
      dG[t] = d;
    }
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    float acc = 0.f, d_c = 0.f, d_1 = 0.f, d_2 = 0.f;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
#pragma unroll
      for (int q1 = 0; q1 < P; ++q1) {
#pragma unroll
        for (int q2 = 0; q2 < P; ++q2) {
          int o[3];
          o[c] = i0[c] - H + t;
          o[a1] = i0[a1] + q1;
          o[a2] = i0[a2] + q2;
          float f = at(o[0], o[1], o[2]);
          float w12 = w[a1][q1] * w[a2][q2];
          acc += G[t] * w12 * f;
          if constexpr (GRAD) {
            d_c += dG[t] * w12 * f;
            d_1 += G[t] * dw[a1][q1] * w[a2][q2] * f;
            d_2 += G[t] * w[a1][q1] * dw[a2][q2] * f;
          }
        }
      }
    }
    A[c] = acc;
    if constexpr (GRAD) {
      dA[c][c] = d_c;
      dA[c][a1] = d_1;
      dA[c][a2] = d_2;
    }
  }
}

}  // namespace pm
