// Particle <-> mesh kernels for gfx950: deterministic fixed-point deposit,
// force gather fused with the kick and drift, and the adjoint kernels.
//
// Mass assignment follows tab. interpolation_kernels (CIC, TSC; the 3D kernel
// is the product of 1D kernels).  Positions enter as an integer mesh
// coordinate U = j r 2^20 + rne(Psi r 2^20) (mod n_g 2^20), exact from the FP32
// displacement Psi because r = n_g/n_p is a power of two.  1D weights are
// integers summing to 2^20; the 3D product is rounded half-to-even to a mass
// unit of 2^32 per particle and the remainder goes to the stencil point with
// the largest exact product (first in x-major order on ties).  Accumulation
// is int64 atomics, so the mesh is bit-identical whatever the atomic order.
//
// The force is A = gather(FD_c phi) with phi the potential mesh: the
// finite-difference gradient of tab. derivative_kernels applied in real space
// equals its Fourier multiplier exactly (the stencils are circular
// convolutions), so one inverse FFT serves all three components.  The gather
// convolves the 1D kernel weights with the FD stencil along the component's
// axis (P + 2h points) and keeps the P-point kernel on the other two axes.
//
// Adjoint (Sec. "Adjoint method", tab. adjoint_dkd; App. "Custom VJP and JVP"):
//   k_adj_kick     reverse kick of the primal, the direct (gather w.r.t.
//                  positions) part of X_bar, scatter of u = beta V_bar onto
//                  three cotangent meshes (gather w.r.t. the mesh), V_bar *= alpha;
//   k_fd_div       d = sum_c FD_c^T g_bar_c on the mesh;
//   k_adj_drift    scatter-w.r.t.-positions part of X_bar from the mesh
//                  cotangent, then the reverse drifts of primal and cotangents.
#include "kernels.h"

namespace pm {

// ------------------------------------------------------------ fixed point

__device__ __forceinline__ long long fixed_coord(long long j, float psi, int log2_r, long long umask) {
  float t = psi * (float)(1 << (log2_r + kFracBits));  // exact power-of-two scaling
  long long f = (long long)rintf(t);                  // round half to even
  return ((j << (log2_r + kFracBits)) + f) & umask;   // mod n_g 2^20
}

__device__ __forceinline__ unsigned long long rne_shift(unsigned long long p, int s) {
  unsigned long long q = p >> s, rem = p & ((1ull << s) - 1), half = 1ull << (s - 1);
  return q + ((rem > half) || (rem == half && (q & 1ull)));
}

// integer 1D weights (sum 2^20), first node i0 (unwrapped), P = 2 or 3 nodes
template <int P>
__device__ __forceinline__ int weights1d(long long U, int w[P]) {
  constexpr long long one = 1ll << kFracBits;
  if constexpr (P == 2) {
    int f = (int)(U & (one - 1));
    w[0] = (int)one - f;
    w[1] = f;
    return (int)(U >> kFracBits);
  } else {
    long long n = (U + (one >> 1)) >> kFracBits;
    long long X = U - (n << kFracBits);
    long long a = (one >> 1) - X, b = (one >> 1) + X;
    int wl = (int)rne_shift((unsigned long long)(a * a), 2 * kFracBits + 1 - kWeightBits);
    int wr = (int)rne_shift((unsigned long long)(b * b), 2 * kFracBits + 1 - kWeightBits);
    w[0] = wl;
    w[1] = (1 << kWeightBits) - wl - wr;
    w[2] = wr;
    return (int)n - 1;
  }
}

// float weights and their derivatives d/du (u in mesh cells)
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
  } else {
    constexpr long long one = 1ll << kFracBits;
    long long n = (U + (one >> 1)) >> kFracBits;
    float x = (float)(U - (n << kFracBits)) * (1.0f / (float)one);
    dw[0] = -(0.5f - x);
    dw[1] = -2.f * x;
    dw[2] = 0.5f + x;
  }
  return i0;
}

struct PartPtrs {
  float* disp;
  float* vel;
  float* xbar;
  float* vbar;
};

__device__ __forceinline__ void lattice_of(long long i, int log2_np, long long j[3]) {
  long long m = (1ll << log2_np) - 1;
  j[2] = i & m;
  j[1] = (i >> log2_np) & m;
  j[0] = i >> (2 * log2_np);
}

// ---------------------------------------------------------------- deposit

template <int P>
__global__ void __launch_bounds__(256) k_deposit(DepositArgs a) {
  const int slot = blockIdx.y;
  if (!((a.active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.N) return;
  const long long ps = slot * a.g.part_stride;
  float px = a.disp[ps + i], py = a.disp[ps + a.g.N + i], pz = a.disp[ps + 2 * a.g.N + i];
  if (a.vel) {  // merged first drift: X += tau V (written back)
    float t = a.tau[slot];
    px += t * a.vel[ps + i];
    py += t * a.vel[ps + a.g.N + i];
    pz += t * a.vel[ps + 2 * a.g.N + i];
    a.disp[ps + i] = px;
    a.disp[ps + a.g.N + i] = py;
    a.disp[ps + 2 * a.g.N + i] = pz;
  }
  long long j[3];
  lattice_of(i, a.g.log2_np, j);
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
  int wx[P], wy[P], wz[P];
  int ix = weights1d<P>(fixed_coord(j[0], px, a.g.log2_r, umask), wx);
  int iy = weights1d<P>(fixed_coord(j[1], py, a.g.log2_r, umask), wy);
  int iz = weights1d<P>(fixed_coord(j[2], pz, a.g.log2_r, umask), wz);
  constexpr int shift = 3 * kWeightBits - kMassBits;
  // pass 1: sum of rounded weights and the home point (largest exact product)
  unsigned long long sum = 0, best = 0;
  int home = 0;
#pragma unroll
  for (int x = 0; x < P; ++x)
#pragma unroll
    for (int y = 0; y < P; ++y) {
      unsigned long long wxy = (unsigned long long)wx[x] * (unsigned)wy[y];
#pragma unroll
      for (int z = 0; z < P; ++z) {
        unsigned long long p = wxy * (unsigned)wz[z];
        sum += rne_shift(p, shift);
        if (p > best) { best = p; home = (x * P + y) * P + z; }
      }
    }
  const long long rem = (1ll << kMassBits) - (long long)sum;
  const int nm = a.g.n_g - 1;
  unsigned long long* mesh = reinterpret_cast<unsigned long long*>(a.mesh) + slot * a.g.mesh_stride;
#pragma unroll
  for (int x = 0; x < P; ++x) {
    long long bx = (long long)((ix + x) & nm) << (2 * a.g.log2_ng);
#pragma unroll
    for (int y = 0; y < P; ++y) {
      long long bxy = bx + ((long long)((iy + y) & nm) << a.g.log2_ng);
      unsigned long long wxy = (unsigned long long)wx[x] * (unsigned)wy[y];
#pragma unroll
      for (int z = 0; z < P; ++z) {
        long long w = (long long)rne_shift(wxy * (unsigned)wz[z], shift);
        if ((x * P + y) * P + z == home) w += rem;
        if (w) atomicAdd(mesh + bxy + ((iz + z) & nm), (unsigned long long)w);
      }
    }
  }
}

// ------------------------------------------------------ FD-gradient gather

// finite-difference stencil c_s, s = -H..H, of d/dx (tab. derivative_kernels)
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

// A_c = sum_j W_j (FD_c phi)_j and, when GRAD, dA_c/du_a (a = 0..2).
// The c-axis weights are the kernel convolved with the stencil (P + 2H points).
template <int P, int ORD, bool GRAD>
__device__ __forceinline__ void fd_gather(const float* __restrict__ phi, int log2n, const int i0[3],
                                          const float w[3][P], const float dw[3][P], float A[3],
                                          float dA[3][3]) {
  constexpr int H = ORD / 2;
  constexpr int Q = P + 2 * H;
  const int nm = (1 << log2n) - 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float G[Q], dG[Q];
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      float g = 0.f, d = 0.f;
#pragma unroll
      for (int q = 0; q < P; ++q) {
        int s = t - H - q;  // node q + s = t - H relative to i0
        if (s >= -H && s <= H) {
          float cs = fd_coef<ORD>(s);
          g += w[c][q] * cs;
          d += dw[c][q] * cs;
        }
      }
      G[t] = g;
      dG[t] = d;
    }
    // the other two axes
    const int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    float acc = 0.f, d_c = 0.f, d_1 = 0.f, d_2 = 0.f;
#pragma unroll
    for (int t = 0; t < Q; ++t) {
      int ic = (i0[c] - H + t) & nm;
#pragma unroll
      for (int q1 = 0; q1 < P; ++q1) {
        int j1 = (i0[a1] + q1) & nm;
#pragma unroll
        for (int q2 = 0; q2 < P; ++q2) {
          int j2 = (i0[a2] + q2) & nm;
          int idx3[3];
          idx3[c] = ic;
          idx3[a1] = j1;
          idx3[a2] = j2;
          float f = phi[((long long)((idx3[0] << log2n) + idx3[1]) << log2n) + idx3[2]];
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

template <int P>
__device__ __forceinline__ void particle_weights(const GatherArgs& a, int slot, long long i, float p[3],
                                                 int i0[3], float w[3][P], float dw[3][P]) {
  long long j[3];
  lattice_of(i, a.g.log2_np, j);
  const long long umask = (1ll << (a.g.log2_ng + kFracBits)) - 1;
#pragma unroll
  for (int c = 0; c < 3; ++c) i0[c] = weights1d_f<P>(fixed_coord(j[c], p[c], a.g.log2_r, umask), w[c], dw[c]);
}

// forward: A = gather(FD phi); V = alpha V + beta A; X += tau_post V
template <int P, int ORD>
__global__ void __launch_bounds__(256) k_gather_kick(GatherArgs a) {
  const int slot = blockIdx.y;
  if (!((a.active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.N) return;
  const long long ps = slot * a.g.part_stride;
  const long long N = a.g.N;
  float p[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
  int i0[3];
  float w[3][P], dw[3][P];
  particle_weights<P>(a, slot, i, p, i0, w, dw);
  float A[3], dA[3][3];
  fd_gather<P, ORD, false>(a.phi + slot * a.g.mesh_stride, a.g.log2_ng, i0, w, dw, A, dA);
  if (a.acc_out) {  // force only (test hook)
#pragma unroll
    for (int c = 0; c < 3; ++c) a.acc_out[ps + c * N + i] = A[c];
    return;
  }
  const float al = a.alpha[slot], be = a.beta[slot], tp = a.tau[slot];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float v = al * a.vel[ps + c * N + i] + be * A[c];
    a.vel[ps + c * N + i] = v;
    a.disp[ps + c * N + i] = p[c] + tp * v;
  }
}

// adjoint kick at X^{n-1/2} (disp), with phi of that position:
//   V^{n-1} = (V^n - beta A) / alpha
//   X_bar  += r sum_c u_c dA_c/du,  u = beta V_bar
//   g_bar_c += scatter(u_c)
//   V_bar  *= alpha
template <int P, int ORD>
__global__ void __launch_bounds__(256) k_adj_kick(GatherArgs a) {
  const int slot = blockIdx.y;
  if (!((a.active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.N) return;
  const long long ps = slot * a.g.part_stride;
  const long long N = a.g.N;
  float p[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
  int i0[3];
  float w[3][P], dw[3][P];
  particle_weights<P>(a, slot, i, p, i0, w, dw);
  float A[3], dA[3][3];
  fd_gather<P, ORD, true>(a.phi + slot * a.g.mesh_stride, a.g.log2_ng, i0, w, dw, A, dA);
  const float al = a.alpha[slot], be = a.beta[slot];
  const float r = (float)(1 << a.g.log2_r);
  float u[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float vb = a.vbar[ps + c * N + i];
    u[c] = be * vb;
    a.vel[ps + c * N + i] = (a.vel[ps + c * N + i] - be * A[c]) / al;
    a.vbar[ps + c * N + i] = al * vb;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    float g = u[0] * dA[0][d] + u[1] * dA[1][d] + u[2] * dA[2][d];
    a.xbar[ps + d * N + i] += r * g;
  }
  // gather w.r.t. the mesh: scatter u_c with the kernel weights
  const int nm = a.g.n_g - 1;
  float* gb = a.gbar + slot * a.g.mesh_stride * 3;
#pragma unroll
  for (int x = 0; x < P; ++x)
#pragma unroll
    for (int y = 0; y < P; ++y) {
      long long bxy = ((long long)(((i0[0] + x) & nm) << a.g.log2_ng) + ((i0[1] + y) & nm)) << a.g.log2_ng;
      float wxy = w[0][x] * w[1][y];
#pragma unroll
      for (int z = 0; z < P; ++z) {
        long long idx = bxy + ((i0[2] + z) & nm);
        float wt = wxy * w[2][z];
        atomicAdd(gb + idx, wt * u[0]);
        atomicAdd(gb + a.g.mesh_stride + idx, wt * u[1]);
        atomicAdd(gb + 2 * a.g.mesh_stride + idx, wt * u[2]);
      }
    }
}

// d = sum_c FD_c^T g_bar_c = -sum_c sum_s c_s g_bar_c(x + s e_c)
template <int ORD>
__global__ void __launch_bounds__(256) k_fd_div(const float* __restrict__ gbar, float* __restrict__ d,
                                                Geom g, unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= g.M) return;
  constexpr int H = ORD / 2;
  const int n = g.n_g, nm = n - 1, L = g.log2_ng;
  int z = (int)(e & nm), y = (int)((e >> L) & nm), x = (int)(e >> (2 * L));
  const float* g0 = gbar + slot * g.mesh_stride * 3;
  float acc = 0.f;
#pragma unroll
  for (int s = -H; s <= H; ++s) {
    if (s == 0) continue;
    float cs = fd_coef<ORD>(s);
    long long ix = ((long long)(((x + s) & nm) << L) + y) << L | z;
    long long iy = ((long long)((x << L) + ((y + s) & nm)) << L) | z;
    long long iz = ((long long)((x << L) + y) << L) | ((z + s) & nm);
    acc += cs * (g0[ix] + g0[g.mesh_stride + iy] + g0[2 * g.mesh_stride + iz]);
  }
  d[slot * g.mesh_stride + e] = -acc;
}

// scatter w.r.t. positions: X_bar += coef r sum_j rho_bar_j dW_j/du, then the
// reverse drift X -= tau V, V_bar += tau X_bar (tau may merge two drifts)
template <int P>
__global__ void __launch_bounds__(256) k_adj_drift(GatherArgs a) {
  const int slot = blockIdx.y;
  if (!((a.active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.g.N) return;
  const long long ps = slot * a.g.part_stride;
  const long long N = a.g.N;
  float p[3] = {a.disp[ps + i], a.disp[ps + N + i], a.disp[ps + 2 * N + i]};
  float xb[3] = {a.xbar[ps + i], a.xbar[ps + N + i], a.xbar[ps + 2 * N + i]};
  if (a.phi) {
    int i0[3];
    float w[3][P], dw[3][P];
    particle_weights<P>(a, slot, i, p, i0, w, dw);
    const int nm = a.g.n_g - 1;
    const float* rb = a.phi + slot * a.g.mesh_stride;
    float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
    for (int x = 0; x < P; ++x)
#pragma unroll
      for (int y = 0; y < P; ++y) {
        long long bxy = ((long long)(((i0[0] + x) & nm) << a.g.log2_ng) + ((i0[1] + y) & nm)) << a.g.log2_ng;
#pragma unroll
        for (int z = 0; z < P; ++z) {
          float f = rb[bxy + ((i0[2] + z) & nm)];
          gx += f * dw[0][x] * w[1][y] * w[2][z];
          gy += f * w[0][x] * dw[1][y] * w[2][z];
          gz += f * w[0][x] * w[1][y] * dw[2][z];
        }
      }
    const float cf = a.coef[slot] * (float)(1 << a.g.log2_r);
    xb[0] += cf * gx;
    xb[1] += cf * gy;
    xb[2] += cf * gz;
  }
  const float t = a.tau[slot];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float v = a.vel[ps + c * N + i];
    a.disp[ps + c * N + i] = p[c] - t * v;
    a.xbar[ps + c * N + i] = xb[c];
    a.vbar[ps + c * N + i] += t * xb[c];
  }
}

// ------------------------------------------------------- dispatch helpers

template <int P>
static hipError_t gather_dispatch(const GatherArgs& a, int kind, int order, hipStream_t s) {
  dim3 grid((unsigned)((a.g.N + 255) / 256), a.batch);
  switch (kind) {
    case GK_KICK:
      if (order == 2) k_gather_kick<P, 2><<<grid, 256, 0, s>>>(a);
      else if (order == 4) k_gather_kick<P, 4><<<grid, 256, 0, s>>>(a);
      else k_gather_kick<P, 6><<<grid, 256, 0, s>>>(a);
      break;
    case GK_ADJ_KICK:
      if (order == 2) k_adj_kick<P, 2><<<grid, 256, 0, s>>>(a);
      else if (order == 4) k_adj_kick<P, 4><<<grid, 256, 0, s>>>(a);
      else k_adj_kick<P, 6><<<grid, 256, 0, s>>>(a);
      break;
    case GK_ADJ_DRIFT: k_adj_drift<P><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, int kind, int mak, int order, hipStream_t s) {
  return mak == 2 ? gather_dispatch<2>(a, kind, order, s) : gather_dispatch<3>(a, kind, order, s);
}

hipError_t launch_deposit(const DepositArgs& a, int mak, hipStream_t s) {
  dim3 grid((unsigned)((a.g.N + 255) / 256), a.batch);
  if (mak == 2) k_deposit<2><<<grid, 256, 0, s>>>(a);
  else k_deposit<3><<<grid, 256, 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_fd_div(const float* gbar, float* d, const Geom& g, int batch, int order,
                         unsigned long long active, hipStream_t s) {
  dim3 grid((unsigned)((g.M + 255) / 256), batch);
  if (order == 2) k_fd_div<2><<<grid, 256, 0, s>>>(gbar, d, g, active);
  else if (order == 4) k_fd_div<4><<<grid, 256, 0, s>>>(gbar, d, g, active);
  else k_fd_div<6><<<grid, 256, 0, s>>>(gbar, d, g, active);
  return hipGetLastError();
}

}  // namespace pm
