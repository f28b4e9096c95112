// 3D real FFT for cubic power-of-two meshes, written for gfx950 (64-wide
// waves, 160 KB LDS per CU).
//
// Layout: real mesh [n][n][n] (z fastest); half spectrum [n][n][rs] of float2
// (modes m_x, m_y in FFT order, m_z = 0..n/2, rows padded to rs >= n/2+1).
// The forward transform is sum_j f_j exp(-2 pi i m.j/n), the inverse
// sum_m F_m exp(+2 pi i m.j/n), both unnormalised.  A 3D transform is three
// HBM passes:
//   z rows   real <-> complex via a half-length complex FFT (the two real
//            halves packed as one complex row);
//   y and x  strided complex passes over tiles of C consecutive z columns
//            (C float2 = 128 B contiguous per row at C = 16).
// Every line transform is held in registers with a four-step split and one
// LDS exchange (fft_reg.h); only the column passes of meshes below n = 16
// use the LDS Stockham radix-4/2 transform (lds_fft).  Twiddles come from one
// table tw[t] = exp(-2 pi i t / Lmax) built in FP64 on the host.
// The PM multiplier (Green's function, deconvolution, normalisation) is fused
// into the x pass: forward x FFT, multiply, inverse x FFT, one HBM round trip
// (Sec. "Force evaluation"; the Poisson solve in Fourier space).
#include "fft.h"
#include "fft_reg.h"
#include "mak.h"
#include "xcd.h"

namespace pm {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Stockham radix-4/2 FFT of C lines of length L in LDS.
// LINE_FAST: element (t, l) at buf[t*C + l] (strided passes), else at
// buf[l*(L+1) + t] (row passes).  tw[e*tws] = exp(-2 pi i e / L).
template <int L, int C, bool LINE_FAST, int NT>
__device__ __forceinline__ void lds_fft(float2* __restrict__ buf, const float2* __restrict__ tw,
                                        int tws, bool inverse) {
  const int tid = threadIdx.x;
  auto at = [](int t, int l) { return LINE_FAST ? t * C + l : l * (L + 1) + t; };
  int Ns = 1;
  if constexpr (L >= 4) {
    constexpr int B4 = (L / 4) * C;
    constexpr int PT = (B4 + NT - 1) / NT;
#pragma unroll 1
    for (; Ns * 4 <= L; Ns *= 4) {
      float2 v[PT][4];
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        int b = tid + p * NT;
        if (b < B4) {
          int j = LINE_FAST ? b / C : b % (L / 4);
          int l = LINE_FAST ? b % C : b / (L / 4);
#pragma unroll
          for (int r = 0; r < 4; ++r) v[p][r] = buf[at(j + r * (L / 4), l)];
        }
      }
      __syncthreads();
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        int b = tid + p * NT;
        if (b < B4) {
          int j = LINE_FAST ? b / C : b % (L / 4);
          int l = LINE_FAST ? b % C : b / (L / 4);
          int k = j & (Ns - 1);
          int e = k * (L / (4 * Ns));
#pragma unroll
          for (int r = 1; r < 4; ++r) {
            float2 w = tw[(r * e) * tws];
            if (inverse) w.y = -w.y;
            v[p][r] = cmul(v[p][r], w);
          }
          float2 t0 = make_float2(v[p][0].x + v[p][2].x, v[p][0].y + v[p][2].y);
          float2 t1 = make_float2(v[p][0].x - v[p][2].x, v[p][0].y - v[p][2].y);
          float2 t2 = make_float2(v[p][1].x + v[p][3].x, v[p][1].y + v[p][3].y);
          float2 t3 = make_float2(v[p][1].x - v[p][3].x, v[p][1].y - v[p][3].y);
          // forward: y1 = t1 - i t3, y3 = t1 + i t3 (inverse swaps them)
          float2 m3 = inverse ? make_float2(-t3.y, t3.x) : make_float2(t3.y, -t3.x);
          int base = (j - k) * 4 + k;
          buf[at(base, l)] = make_float2(t0.x + t2.x, t0.y + t2.y);
          buf[at(base + Ns, l)] = make_float2(t1.x + m3.x, t1.y + m3.y);
          buf[at(base + 2 * Ns, l)] = make_float2(t0.x - t2.x, t0.y - t2.y);
          buf[at(base + 3 * Ns, l)] = make_float2(t1.x - m3.x, t1.y - m3.y);
        }
      }
      __syncthreads();
    }
  }
  if (Ns < L) {  // one radix-2 stage
    constexpr int B2 = (L / 2) * C;
    constexpr int PT = (B2 + NT - 1) / NT;
    float2 v[PT][2];
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      int b = tid + p * NT;
      if (b < B2) {
        int j = LINE_FAST ? b / C : b % (L / 2);
        int l = LINE_FAST ? b % C : b / (L / 2);
        v[p][0] = buf[at(j, l)];
        v[p][1] = buf[at(j + L / 2, l)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < PT; ++p) {
      int b = tid + p * NT;
      if (b < B2) {
        int j = LINE_FAST ? b / C : b % (L / 2);
        int l = LINE_FAST ? b % C : b / (L / 2);
        int k = j & (Ns - 1);
        float2 w = tw[(k * (L / (2 * Ns))) * tws];
        if (inverse) w.y = -w.y;
        float2 a1 = cmul(v[p][1], w);
        int base = (j - k) * 2 + k;
        buf[at(base, l)] = make_float2(v[p][0].x + a1.x, v[p][0].y + a1.y);
        buf[at(base + Ns, l)] = make_float2(v[p][0].x - a1.x, v[p][0].y - a1.y);
      }
    }
    __syncthreads();
  }
}

// --------------------------------------------------------- column passes

__device__ __forceinline__ int signed_mode(int i, int n) { return i < n / 2 ? i : i - n; }

// the PM multiplier's per-slot coefficient (from the device schedule in
// device-indexed steps)
__device__ __forceinline__ float fused_coef(const ColArgs& a, int slot) {
  return slot_f(a.gate, a.sched, a.sched_steps, a.coef, slot, kSchCoef);
}

template <int L, int C, int MODE>
__global__ void __launch_bounds__(256) k_cols(ColArgs a) {
  __shared__ float2 buf[L * C];
  const int slot = blockIdx.z;
  if (!slot_on(a.gate, a.active, slot)) return;
  const int outer = blockIdx.y;          // x for the y pass, y for the x pass
  const int z0 = blockIdx.x * C;
  const long long stride_t = a.axis == 1 ? (long long)a.rs : (long long)a.n * a.rs;
  const long long base0 = a.axis == 1 ? (long long)outer * a.n * a.rs : (long long)outer * a.rs;
  const long long sbase = slot * a.slot_stride + base0 + z0;
  for (int e = threadIdx.x; e < L * C; e += 256) {
    int t = e / C, c = e - t * C;
    float2 v = make_float2(0.f, 0.f);
    if (z0 + c < a.nh) {
      long long gi = sbase + t * stride_t + c;
      if constexpr (MODE == MODE_COMBINE_IC) {
        // x pass: t = ix, outer = iy, z = z0 + c: sum_c conj(h_c) S_c
        int mz = z0 + c, mx = signed_mode(t, a.n), my = signed_mode(outer, a.n);
        float amp = a.amp[mx * mx + my * my + mz * mz] * a.fac[slot];
        int ms[3] = {mx, my, mz};
        const float2* s3 = a.src3 + slot * a.slot_stride + base0 + z0 + t * stride_t + c;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (ms[q] == -a.n / 2 || ms[q] == a.n / 2) continue;
          float2 s = s3[q * a.comp_stride];
          float h = amp * ms[q];     // h_c = i h, conj(h_c) s = -i h s
          v.x += h * s.y;
          v.y -= h * s.x;
        }
      } else {
        v = a.data[gi];
      }
      if constexpr (MODE == MODE_NUFFT_C) {
        // x pass: t = ix, outer = iy, z = z0 + c
        int iz = z0 + c;
        float dec = a.esdec[t] * a.esdec[outer] * a.esdec[iz];
        int ms[3] = {signed_mode(t, a.n), signed_mode(outer, a.n), iz};
        float th2 = 0.f;
        const float k0 = 6.283185307179586f / (float)a.n_p;
#pragma unroll
        for (int q = 0; q < 3; ++q) th2 += (k0 * ms[q]) * (k0 * ms[q]);
        float h = (dec == 0.f || th2 == 0.f) ? 0.f : a.coef[slot] * dec * (k0 * ms[a.comp]) / th2;
        v = make_float2(-h * v.y, h * v.x);  // i h v
      }
      if constexpr (MODE == MODE_IC_C) {
        int mz = z0 + c, mx = signed_mode(t, a.n), my = signed_mode(outer, a.n);
        int ms[3] = {mx, my, mz};
        int mc = ms[a.comp];
        float h = (mc == -a.n / 2 || mc == a.n / 2)
                      ? 0.f
                      : a.amp[mx * mx + my * my + mz * mz] * a.fac[slot] * mc;
        v = make_float2(-h * v.y, h * v.x);  // i h v
      }
    }
    buf[e] = v;
  }
  __syncthreads();
  if constexpr (MODE == MODE_FWD || MODE == MODE_FUSED_H || MODE == MODE_NUFFT_ADJ)
    lds_fft<L, C, true, 256>(buf, a.tw, a.tws, false);
  if constexpr (MODE == MODE_NUFFT_ADJ) {
    // transposed NUFFT multiplier of component comp, conj(i h) = -i h, summed
    // over the components into dst3; the last component also runs the
    // inverse x transform of the sum
    const float k0 = 6.283185307179586f / (float)a.n_p;
    for (int e = threadIdx.x; e < L * C; e += 256) {
      int t = e / C, c = e - t * C;
      int iz = z0 + c;
      if (iz >= a.nh) continue;
      float dec = a.esdec[t] * a.esdec[outer] * a.esdec[iz];
      int ms[3] = {signed_mode(t, a.n), signed_mode(outer, a.n), iz};
      float th2 = 0.f;
#pragma unroll
      for (int q = 0; q < 3; ++q) th2 += (k0 * ms[q]) * (k0 * ms[q]);
      float h = (dec == 0.f || th2 == 0.f) ? 0.f : a.coef[slot] * dec * (k0 * ms[a.comp]) / th2;
      float2 v = buf[e];
      float2 r = make_float2(h * v.y, -h * v.x);  // -i h v
      if (a.comp > 0) {
        float2 acc = a.dst3[sbase + t * stride_t + c];
        r.x += acc.x;
        r.y += acc.y;
      }
      buf[e] = r;
    }
    __syncthreads();
    if (a.comp == 2) lds_fft<L, C, true, 256>(buf, a.tw, a.tws, true);
  }
  if constexpr (MODE == MODE_FUSED_H) {
    for (int e = threadIdx.x; e < L * C; e += 256) {
      int t = e / C, c = e - t * C;
      int iz = z0 + c;
      if (iz >= a.nh) continue;  // padding columns of the last tile
      float l = a.lap[t] + a.lap[outer] + a.lap[iz];
      float w = a.win2[t] * a.win2[outer] * a.win2[iz];
      float h = (t == 0 && outer == 0 && iz == 0) ? 0.f : fused_coef(a, slot) / (l * w);
      buf[e].x *= h;
      buf[e].y *= h;
    }
    __syncthreads();
  }
  if constexpr (MODE != MODE_FWD && MODE != MODE_NUFFT_ADJ) lds_fft<L, C, true, 256>(buf, a.tw, a.tws, true);
  float2* out = (MODE == MODE_IC_C || MODE == MODE_NUFFT_C || MODE == MODE_NUFFT_ADJ || MODE == MODE_LPT_D) ? a.dst3
                                                                                                       : a.data;
  for (int e = threadIdx.x; e < L * C; e += 256) {
    int t = e / C, c = e - t * C;
    if (z0 + c < a.nh) out[sbase + t * stride_t + c] = buf[e];
  }
}

// ------------------------------------------- row passes, register FFT

// Real rows -> half-spectrum rows with the half-length complex transform held
// in registers (fft_reg.h, RowShape).  SRC selects the input conversion:
//   SRC_I64:  (double)m * scale - shift   (int64 fixed-point mass mesh)
//   SRC_F32:  f * (float)scale            (float mesh)
// A block transforms R rows.  The loads are unconditional (rows past the end read the slot's first row,
// which `base` then points at) and such rows are zeroed by a zero scale, not
// by a branch: a load under a per-row branch is waited for inside it, which
// serialises a thread's E round trips.
template <class S, int SRC, int E>
__device__ __forceinline__ void r2c_load(float2 (&v)[E], const void* __restrict__ src, long long base, int n1,
                                         bool valid, double scale, double shift) {
  static_assert(E == S::E, "one row slice per thread");
  if constexpr (SRC == SRC_I64) {
    const double sc = valid ? scale : 0.0, sh = valid ? shift : 0.0;
#pragma unroll
    for (int r = 0; r < S::E; ++r) {  // z[t] = x[2t] + i x[2t+1]
      const longlong2 m =
          *reinterpret_cast<const longlong2*>(reinterpret_cast<const long long*>(src) + base + 2 * S::t_in(n1, r));
      v[r] = make_float2((float)((double)m.x * sc - sh), (float)((double)m.y * sc - sh));
    }
  } else {
    const float sc = valid ? (float)scale : 0.f;
#pragma unroll
    for (int r = 0; r < S::E; ++r) {
      const float2 f = *reinterpret_cast<const float2*>(reinterpret_cast<const float*>(src) + base + 2 * S::t_in(n1, r));
      v[r] = make_float2(f.x * sc, f.y * sc);
    }
  }
}

template <int L, int P, int SRC, int NT>
__global__ void __launch_bounds__(NT, 2) k_r2c_rows_reg(const void* __restrict__ src, long long src_stride,
                                                     float2* __restrict__ dst, long long dst_stride,
                                                     int n_rows, const float2* __restrict__ tw, int tws_half,
                                                     int tws_full, double scale, double shift,
                                                     unsigned long long active, int rs, int kz_lim,
                                                     const int32_t* __restrict__ gate) {
  using S = freg::RowShape<L, P, NT>;
  constexpr int n = 2 * L;
  __shared__ float2 lds[S::LDS];
  const int slot = blockIdx.y;
  if (!slot_on(gate, active, slot)) return;
  const int n1 = S::lane_n1(threadIdx.x), c = S::lane_c(threadIdx.x);
  const long long row = (long long)blockIdx.x * S::R + c;
  const bool valid = row < n_rows;
  const int klim = kz_lim > 0 ? kz_lim : L + 1;
  float2 v[S::E];
  r2c_load<S, SRC>(v, src, slot * src_stride + (valid ? row : 0) * n, n1, valid, scale, shift);
  freg::pass_a<S, false>(v, n1, tw, tws_half);
  freg::store_y<S>(v, lds, n1, c);
  __syncthreads();
  freg::pass_b<S, false>(v, lds, n1, c);
  __syncthreads();
  freg::store_nat_out<S>(v, lds, n1, c);
  __syncthreads();
  if (!valid) return;
  // unpack: X[k] = (Z[k] + conj Z[L-k])/2 + w^k (Z[k] - conj Z[L-k])/(2i)
  const float2* zr = lds + S::nat_idx(0, c);
  float2* out = dst + slot * dst_stride + row * rs;
  for (int k = n1; k <= L / 2; k += P) {
    const int kk = (L - k) & (L - 1);
    const float2 zk = zr[k], zm = zr[kk];
    if (k == 0) {
      out[0] = make_float2(zk.x + zk.y, 0.f);
      if (L < klim) out[L] = make_float2(zk.x - zk.y, 0.f);
      continue;
    }
    if (k >= klim && kk >= klim) continue;
    const float2 fe = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    const float2 fo = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    const float2 wf = cmul(tw[k * tws_full], fo);
    if (k < klim) out[k] = make_float2(fe.x + wf.x, fe.y + wf.y);
    if (kk != k && kk < klim) {
      const float2 wf2 = cmul(tw[(L - k) * tws_full], make_float2(fo.x, -fo.y));
      out[kk] = make_float2(fe.x + wf2.x, -fe.y + wf2.y);
    }
  }
}

// Half-spectrum rows -> real rows (unnormalised inverse), register
// transform.  DST_F32 writes the real row scaled by `scale`; DST_IC writes
// psi = scale * x into vel[c] and D0 * psi into disp[c] (Zel'dovich state).
template <int L, int P, int DST, int NT>
__global__ void __launch_bounds__(NT) k_c2r_rows_reg(const float2* __restrict__ src, long long src_stride,
                                                      float* __restrict__ dst, long long dst_stride,
                                                      float* __restrict__ dst2, int n_rows,
                                                      const float2* __restrict__ tw, int tws_half, int tws_full,
                                                      float scale, float scale2, unsigned long long active,
                                                      int rs, int kz_lim, int log2pb,
                                                      const int32_t* __restrict__ gate) {
  using S = freg::RowShape<L, P, NT>;
  constexpr int n = 2 * L;
  __shared__ float2 lds[S::LDS];
  const int slot = blockIdx.y;
  if (!slot_on(gate, active, slot)) return;
  const int n1 = S::lane_n1(threadIdx.x), c = S::lane_c(threadIdx.x);
  const long long row = (long long)blockIdx.x * S::R + c;
  const bool valid = row < n_rows;
  float2* zr = lds + S::nat_idx(0, c);
  const float2* in = src + slot * src_stride + row * rs;
  // pack: Z[k] = (X[k] + conj X[L-k]) + i e^{+2 pi i k/n} (X[k] - conj X[L-k])
  const int klim = kz_lim > 0 ? kz_lim : L + 1;
  // all of this thread's loads first (k = n1 + P q), then the arithmetic
  constexpr int NK = L / 2 / P + 1;
  float2 xks[NK], xms[NK];
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    const int k = n1 + P * q;
    xks[q] = make_float2(0.f, 0.f);
    xms[q] = xks[q];
    if (valid && k <= L / 2) {
      if (k < klim) xks[q] = in[k];
      if (L - k < klim) xms[q] = in[L - k];
    }
  }
#pragma unroll
  for (int q = 0; q < NK; ++q) {
    const int k = n1 + P * q;
    if (k > L / 2) continue;
    float2 xk = xks[q], xm = xms[q];
    // a real row takes the real parts of its k = 0 and k = n/2 coefficients
    // (zero imaginary parts for a Hermitian spectrum; interlaced grids'
    // phase leaves them nonzero on those planes)
    if (k == 0) xk.y = xm.y = 0.f;
    const float2 a = make_float2(xk.x + xm.x, xk.y - xm.y);
    const float2 d = make_float2(xk.x - xm.x, xk.y + xm.y);
    float2 w = tw[k * tws_full];
    w.y = -w.y;
    const float2 wd = cmul(w, d);
    zr[k] = make_float2(a.x - wd.y, a.y + wd.x);  // k < L here (k <= L / 2)
    if (L - k != k && L - k < L) {
      float2 w2 = tw[(L - k) * tws_full];
      w2.y = -w2.y;
      const float2 wd2 = cmul(w2, make_float2(-d.x, d.y));
      zr[L - k] = make_float2(a.x - wd2.y, -a.y + wd2.x);
    }
  }
  __syncthreads();
  float2 v[S::E];
  freg::load_nat_in<S>(v, lds, n1, c);
  freg::pass_a<S, true>(v, n1, tw, tws_half);
  __syncthreads();
  freg::store_y<S>(v, lds, n1, c);
  __syncthreads();
  freg::pass_b<S, true>(v, lds, n1, c);
  if (!valid) return;
  constexpr int log2n = __builtin_ctz(n);
  if constexpr (DST == DST_IC2) {
    // second-order LPT grid (n = 2 n_p): the lattice points are its even
    // nodes; add scale v to vel and scale2 v to disp (lattice-block order)
    const long long x = row >> log2n, y = row & (n - 1);
    if ((x | y) & 1) return;
#pragma unroll
    for (int r = 0; r < S::E; ++r) {
      const long long gi = slot * dst_stride + blocked_index(x >> 1, y >> 1, S::t_out(n1, r), log2n - 1, log2pb);
      dst[gi] += scale * v[r].x;
      dst2[gi] += scale2 * v[r].x;
    }
    return;
  }
  if constexpr (DST == DST_ACC || DST == DST_GBAR_DIAG || DST == DST_GBAR_OFF) {
#pragma unroll
    for (int r = 0; r < S::E; ++r) {
      const long long e = row * n + 2 * S::t_out(n1, r);
      const float2 z = make_float2(v[r].x * scale, v[r].y * scale);
      float2* op = reinterpret_cast<float2*>(dst + slot * dst_stride + e);
      if constexpr (DST == DST_ACC) {
        const float2 ov = *op;
        *op = make_float2(ov.x + z.x, ov.y + z.y);
      } else {
        const float* mb = dst2 + slot * 2 * dst_stride + e;
        const float2 m = *reinterpret_cast<const float2*>(mb);
        if constexpr (DST == DST_GBAR_DIAG) {
          const float2 sd = *reinterpret_cast<const float2*>(mb + dst_stride);
          *op = make_float2(m.x * (sd.x - z.x), m.y * (sd.y - z.y));
        } else {
          *op = make_float2(-2.f * m.x * z.x, -2.f * m.y * z.y);
        }
      }
    }
    return;
  }
  if constexpr (DST == DST_MU_AB || DST == DST_MU_ACC || DST == DST_MU_SQ) {
    // dst = A (running sum of the diagonal derivatives), dst2 = mu
#pragma unroll
    for (int r = 0; r < S::E; ++r) {
      const long long gi = slot * dst_stride + row * n + 2 * S::t_out(n1, r);
      const float2 z = make_float2(v[r].x * scale, v[r].y * scale);
      float2* ap = reinterpret_cast<float2*>(dst + gi);
      float2* mp = reinterpret_cast<float2*>(dst2 + gi);
      if constexpr (DST == DST_MU_AB) {  // mu = A v, A = A + v
        const float2 av = *ap;
        *mp = make_float2(av.x * z.x, av.y * z.y);
        *ap = make_float2(av.x + z.x, av.y + z.y);
      } else if constexpr (DST == DST_MU_ACC) {  // mu += A v
        const float2 av = *ap, mv = *mp;
        *mp = make_float2(mv.x + av.x * z.x, mv.y + av.y * z.y);
      } else {  // mu -= v^2
        const float2 mv = *mp;
        *mp = make_float2(mv.x - z.x * z.x, mv.y - z.y * z.y);
      }
    }
    return;
  }
#pragma unroll
  for (int r = 0; r < S::E; ++r) {
    // DST_IC: particle arrays in lattice-block order (z pairs stay adjacent)
    const long long gi = slot * dst_stride + (DST == DST_IC ? blocked_index(row / n, row % n, 2 * S::t_out(n1, r),
                                                                            log2n, log2pb)
                                                            : row * n + 2 * S::t_out(n1, r));
    const float2 z = make_float2(v[r].x * scale, v[r].y * scale);
    *reinterpret_cast<float2*>(dst + gi) = z;
    if constexpr (DST == DST_IC) *reinterpret_cast<float2*>(dst2 + gi) = make_float2(z.x * scale2, z.y * scale2);
  }
}

// ---------------------------------------- column passes, register FFT

// The same passes as k_cols, with the column transform held in registers
// (four-step split, one LDS exchange per transform; fft_reg.h).  Per-mode
// arithmetic is applied on load (input layout, t = n1 + P r) or after the
// forward transform (output layout).
template <int L, int C, int MODE>
__global__ void __launch_bounds__(256, 2) k_cols_reg(ColArgs a) {  // <= 256 VGPRs: two blocks per CU (their LDS allows two)
  using S = freg::Shape<L, C>;
  __shared__ float2 lds[S::LDS];
  const int slot = blockIdx.z;
  if (!slot_on(a.gate, a.active, slot)) return;
  // adjacent column groups (halves of one 128-byte line) share an XCD's L2
  const unsigned lid = xcd_pair(blockIdx.x + gridDim.x * blockIdx.y, gridDim.x * gridDim.y);
  const int outer = (int)(lid / gridDim.x);  // x for the y pass, y for the x pass
  const int c = threadIdx.x % C, n1 = threadIdx.x / C;
  const int iz = (int)(lid % gridDim.x) * C + c;
  const int zl = a.zlim > 0 && a.zlim < a.nh ? a.zlim : a.nh;
  const bool valid = iz < zl;
  const int izc = valid ? iz : 0;  // an in-range column for table reads of the lanes past the last
  auto kept = [&](int t) { int m = signed_mode(t, a.n); return 2 * (m < 0 ? -m : m) < a.keep; };
  if (a.keep_outer && !kept(outer)) return;  // block-uniform
  // the 1D tables of a fused multiplier, staged in LDS (visible after the
  // forward transform's barriers): read from global memory inside the
  // multiplier loop, a thread's E reads were waited for one at a time (the
  // kernel sits at its register cap)
  constexpr bool kTabDec = MODE == MODE_NUFFT_C || MODE == MODE_NUFFT_ADJ;
  constexpr bool kTabLap = MODE == MODE_FUSED_H || MODE == MODE_FUSED_IL;
  __shared__ float tab0[(kTabDec || kTabLap) ? L : 1], tab1[kTabLap ? L : 1];
  if constexpr (kTabDec) {
    for (int k = threadIdx.x; k < L; k += 256) tab0[k] = a.esdec[k];
  }
  if constexpr (kTabLap) {
    for (int k = threadIdx.x; k < L; k += 256) {
      tab0[k] = a.lap[k];
      tab1[k] = a.win2[k];
    }
  }
  // the slot's multiplier coefficient, read once (inside the loop it was
  // re-read, and waited for, per element)
  const float fc = kTabLap ? fused_coef(a, slot) : 0.f;
  const long long stride_t = a.axis == 1 ? (long long)a.rs : (long long)a.n * a.rs;
  const long long base0 = a.axis == 1 ? (long long)outer * a.n * a.rs : (long long)outer * a.rs;
  const long long col = slot * a.slot_stride + base0 + iz;
  float2 v[S::E];
#pragma unroll
  for (int r = 0; r < S::E; ++r) {
    const int t = S::t_in(n1, r);
    float2 x = make_float2(0.f, 0.f);
    if (valid && !(a.keep_in && !kept(t))) {
      if constexpr (MODE == MODE_COMBINE_IC) {
        // x pass: t = ix, outer = iy: sum_c conj(h_c) S_c, h_c = i h
        if (a.combine_add) x = a.data[col + t * stride_t];
        int mx = signed_mode(t, a.n), my = signed_mode(outer, a.n);
        float amp = a.amp[mx * mx + my * my + iz * iz] * a.fac[slot];
        int ms[3] = {mx, my, iz};
        const float2* s3 = a.src3 + col + t * stride_t;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          if (ms[q] == -a.n / 2 || ms[q] == a.n / 2) continue;
          float2 sv = s3[q * a.comp_stride];
          float h = amp * ms[q];
          x.x += h * sv.y;
          x.y -= h * sv.x;
        }
      } else if constexpr (MODE == MODE_LPT_MUBAR) {
        // x pass: t = ix, outer = iy on the padded grid; kept modes only
        const int mx = signed_mode(t, a.n), my = signed_mode(outer, a.n), np = a.n_p;
        if (2 * (mx < 0 ? -mx : mx) < np && 2 * (my < 0 ? -my : my) < np && 2 * iz < np) {
          const int ms[3] = {mx, my, iz};
          const float k0 = 6.283185307179586f / (float)np;
          float th2 = 0.f;
#pragma unroll
          for (int q = 0; q < 3; ++q) th2 += (k0 * ms[q]) * (k0 * ms[q]);
          if (th2 > 0.f) {
            const float2* s3 = a.src3 + slot * a.src_slot_stride +
                               (long long)((mx & (np - 1)) * np + (my & (np - 1))) * a.src_rs + iz;
#pragma unroll
            for (int q = 0; q < 3; ++q) {
              const float2 sv = s3[q * a.comp_stride];
              const float h = a.coef[slot] * (k0 * ms[q]) / th2;
              x.x += h * sv.y;  // conj(i h) sv
              x.y -= h * sv.x;
            }
          }
        }
      } else if constexpr (MODE == MODE_LPT_DT) {
        x = a.data[col + t * stride_t];
      } else if constexpr (MODE == MODE_LPT_D) {
        // x pass: t = ix, outer = iy on the padded grid; kept modes only
        const int mx = signed_mode(t, a.n), my = signed_mode(outer, a.n), np = a.n_p;
        if (2 * (mx < 0 ? -mx : mx) < np && 2 * (my < 0 ? -my : my) < np && 2 * iz < np) {
          const int ms[3] = {mx, my, iz};
          const float2 sv = a.src3[slot * a.src_slot_stride +
                                   (long long)((mx & (np - 1)) * np + (my & (np - 1))) * a.src_rs + iz];
          const float h = -(6.283185307179586f / (float)np) * (float)(ms[a.comp] * ms[a.comp2]) *
                          a.amp[mx * mx + my * my + iz * iz] * a.fac[slot];
          x = make_float2(h * sv.x, h * sv.y);
        }
      } else {
        x = a.data[col + t * stride_t];
      }
      if constexpr (MODE == MODE_IC_C) {
        int mx = signed_mode(t, a.n), my = signed_mode(outer, a.n);
        int ms[3] = {mx, my, iz};
        int mc = ms[a.comp];
        float h = (mc == -a.n / 2 || mc == a.n / 2) ? 0.f : a.amp[mx * mx + my * my + iz * iz] * a.fac[slot] * mc;
        x = make_float2(-h * x.y, h * x.x);  // i h x
      }
    }
    v[r] = x;
  }
  constexpr bool kFwdFirst = MODE == MODE_FWD || MODE == MODE_FUSED_H || MODE == MODE_NUFFT_C ||
                             MODE == MODE_NUFFT_ADJ || MODE == MODE_FUSED_IL || MODE == MODE_LPT_DT;
  bool inverse_next = !kFwdFirst;  // input layout holds data for an inverse transform
  if constexpr (kFwdFirst) {
    freg::pass_a<S, false>(v, n1, a.tw, a.tws);
    freg::store_y<S>(v, lds, n1, c);
    __syncthreads();
    freg::pass_b<S, false>(v, lds, n1, c);
    if constexpr (MODE == MODE_FUSED_H) {
#pragma unroll
      for (int r = 0; r < S::E; ++r) {
        const int t = S::t_out(n1, r);
        float l = tab0[t] + tab0[outer] + (valid ? tab0[izc] : 0.f);
        float w = tab1[t] * tab1[outer] * (valid ? tab1[izc] : 1.f);
        float h = (t == 0 && outer == 0 && iz == 0) || !valid ? 0.f : fc / (l * w);
        v[r].x *= h;
        v[r].y *= h;
      }
      inverse_next = true;
    }
    if constexpr (MODE == MODE_LPT_DT) {
      // output t = ix: the kept modes add h v to the particle-grid spectrum
      if (!valid) return;
      const int my = signed_mode(outer, a.n), np = a.n_p;
#pragma unroll
      for (int r = 0; r < S::E; ++r) {
        const int t = S::t_out(n1, r), mx = signed_mode(t, a.n);
        if (!(2 * (mx < 0 ? -mx : mx) < np && 2 * (my < 0 ? -my : my) < np && 2 * iz < np)) continue;
        const int ms[3] = {mx, my, iz};
        const float h = -(6.283185307179586f / (float)np) * (float)(ms[a.comp] * ms[a.comp2]) *
                        a.amp[mx * mx + my * my + iz * iz] * a.fac[slot];
        float2* q = a.dst3 + slot * a.src_slot_stride + (long long)((mx & (np - 1)) * np + (my & (np - 1))) * a.src_rs + iz;
        const float2 qv = *q;
        *q = make_float2(qv.x + h * v[r].x, qv.y + h * v[r].y);
      }
      return;
    }
    if constexpr (MODE == MODE_FUSED_IL) {
      const float inv_n = 1.f / (float)a.n;  // phi = pi (m_x + m_y + m_z) / n
#pragma unroll
      for (int r = 0; r < S::E; ++r) {
        const int t = S::t_out(n1, r);
        float l = tab0[t] + tab0[outer] + (valid ? tab0[izc] : 0.f);
        float w = tab1[t] * tab1[outer] * (valid ? tab1[izc] : 1.f);
        float h = (t == 0 && outer == 0 && iz == 0) || !valid ? 0.f : fc / (l * w);
        float2 d2 = make_float2(0.f, 0.f);
        float cs = 1.f, sn = 0.f;
        if (valid) {
          d2 = a.src3[col + t * stride_t];
          sincospif((float)(signed_mode(t, a.n) + signed_mode(outer, a.n) + iz) * inv_n, &sn, &cs);
        }
        // delta = (d1 + e^{i phi} d2) / 2; grid 1 keeps H delta, grid 2 gets H delta e^{-i phi}
        const float dr = 0.5f * (v[r].x + cs * d2.x - sn * d2.y), di = 0.5f * (v[r].y + cs * d2.y + sn * d2.x);
        v[r] = make_float2(h * dr, h * di);
        if (valid) a.dst3[col + t * stride_t] = make_float2(h * (cs * dr + sn * di), h * (cs * di - sn * dr));
      }
      inverse_next = true;
    }
    // NUFFT multipliers: the table reads are unconditional (lanes past the
    // last column read column 0 and hold zeros, so their h is harmless): a
    // read under the per-lane `valid` branch would be waited for in turn
    if constexpr (MODE == MODE_NUFFT_C) {
      // truncation, deconvolution and i k_c s / k^2 of component comp
      const float k0 = 6.283185307179586f / (float)a.n_p;
      const float dyz = tab0[outer] * tab0[izc];
#pragma unroll
      for (int r = 0; r < S::E; ++r) {
        const int t = S::t_out(n1, r);
        const float dec = tab0[t] * dyz;
        const int ms[3] = {signed_mode(t, a.n), signed_mode(outer, a.n), izc};
        float th2 = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) th2 += (k0 * ms[q]) * (k0 * ms[q]);
        const float h = (dec == 0.f || th2 == 0.f) ? 0.f : a.coef[slot] * dec * (k0 * ms[a.comp]) / th2;
        v[r] = make_float2(-h * v[r].y, h * v[r].x);  // i h v
      }
      inverse_next = true;
    }
    if constexpr (MODE == MODE_NUFFT_ADJ) {
      // adjoint mesh term: the spread kernel gradient already carries the
      // -i k_c of the transposed multiplier, what is left is real:
      // coef / (k^2 Phi^2) on the kept modes (coef includes n_f / n_p)
      const float k0 = 6.283185307179586f / (float)a.n_p;
      const float dyz = tab0[outer] * tab0[izc];
#pragma unroll
      for (int r = 0; r < S::E; ++r) {
        const int t = S::t_out(n1, r);
        const float dec = tab0[t] * dyz;
        const int ms[3] = {signed_mode(t, a.n), signed_mode(outer, a.n), izc};
        float th2 = 0.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) th2 += (k0 * ms[q]) * (k0 * ms[q]);
        const float h = (dec == 0.f || th2 == 0.f) ? 0.f : a.coef[slot] * dec / th2;
        v[r].x *= h;
        v[r].y *= h;
      }
      inverse_next = true;
    }
    if (inverse_next) {  // back to the input layout for the inverse transform
      __syncthreads();
      freg::store_nat_out<S>(v, lds, n1, c);
      __syncthreads();
      freg::load_nat_in<S>(v, lds, n1, c);
    }
  }
  if (inverse_next) {
    freg::pass_a<S, true>(v, n1, a.tw, a.tws);
    __syncthreads();
    freg::store_y<S>(v, lds, n1, c);
    __syncthreads();
    freg::pass_b<S, true>(v, lds, n1, c);
  }
  if (!valid) return;
  float2* out = (MODE == MODE_IC_C || MODE == MODE_NUFFT_C || MODE == MODE_NUFFT_ADJ || MODE == MODE_LPT_D) ? a.dst3
                                                                                                       : a.data;
#pragma unroll
  for (int r = 0; r < S::E; ++r) {
    const int t = S::t_out(n1, r);
    if (a.keep_out && !kept(t)) continue;
    out[col + t * stride_t] = v[r];
  }
}

// ------------------------------------------------------------ dispatch

// NT: threads per block of the C2R, of the FP32 R2C and of the int64 R2C
template <int L, int P, int NT = 256, int NTF = 256, int NTI = 256>
static hipError_t launch_rows_reg(const RowLaunch& r) {
  const int R = (r.inverse ? NT : r.src_mode == SRC_I64 ? NTI : NTF) / P;
  dim3 grid((unsigned)((r.n_rows + R - 1) / R), r.batch);
  if (r.inverse) {
#define PM_C2R(D)                                                                                                \
  k_c2r_rows_reg<L, P, D, NT><<<grid, NT, 0, r.stream>>>((const float2*)r.src, r.src_stride, (float*)r.dst,          \
                                                      r.dst_stride, (float*)r.dst2, r.n_rows, r.tw, r.tws_half,   \
                                                      r.tws_full, (float)r.scale, (float)r.scale2, r.active,      \
                                                      r.rs, r.kz_lim, r.ic_log2pb, r.gate)
    switch (r.dst_mode) {
      case DST_F32: PM_C2R(DST_F32); break;
      case DST_IC: PM_C2R(DST_IC); break;
      case DST_MU_AB: PM_C2R(DST_MU_AB); break;
      case DST_MU_ACC: PM_C2R(DST_MU_ACC); break;
      case DST_MU_SQ: PM_C2R(DST_MU_SQ); break;
      case DST_IC2: PM_C2R(DST_IC2); break;
      case DST_ACC: PM_C2R(DST_ACC); break;
      case DST_GBAR_DIAG: PM_C2R(DST_GBAR_DIAG); break;
      case DST_GBAR_OFF: PM_C2R(DST_GBAR_OFF); break;
      default: return hipErrorInvalidValue;
    }
#undef PM_C2R
  } else {
    if (r.src_mode == SRC_I64)
      k_r2c_rows_reg<L, P, SRC_I64, NTI><<<grid, NTI, 0, r.stream>>>(r.src, r.src_stride, (float2*)r.dst, r.dst_stride,
                                                                r.n_rows, r.tw, r.tws_half, r.tws_full, r.scale,
                                                                r.shift, r.active, r.rs, r.kz_lim, r.gate);
    else
      k_r2c_rows_reg<L, P, SRC_F32, NTF><<<grid, NTF, 0, r.stream>>>(r.src, r.src_stride, (float2*)r.dst, r.dst_stride,
                                                                r.n_rows, r.tw, r.tws_half, r.tws_full, r.scale,
                                                                r.shift, r.active, r.rs, r.kz_lim, r.gate);
  }
  return hipGetLastError();
}

hipError_t fft_rows(const RowLaunch& r) {
  // P threads per row with P <= L / P (L = n / 2)
  switch (r.n) {
    case 4: return launch_rows_reg<2, 1>(r);
    case 8: return launch_rows_reg<4, 2>(r);
    case 16: return launch_rows_reg<8, 2>(r);
    case 32: return launch_rows_reg<16, 4>(r);
    case 64: return launch_rows_reg<32, 4>(r);
    case 128: return launch_rows_reg<64, 8>(r);
    case 256: return launch_rows_reg<128, 8>(r);
    case 512: return launch_rows_reg<256, 16>(r);
    // n = 1024: smaller blocks (each holds R rows of LDS exchange; 68 KB at
    // 256 threads allow two per CU) overlap one another's load and FFT
    // phases better (measured: C2R 1.79 -> 1.65 ms, FP32 R2C 1.82 -> 1.62 ms)
    case 1024: return launch_rows_reg<512, 16, 128, 64, 128>(r);
    default: return hipErrorInvalidValue;
  }
}

template <int L, int C>
static hipError_t launch_cols_c(const ColArgs& a, int mode, int batch, hipStream_t s) {
  dim3 grid((unsigned)((a.nh + C - 1) / C), (unsigned)a.n, (unsigned)batch);
  switch (mode) {
    case MODE_FWD: k_cols<L, C, MODE_FWD><<<grid, 256, 0, s>>>(a); break;
    case MODE_INV: k_cols<L, C, MODE_INV><<<grid, 256, 0, s>>>(a); break;
    case MODE_FUSED_H: k_cols<L, C, MODE_FUSED_H><<<grid, 256, 0, s>>>(a); break;
    case MODE_IC_C: k_cols<L, C, MODE_IC_C><<<grid, 256, 0, s>>>(a); break;
    case MODE_COMBINE_IC: k_cols<L, C, MODE_COMBINE_IC><<<grid, 256, 0, s>>>(a); break;
    case MODE_NUFFT_C: k_cols<L, C, MODE_NUFFT_C><<<grid, 256, 0, s>>>(a); break;
    case MODE_NUFFT_ADJ: k_cols<L, C, MODE_NUFFT_ADJ><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L, int C>
static hipError_t launch_cols_r(const ColArgs& a, int mode, int batch, hipStream_t s) {
  const int zl = a.zlim > 0 && a.zlim < a.nh ? a.zlim : a.nh;
  dim3 grid((unsigned)((zl + C - 1) / C), (unsigned)a.n, (unsigned)batch);
  switch (mode) {
    case MODE_FWD: k_cols_reg<L, C, MODE_FWD><<<grid, 256, 0, s>>>(a); break;
    case MODE_INV: k_cols_reg<L, C, MODE_INV><<<grid, 256, 0, s>>>(a); break;
    case MODE_FUSED_H: k_cols_reg<L, C, MODE_FUSED_H><<<grid, 256, 0, s>>>(a); break;
    case MODE_IC_C: k_cols_reg<L, C, MODE_IC_C><<<grid, 256, 0, s>>>(a); break;
    case MODE_COMBINE_IC: k_cols_reg<L, C, MODE_COMBINE_IC><<<grid, 256, 0, s>>>(a); break;
    case MODE_NUFFT_C: k_cols_reg<L, C, MODE_NUFFT_C><<<grid, 256, 0, s>>>(a); break;
    case MODE_NUFFT_ADJ: k_cols_reg<L, C, MODE_NUFFT_ADJ><<<grid, 256, 0, s>>>(a); break;
    case MODE_LPT_D: k_cols_reg<L, C, MODE_LPT_D><<<grid, 256, 0, s>>>(a); break;
    case MODE_FUSED_IL: k_cols_reg<L, C, MODE_FUSED_IL><<<grid, 256, 0, s>>>(a); break;
    case MODE_LPT_MUBAR: k_cols_reg<L, C, MODE_LPT_MUBAR><<<grid, 256, 0, s>>>(a); break;
    case MODE_LPT_DT: k_cols_reg<L, C, MODE_LPT_DT><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int L>
static hipError_t launch_cols(const ColArgs& a, int mode, int batch, hipStream_t s) {
  // register FFT from L = 16: P = 256 / C threads per column must not exceed
  // the E = L / P elements each holds
  if constexpr (L >= 16) {
    constexpr int C = L >= 1024 ? 8 : (L >= 256 ? 16 : (L >= 64 ? 32 : 64));
    return launch_cols_r<L, C>(a, mode, batch, s);
  } else {
    // the NUFFT passes and pruning exist only in the register kernels
    if (mode == MODE_NUFFT_C || mode == MODE_NUFFT_ADJ || mode == MODE_LPT_D || mode == MODE_FUSED_IL ||
        mode == MODE_LPT_MUBAR || mode == MODE_LPT_DT || a.keep ||
        a.zlim)
      return hipErrorInvalidValue;
    return launch_cols_c<L, 16>(a, mode, batch, s);
  }
}

hipError_t fft_cols(const ColArgs& a, int mode, int batch, hipStream_t s) {
  switch (a.n) {
    case 4: return launch_cols<4>(a, mode, batch, s);
    case 8: return launch_cols<8>(a, mode, batch, s);
    case 16: return launch_cols<16>(a, mode, batch, s);
    case 32: return launch_cols<32>(a, mode, batch, s);
    case 64: return launch_cols<64>(a, mode, batch, s);
    case 128: return launch_cols<128>(a, mode, batch, s);
    case 256: return launch_cols<256>(a, mode, batch, s);
    case 512: return launch_cols<512>(a, mode, batch, s);
    case 1024: return launch_cols<1024>(a, mode, batch, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pm
