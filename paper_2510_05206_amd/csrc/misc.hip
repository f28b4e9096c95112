// Auxiliary kernels: fills, white noise, the IC-adjoint source, deterministic
// FP64 reductions and the binned power spectrum.
#include "kernels.h"
#include "mak.h"

namespace pm {

__global__ void k_fill(uint4* p, long long n16) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long step = (long long)gridDim.x * blockDim.x;
  for (; i < n16; i += step) p[i] = make_uint4(0, 0, 0, 0);
}

hipError_t launch_fill(void* p, long long bytes, hipStream_t s) {
  // bytes is a multiple of 16 for every buffer carved by the context
  long long n16 = bytes / 16;
  long long blocks = (n16 + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  k_fill<<<(unsigned)blocks, 256, 0, s>>>((uint4*)p, n16);
  return hipGetLastError();
}

__global__ void k_lincomb(const float* a, const float* x, float* out, long long n, SlotCoef coef,
                          unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  const float k = coef.v[slot];
  const long long o = slot * n;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[o + i] = a[o + i] + k * x[o + i];
}

hipError_t launch_lincomb(const float* a, const float* x, float* out, long long n, const SlotCoef& coef, int batch,
                          unsigned long long active, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_lincomb<<<dim3((unsigned)blocks, batch), 256, 0, s>>>(a, x, out, n, coef, active);
  return hipGetLastError();
}

__global__ void k_mul(const float* a, long long sa, const float* b, long long sb, float* out, long long so,
                      long long n, unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    out[slot * so + i] = a[slot * sa + i] * b[slot * sb + i];
}

hipError_t launch_mul(const float* a, long long sa, const float* b, long long sb, float* out, long long so,
                      long long n, int batch, unsigned long long active, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_mul<<<dim3((unsigned)blocks, batch), 256, 0, s>>>(a, sa, b, sb, out, so, n, active);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256) k_tan_drift(float* xd, const float* vd, long long n, long long stride,
                                                   SlotCoef tau, unsigned int* amax, unsigned long long active) {
  __shared__ float red[256];
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  const float tp = tau.v[slot];
  const long long o = slot * stride;
  float m = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    float x = xd[o + i];
    if (tp != 0.f) {
      x += tp * vd[o + i];
      xd[o + i] = x;
    }
    m = fmaxf(m, fabsf(x));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0] > 0.f) atomicMax(amax + slot, __float_as_uint(red[0]));
}

hipError_t launch_tan_drift(float* xd, const float* vd, long long n, long long stride, const SlotCoef& tau,
                            unsigned int* amax, int batch, unsigned long long active, hipStream_t s) {
  long long blocks = (n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  k_tan_drift<<<dim3((unsigned)blocks, batch), 256, 0, s>>>(xd, vd, n, stride, tau, amax, active);
  return hipGetLastError();
}

// ---------------------------------------------- device-indexed step state
// gate[b]: the step slot b runs next (-1 idle).  Set from the host by value
// (k[b] = -2 keeps the current value), advanced at the end of each device
// step (the last step of a slot returns it to -1).
__global__ void k_set_gate(int32_t* gate, GateSet g) {
  const int b = threadIdx.x;
  if (b < g.batch && g.k[b] != -2) gate[b] = g.k[b];
}

__global__ void k_advance_gate(int32_t* gate, const int32_t* nsteps, int batch) {
  const int b = threadIdx.x;
  if (b < batch && gate[b] >= 0) gate[b] = gate[b] + 1 < nsteps[b] ? gate[b] + 1 : -1;
}

// one slot's schedule rows (kSch floats per step) and its step count
__global__ void k_set_sched(float* sched, int32_t* nsteps, SchedRows r) {
  for (int e = threadIdx.x; e < r.n * kSch; e += blockDim.x) sched[(long long)r.slot * r.stride * kSch + e] = r.v[e];
  if (threadIdx.x == 0) nsteps[r.slot] = r.n;
}

hipError_t launch_set_gate(int32_t* gate, const GateSet& g, hipStream_t s) {
  k_set_gate<<<1, kMaxBatch, 0, s>>>(gate, g);
  return hipGetLastError();
}

hipError_t launch_advance_gate(int32_t* gate, const int32_t* nsteps, int batch, hipStream_t s) {
  k_advance_gate<<<1, kMaxBatch, 0, s>>>(gate, nsteps, batch);
  return hipGetLastError();
}

hipError_t launch_set_sched(float* sched, int32_t* nsteps, const SchedRows& r, hipStream_t s) {
  k_set_sched<<<1, 256, 0, s>>>(sched, nsteps, r);
  return hipGetLastError();
}

// Philox-4x32-10 (Salmon, Moraes, Dror & Shaw 2011) keyed by the seed, counter
// = (i mod 2^32, i div 2^32, 0, 0); one standard normal per lattice site by
// Box-Muller in FP64, rounded once to FP32.
struct Seeds {
  uint32_t k0[kMaxBatch], k1[kMaxBatch];
};

__global__ void k_white_noise(float* w, long long N, long long slot_stride, Seeds sd,
                              unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  uint32_t c0 = (uint32_t)i, c1 = (uint32_t)(i >> 32), c2 = 0, c3 = 0;
  uint32_t k0 = sd.k0[slot], k1 = sd.k1[slot];
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  unsigned long long h1 = (((unsigned long long)c0 << 32) | c1) >> 11;
  unsigned long long h2 = (((unsigned long long)c2 << 32) | c3) >> 11;
  double u1 = ((double)h1 + 0.5) * 0x1p-53;
  double u2 = (double)h2 * 0x1p-53;
  double v = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  w[slot * slot_stride + i] = (float)v;
}

hipError_t launch_white_noise(float* w, long long N, long long slot_stride, int batch,
                              const uint64_t* seeds, unsigned long long active, hipStream_t s) {
  Seeds sd;
  for (int b = 0; b < batch; ++b) {
    if (!((active >> b) & 1ull)) continue;
    sd.k0[b] = (uint32_t)(seeds[b] & 0xFFFFFFFFu);
    sd.k1[b] = (uint32_t)(seeds[b] >> 32);
  }
  dim3 grid((unsigned)((N + 255) / 256), batch);
  k_white_noise<<<grid, 256, 0, s>>>(w, N, slot_stride, sd, active);
  return hipGetLastError();
}

// psi_bar_c = D0 X_bar_c + V_bar_c (the IC pullback of Psi = D0 psi, V = psi)
struct D0s { float d0[kMaxBatch]; };
// psi_bar = D0 X_bar + V_bar, from the lattice-block particle order into
// row-major lattice order (the layout of the initial-condition transforms)
__global__ void k_psibar(const float* xbar, const float* vbar, float* out, long long N,
                         long long stride, D0s d, int log2_np, int log2_pb, unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * N) return;
  const long long c = i / N, p = i - c * N;
  long long j[3];
  lattice_of(p, log2_np, log2_pb, j);
  const long long g = slot * stride + i;
  out[slot * stride + c * N + ((j[0] << log2_np | j[1]) << log2_np | j[2])] = d.d0[slot] * xbar[g] + vbar[g];
}

hipError_t launch_psibar(const float* xbar, const float* vbar, float* out, long long N,
                         long long part_stride, int batch, const float* d0, int log2_np, int log2_pb,
                         unsigned long long active, hipStream_t s) {
  D0s d;
  for (int b = 0; b < batch; ++b) d.d0[b] = d0[b];
  dim3 grid((unsigned)((3 * N + 255) / 256), batch);
  k_psibar<<<grid, 256, 0, s>>>(xbar, vbar, out, N, part_stride, d, log2_np, log2_pb, active);
  return hipGetLastError();
}

// particle arrays [B][ncomp][N] between row-major lattice order and the
// lattice-block storage order (to_blocked: row-major in, blocked out)
__global__ void k_reorder(const float* src, float* dst, long long N, long long stride, int ncomp, int log2_np,
                          int log2_pb, bool to_blocked, unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncomp * N) return;
  const long long c = i / N, r = i - c * N;  // r: row-major lattice index
  const long long m = (1ll << log2_np) - 1;
  const long long b = blocked_index(r >> (2 * log2_np), (r >> log2_np) & m, r & m, log2_np, log2_pb);
  const long long base = slot * stride + c * N;
  if (to_blocked)
    dst[base + b] = src[base + r];
  else
    dst[base + r] = src[base + b];
}

hipError_t launch_reorder(const float* src, float* dst, long long N, long long stride, int ncomp, int batch,
                          int log2_np, int log2_pb, bool to_blocked, unsigned long long active, hipStream_t s) {
  dim3 grid((unsigned)((ncomp * N + 255) / 256), batch);
  k_reorder<<<grid, 256, 0, s>>>(src, dst, N, stride, ncomp, log2_np, log2_pb, to_blocked, active);
  return hipGetLastError();
}

// deterministic FP64 dot product: fixed per-thread striding, fixed tree in
// the block, fixed-order sum of the block partials
constexpr int kDotBlocks = 256;

__global__ void k_dot_partial(const float* a, const float* b, long long n, long long stride,
                              double* partial, unsigned long long active) {
  __shared__ double sh[256];
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)kDotBlocks * 256)
    acc += (double)a[slot * stride + i] * (double)b[slot * stride + i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[slot * kDotBlocks + blockIdx.x] = sh[0];
}

struct Scales {
  double s[kMaxBatch];
  long long idx[kMaxBatch];  // output element of each slot
};
__global__ void k_dot_final(const double* partial, double* out, Scales sc, unsigned long long active) {
  const int slot = blockIdx.x;
  if (!((active >> slot) & 1ull)) return;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kDotBlocks; ++i) t += partial[slot * kDotBlocks + i];
    out[sc.idx[slot]] = t * sc.s[slot];
  }
}

// out[out_idx[b]] = scale[b] sum_i a[b][i] b[b][i] (FP64, fixed order);
// out_idx null: out[b]
hipError_t launch_dot(const float* a, const float* b, long long n, long long stride, int batch,
                      double* partial, double* out, const double* scale, unsigned long long active,
                      hipStream_t s, const long long* out_idx) {
  k_dot_partial<<<dim3(kDotBlocks, batch), 256, 0, s>>>(a, b, n, stride, partial, active);
  Scales sc;
  for (int i = 0; i < batch; ++i) {
    sc.s[i] = scale[i];
    sc.idx[i] = out_idx ? out_idx[i] : i;
  }
  k_dot_final<<<batch, 64, 0, s>>>(partial, out, sc, active);
  return hipGetLastError();
}

// temporal adjoints of one reverse step from the dots taken around its
// adjoint kick: d1 = V_bar^{n+1/2} . V^{n+1} before it, d2 = (alpha
// V_bar^{n+1/2}) . V^n after it; alpha_bar = d2 / alpha, beta_bar =
// V_bar^{n+1/2} . A = (d1 - d2) / beta (V^{n+1} - alpha V^n = beta A)
__global__ void k_time_ab(const double* d1, const double* d2, double* out, TimeAB t, unsigned long long active) {
  const int slot = threadIdx.x;
  if (slot >= kMaxBatch || !((active >> slot) & 1ull)) return;
  out[t.idx[slot] + 2] = d2[slot] / t.alpha[slot];
  out[t.idx[slot] + 3] = t.beta[slot] != 0.0 ? (d1[slot] - d2[slot]) / t.beta[slot] : 0.0;
}

hipError_t launch_time_ab(const double* d1, const double* d2, double* out, const TimeAB& t,
                          unsigned long long active, hipStream_t s) {
  k_time_ab<<<1, kMaxBatch, 0, s>>>(d1, d2, out, t, active);
  return hipGetLastError();
}

__global__ void k_i64_to_delta(const long long* m, float* delta, long long M, long long stride,
                               double scale, unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M) return;
  delta[slot * stride + i] = (float)((double)m[slot * stride + i] * scale - 1.0);
}

hipError_t launch_i64_to_delta(const long long* m, float* delta, long long M, long long stride,
                               int batch, double scale, unsigned long long active, hipStream_t s) {
  dim3 grid((unsigned)((M + 255) / 256), batch);
  k_i64_to_delta<<<grid, 256, 0, s>>>(m, delta, M, stride, scale, active);
  return hipGetLastError();
}

// ------------------------------------------------------------------ P(k)
// One block per (x plane, slot).  Each wave walks rows y = wave, wave+4, ...
// in 64-wide z chunks; within a chunk the bins are non-decreasing in z, so a
// segmented shuffle scan sums each run of equal bins and the run's last lane
// adds it to the wave's own LDS column.  Wave columns and then x planes are
// summed in a fixed order: the FP64 result does not depend on scheduling.

// bin of |m|^2 = m2 from s = sqrt(m2) (sqrt(4 m2) = 2 s exactly, and the
// integer steps make r = floor(sqrt(4 m2)) exact)
__device__ __forceinline__ int pk_bin(long long m2, double s) {
  const long long t = 4 * m2;
  long long r = (long long)(2.0 * s);
  while (r * r > t) --r;
  while ((r + 1) * (r + 1) <= t) ++r;
  return (int)((r + 1) / 2);
}

// bins of |X|^2, or of 2 Re(conj(X) Y) with a second spectrum Y (the
// tangent of |X|^2 when X moves along Y)
__global__ void __launch_bounds__(256) k_pk_partial(const float2* spec, const float2* spec2, long long slot_stride,
                                                    int n, int n_bins, double kf, const double* cic4,
                                                    int deconv, double* partial,
                                                    unsigned long long active, int rs) {
  extern __shared__ double acc[];  // [3][n_bins][4]
  const int slot = blockIdx.y, x = blockIdx.x;
  if (!((active >> slot) & 1ull)) return;
  const int nh = n / 2 + 1;
  for (int e = threadIdx.x; e < 3 * n_bins * 4; e += 256) acc[e] = 0.0;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long mx = x < n / 2 ? x : x - n;
  constexpr int kChunks = 9;  // 64-wide z chunks of a half row (n <= 1024)
  for (int y = wave; y < n; y += 4) {
    const long long my = y < n / 2 ? y : y - n;
    // the whole half row's values first (in-range z for every lane), so that
    // a row costs one memory round trip rather than one per chunk
    // (unconditional reads: a read under a condition is waited for inside it)
    const long long row = slot * slot_stride + ((long long)x * n + y) * rs;
    const float2* s2 = spec2 ? spec2 : spec;
    float2 Xs[kChunks], Ys[kChunks];
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {
      const long long e = row + min(64 * ch + lane, nh - 1);
      Xs[ch] = spec[e];
      Ys[ch] = s2[e];
    }
#pragma unroll
    for (int ch = 0; ch < kChunks; ++ch) {
      if (64 * ch >= nh) break;
      int z = 64 * ch + lane;
      int b = 0, vc = 0;  // (the mode count is an integer: one shuffle instead of two)
      double vp = 0.0, vk = 0.0;
      if (z < nh) {
        long long m2 = mx * mx + my * my + (long long)z * z;
        const double sm = sqrt((double)m2);  // one square root for the bin and |k|
        if (m2 > 0) {
          b = pk_bin(m2, sm);
          if (b > n_bins) b = 0;
        }
        if (b) {
          double wm = (z == 0 || z == n / 2) ? 1.0 : 2.0;
          const float2 X = Xs[ch];
          double p;
          if (spec2) {
            const float2 Y = Ys[ch];
            p = 2.0 * ((double)X.x * Y.x + (double)X.y * Y.y);
          } else {
            p = (double)X.x * X.x + (double)X.y * X.y;
          }
          if (deconv) p /= cic4[x] * cic4[y] * cic4[z];
          vp = wm * p;
          vk = wm * kf * sm;
          vc = (int)wm;
        }
      }
      for (int off = 1; off < 64; off <<= 1) {
        double up = __shfl_up(vp, off), uk = __shfl_up(vk, off);
        int uc = __shfl_up(vc, off);
        int ub = __shfl_up(b, off);
        if (lane >= off && ub == b) { vp += up; vk += uk; vc += uc; }
      }
      int nb = __shfl_down(b, 1);
      bool last = (lane == 63) || (nb != b);
      if (b && last) {
        acc[(0 * n_bins + b - 1) * 4 + wave] += vp;
        acc[(1 * n_bins + b - 1) * 4 + wave] += vk;
        acc[(2 * n_bins + b - 1) * 4 + wave] += (double)vc;
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 3 * n_bins; e += 256) {
    double t = acc[e * 4 + 0] + acc[e * 4 + 1];
    t += acc[e * 4 + 2];
    t += acc[e * 4 + 3];
    int q = e / n_bins, bb = e - q * n_bins;
    partial[(((long long)slot * n + x) * n_bins + bb) * 3 + q] = t;
  }
}

__global__ void k_pk_final(const double* partial, int n, int n_bins, double norm, double* k_mean,
                           double* pk, long long* n_modes, unsigned long long active) {
  const int slot = blockIdx.y;
  if (!((active >> slot) & 1ull)) return;
  int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  double sp = 0.0, sk = 0.0, sc = 0.0;
  for (int x = 0; x < n; ++x) {
    const double* p = partial + (((long long)slot * n + x) * n_bins + b) * 3;
    sp += p[0];
    sk += p[1];
    sc += p[2];
  }
  long long o = (long long)slot * n_bins + b;
  k_mean[o] = sc > 0 ? sk / sc : 0.0;
  pk[o] = sc > 0 ? norm * sp / sc : 0.0;
  n_modes[o] = (long long)sc;
}

hipError_t launch_pk(const float2* spec, long long slot_stride, int n, int batch, int n_bins,
                     double kf, double norm, const double* cic4, int deconv, double* partial,
                     double* k_mean, double* pk, long long* n_modes, unsigned long long active,
                     int rs, hipStream_t s, const float2* spec2) {
  size_t lds = (size_t)3 * n_bins * 4 * sizeof(double);
  k_pk_partial<<<dim3(n, batch), 256, lds, s>>>(spec, spec2, slot_stride, n, n_bins, kf, cic4, deconv,
                                                partial, active, rs);
  k_pk_final<<<dim3((n_bins + 63) / 64, batch), 64, 0, s>>>(partial, n, n_bins, norm, k_mean, pk,
                                                           n_modes, active);
  return hipGetLastError();
}

}  // namespace pm
