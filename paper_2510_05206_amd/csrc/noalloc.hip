// Power spectrum of a given fixed-point mass mesh without any allocation:
// the variant of pm_power_spectrum for callers that cannot allocate device
// memory (code under graph capture, tight serving loops).  Its intermediate
// storage (FFT twiddles, CIC window table, the half spectrum and the partial
// bin sums) lives in one file-scope device array, `scratch`, whose address is
// looked up once per device; meshes up to kNoAllocMaxN cells per axis.
#include <mutex>

#include "fft.h"
#include "kernels.h"
#include "pm_internal.h"

namespace pm {
namespace {

constexpr int kNoAllocMaxN = 128;
constexpr size_t kAl = 256;
constexpr size_t al(size_t x) { return (x + kAl - 1) / kAl * kAl; }
constexpr int rs_of(int n) { return n >= 32 ? (n / 2 + 1 + 15) / 16 * 16 : n / 2 + 1; }
// sections: twiddles [n] float2, cic4 [n] double, spectrum [n][n][rs] float2,
// partial bin sums [n][n_bins <= n][3] double
constexpr size_t kOffTw = 0;
constexpr size_t kOffCic = al(kOffTw + sizeof(float2) * kNoAllocMaxN);
constexpr size_t kOffSpec = al(kOffCic + sizeof(double) * kNoAllocMaxN);
constexpr size_t kOffPart =
    al(kOffSpec + sizeof(float2) * (size_t)kNoAllocMaxN * kNoAllocMaxN * rs_of(kNoAllocMaxN));
constexpr size_t kScratchBytes = al(kOffPart + sizeof(double) * 3 * (size_t)kNoAllocMaxN * kNoAllocMaxN);

// one copy per device, held until the process ends (about 11 MB)
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// device address of this device's `scratch` (looked up once per device, with
// that device current); nullptr on failure
void* scratch_ptr(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_ptr[dev] = p;
  }
  return g_ptr[dev];
}

// twiddles exp(-2 pi i t / n) and the CIC window sinc^4(pi m / n) of the mesh
__global__ void k_noalloc_tables(float2* tw, double* cic4, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s, c;
  sincospi(-2.0 * (double)t / (double)n, &s, &c);
  tw[t] = make_float2((float)c, (float)s);
  const int m = t < n / 2 ? t : t - n;
  const double h = M_PI * (double)m / (double)n;
  const double sinc = m == 0 ? 1.0 : sin(h) / h;
  cic4[t] = sinc * sinc * sinc * sinc;
}

}  // namespace
}  // namespace pm

using namespace pm;

extern "C" pm_status pm_power_spectrum_mesh_noalloc(const int64_t* mesh, int32_t n, int64_t n_particles,
                                                    double box, int32_t n_bins, int32_t deconvolve_cic,
                                                    double* k_mean, double* pk, int64_t* n_modes,
                                                    void* hip_stream) {
  if (!mesh || !k_mean || !pk || !n_modes) return PM_EINVAL;
  if (n < 4 || (n & (n - 1)))
    return PM_EINVAL;
  if (n > kNoAllocMaxN) return PM_ENOMEM;  // beyond the static scratch
  if (n_bins < 1 || n_bins > n) return PM_EINVAL;
  if (n_particles < 1 || !(box > 0)) return PM_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return PM_EHIP;
  char* base = static_cast<char*>(scratch_ptr(dev));
  if (!base) return PM_EHIP;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  float2* tw = reinterpret_cast<float2*>(base + kOffTw);
  double* cic4 = reinterpret_cast<double*>(base + kOffCic);
  float2* spec = reinterpret_cast<float2*>(base + kOffSpec);
  double* part = reinterpret_cast<double*>(base + kOffPart);
  k_noalloc_tables<<<(n + 63) / 64, 64, 0, s>>>(tw, cic4, n);
  if (hipGetLastError() != hipSuccess) return PM_EHIP;
  const double M = (double)n * n * n, N = (double)n_particles;
  const long long spec_elems = (long long)n * n * rs_of(n);
  // contrast m n^3 / (N 2^32) - 1 -> z-row R2C, then the y and x passes
  RowLaunch r{};
  r.n = n;
  r.rs = rs_of(n);
  r.n_rows = (long long)n * n;
  r.batch = 1;
  r.inverse = false;
  r.src_mode = SRC_I64;
  r.src = mesh;
  r.src_stride = (long long)M;
  r.dst = spec;
  r.dst_stride = spec_elems;
  r.tw = tw;
  r.tws_half = 2;  // the table has n entries: the n/2 transform reads every second one
  r.tws_full = 1;
  r.scale = M / N / 4294967296.0;
  r.shift = 1.0;
  r.stream = s;
  r.active = 1;
  if (fft_rows(r) != hipSuccess) return PM_EHIP;
  ColArgs a{};
  a.data = spec;
  a.slot_stride = spec_elems;
  a.n = n;
  a.nh = n / 2 + 1;
  a.rs = rs_of(n);
  a.tw = tw;
  a.tws = 1;
  a.active = 1;
  a.axis = 1;
  if (fft_cols(a, MODE_FWD, 1, s) != hipSuccess) return PM_EHIP;
  a.axis = 0;
  if (fft_cols(a, MODE_FWD, 1, s) != hipSuccess) return PM_EHIP;
  if (launch_pk(spec, spec_elems, n, 1, n_bins, 2.0 * M_PI / box, box * box * box / (M * M), cic4, deconvolve_cic,
                part, k_mean, pk, (long long*)n_modes, 1, rs_of(n), s) != hipSuccess)
    return PM_EHIP;
  return PM_OK;
}
