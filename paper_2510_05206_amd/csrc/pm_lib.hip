// C ABI of libpm.so: context, workspace carving and the call sequences of the
// PM hot path (see include/pm.h for the contract of every entry point).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "fft.h"
#include "kernels.h"

using namespace pm;

struct pm_ctx {
  pm_config cfg;
  std::string err;
  Growth growth;
  std::vector<StepCoef> table;       // full schedule of cfg.n_steps
  std::vector<std::vector<StepCoef>> slot_table;
  std::vector<int> slot_steps;
  std::vector<double> slot_sigma8;
  double D0 = 0, D_ref = 1, amp = 0;
  double vfac = 1;  // initial velocity per unit dX/dD: zeta(a_start) for the canonical momentum, else 1
  int Lmax = 0;
  // host tables
  std::vector<float2> tw;
  std::vector<float> lap, win2, amp_tab;
  std::vector<double> cic4;
  std::vector<int32_t> es_tab;       // NUFFT: integer ES table (4096 samples per cell)
  std::vector<float> esdec;          // NUFFT: 1/phi_hat^2 on kept modes, 0 elsewhere
  std::vector<float> lptkeep;        // 2LPT: 1 on the modes |m| < n_p/2 of the 2 n_p grid, 0 elsewhere
  // binding
  bool bound = false, with_adj = false;
  hipStream_t stream = nullptr;
  Geom g{}, gp{};   // mesh geometry, particle-grid geometry (IC FFTs)
  // device pointers
  float2* d_tw = nullptr;
  float *d_lap = nullptr, *d_win2 = nullptr, *d_amp = nullptr;
  double* d_cic4 = nullptr;
  int32_t* d_es_tab = nullptr;
  float* d_esdec = nullptr;
  float* d_lptkeep = nullptr;
  // device-indexed steps (pm_set_step_index / pm_step_device)
  int32_t *d_gate = nullptr, *d_gsteps = nullptr;
  float* d_sched = nullptr;
  std::vector<char> sched_dirty;     // slots whose device schedule must be re-uploaded
  hipGraphExec_t step_exec = nullptr;
  unsigned long long bind_gen = 0, step_bind_gen = 0;
  float* force3 = nullptr;           // NUFFT: 3 force meshes [B][3][M]
  float2* spec2 = nullptr;           // NUFFT: per-component spectrum; interlaced PM: the second grid's
  float* accbuf = nullptr;           // interlaced PM: one grid's per-particle terms [B][6][N]
  float* phi2 = nullptr;
  bool tangent_valid = false;        // xbar/vbar hold pm_jvp's final tangents             // interlaced PM: the second grid's potential (in the mesh buffer)
  float *disp = nullptr, *vel = nullptr, *w = nullptr, *xbar = nullptr, *vbar = nullptr;
  long long* mesh = nullptr;
  float2* spec = nullptr;
  float* phi = nullptr;
  // tile binning and window slabs
  int T = 16, log2T = 4, log2nt = 0, n_tiles = 1;
  long long ts = 0;
  int32_t *key = nullptr, *rank = nullptr, *sorted = nullptr, *count = nullptr, *offset = nullptr;
  int32_t* scan_partial = nullptr;  // block totals of the tile-count scan
  void* scratch = nullptr;
  float* u_sorted = nullptr;    // adjoint: u in sorted order; IC adjoint: psi_bar
  float* umax = nullptr;
  double *scale = nullptr, *inv_scale = nullptr;
  float2* icspec = nullptr;          // 4 spectra on the particle grid per slot
  long long icspec_stride = 0;       // float2 per slot (4 spectra)
  long long icspec_comp = 0;         // float2 per spectrum
  double* pk_partial = nullptr;
  double* dot_partial = nullptr;
  double* tdots = nullptr;           // temporal adjoints: the two dots around each adjoint kick [2][kMaxBatch]
  // state
  bool ics_done = false, ran = false;
  unsigned long long user_mask = 1;  // slots the whole-context calls act on (pm_set_active)
  // per-kernel-class event timing (pm_profile / pm_kernel_times)
  bool prof = false;
  struct Pending { int cls; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[PM_K_COUNT] = {};
  long long prof_n[PM_K_COUNT] = {};
  // pm_run as one captured HIP graph, rebuilt when anything it bakes in
  // (buffers, per-slot schedules, slot mask) changes: gen counts such changes
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraphExec_t run_exec = nullptr;
  unsigned long long gen = 1, run_gen = 0;
  ~pm_ctx() {
    // teardown: nothing useful can be done with an error here
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
    if (run_exec) (void)hipGraphExecDestroy(run_exec);
    if (step_exec) (void)hipGraphExecDestroy(step_exec);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
int ilog2(long long v) { int l = 0; while ((1ll << l) < v) ++l; return l; }
bool pow2(long long v) { return v > 0 && (v & (v - 1)) == 0; }

pm_status fail(pm_ctx* c, pm_status s, const std::string& m) {
  if (c) c->err = m;
  return s;
}

#define HIPCHK(ctx, expr)                                                              \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess)                                                              \
      return fail(ctx, PM_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));   \
  } while (0)

hipEvent_t take_event(pm_ctx* c) {
  hipEvent_t e = nullptr;
  if (!c->pool.empty()) {
    e = c->pool.back();
    c->pool.pop_back();
  } else if (hipEventCreate(&e) != hipSuccess) {
    e = nullptr;
  }
  return e;
}

void prof_begin(pm_ctx* c, int cls) {
  if (!c->prof) return;
  hipEvent_t a = take_event(c), b = take_event(c);
  if (!a || !b) return;
  (void)hipEventRecord(a, c->stream);  // timing is best effort: a failed record reads as no time
  c->pending.push_back({cls, a, b});
}

void prof_end(pm_ctx* c) {
  if (!c->prof || c->pending.empty()) return;
  (void)hipEventRecord(c->pending.back().b, c->stream);
}

// two launches timed as one stage (the first error wins)
hipError_t both(hipError_t a, hipError_t b) { return a != hipSuccess ? a : b; }

// launch with optional event timing of its kernel class
#define KLAUNCH(ctx, cls, expr)   \
  do {                            \
    prof_begin(ctx, cls);         \
    HIPCHK(ctx, expr);            \
    prof_end(ctx);                \
  } while (0)

struct Layout {
  size_t off_tw, off_lap, off_win2, off_amp, off_cic4;
  size_t off_disp, off_vel, off_w, off_xbar, off_vbar;
  size_t off_mesh, off_spec, off_phi, off_icspec, off_pk, off_dot;
  size_t off_key, off_rank, off_sorted, off_count, off_offset, off_scanp, off_scratch, off_u, off_umax, off_scale;
  size_t off_tdots, off_accbuf;
  size_t off_es_tab, off_esdec, off_force3, off_spec2, off_lptkeep, off_gate, off_gsteps, off_sched;
  size_t total;
};

// tile edge (16 cells, or the whole mesh when smaller), and the window halo
// of the adjoint's transposed FD gather (kernel reach 1 + FD reach)
int tile_edge(int n) { return n < 16 ? n : 16; }
int kernel_reach_of(int mak) { return mak == 4 ? 2 : 1; }  // mass-assignment stencil reach (mak.h)
int dipole_halo(int grad_order, int mak) { return kernel_reach_of(mak) + grad_order / 2; }
// block totals of the tile-count scan (1024 tiles per block), padded
int scan_np(long long n_tiles) { return (int)((n_tiles + 1023) / 1024 + 63) / 64 * 64; }

// half-spectrum row stride: n/2 + 1 complex, padded to 16 (one 128-byte line)
// from n = 32 so that column tiles read whole aligned lines
int spec_rs(int n) { int nh = n / 2 + 1; return n >= 32 ? (nh + 15) / 16 * 16 : nh; }
long long spec_elems(int n) { return (long long)n * n * spec_rs(n); }

Layout layout(const pm_ctx* c, bool adj) {
  Layout L{};
  const int B = c->cfg.batch;
  const long long N = (long long)c->cfg.n_p * c->cfg.n_p * c->cfg.n_p;
  const long long M = (long long)c->cfg.n_g * c->cfg.n_g * c->cfg.n_g;
  const int n = c->cfg.n_g, np = c->cfg.n_p;
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  L.off_tw = take(sizeof(float2) * c->Lmax);
  L.off_lap = take(sizeof(float) * n);
  L.off_win2 = take(sizeof(float) * n);
  L.off_amp = take(sizeof(float) * c->amp_tab.size());
  L.off_cic4 = take(sizeof(double) * n);
  L.off_disp = take(sizeof(float) * 3 * N * B);
  L.off_vel = take(sizeof(float) * 3 * N * B);
  L.off_w = take(sizeof(float) * N * B);
  L.off_xbar = adj ? take(sizeof(float) * 3 * N * B) : 0;
  L.off_vbar = adj ? take(sizeof(float) * 3 * N * B) : 0;
  L.off_mesh = take(sizeof(long long) * M * B);
  L.off_spec = take(sizeof(float2) * spec_elems(n) * B);
  L.off_phi = take(sizeof(float) * M * B);
  const int T = tile_edge(n);
  const long long nt = n / T, n_tiles = nt * nt * nt;
  const long long ts = (n_tiles + 1 + 63) / 64 * 64;
  L.off_key = take(sizeof(int32_t) * N * B);
  L.off_rank = take(sizeof(int32_t) * N * B);
  L.off_sorted = take(sizeof(int32_t) * N * B);
  L.off_count = take(sizeof(int32_t) * ts * B);
  L.off_offset = take(sizeof(int32_t) * ts * B);
  L.off_scanp = take(sizeof(int32_t) * scan_np(n_tiles) * B);
  const bool nufft = c->cfg.force == PM_FORCE_NUFFT;
  long long W = T + 2 * kernel_reach_of(c->cfg.mak);
  if (adj) W = std::max(W, (long long)T + 2 * dipole_halo(c->cfg.grad_order, c->cfg.mak));
  if (nufft) W = std::max(W, (long long)T + kEsHaloLo + kEsHaloHi);
  L.off_es_tab = take(sizeof(int32_t) * c->es_tab.size());
  L.off_esdec = take(sizeof(float) * n);
  L.off_lptkeep = take(sizeof(float) * n);
  L.off_gate = take(sizeof(int32_t) * kMaxBatch);
  L.off_gsteps = take(sizeof(int32_t) * kMaxBatch);
  L.off_sched = take(sizeof(float) * kSch * (size_t)kMaxSchedSteps * B);  // fixed: memory independent of n_steps
  L.off_force3 = nufft ? take(sizeof(float) * 3 * M * B) : 0;
  L.off_spec2 = (nufft || c->cfg.antialias) ? take(sizeof(float2) * spec_elems(n) * B) : 0;
  L.off_accbuf = c->cfg.antialias ? take(sizeof(float) * 6 * N * B) : 0;
  L.off_scratch = take(sizeof(long long) * W * W * W * n_tiles * B);
  L.off_u = adj ? take(sizeof(float) * 3 * N * B) : 0;
  L.off_umax = take(sizeof(float) * kMaxBatch);
  L.off_scale = take(sizeof(double) * 2 * kMaxBatch);
  L.off_icspec = take(sizeof(float2) * 4 * align_up(spec_elems(np)) * B);
  L.off_pk = take(sizeof(double) * 3 * (size_t)n * n * B);  // n_bins <= n
  L.off_dot = take(sizeof(double) * 256 * B);
  L.off_tdots = take(sizeof(double) * 2 * kMaxBatch);
  L.total = o;
  return L;
}

// Fourier-space 1D tables for the mesh multiplier and P(k), in FP64 on the host
void build_tables(pm_ctx* c) {
  const pm_config& cf = c->cfg;
  const int n = cf.n_g;
  c->Lmax = n;
  c->tw.resize(c->Lmax);
  for (int t = 0; t < c->Lmax; ++t) {
    double a = -2.0 * M_PI * t / c->Lmax;
    c->tw[t] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  c->lap.resize(n);
  c->win2.resize(n);
  c->cic4.resize(n);
  for (int i = 0; i < n; ++i) {
    int m = i < n / 2 ? i : i - n;
    double th = 2.0 * M_PI * m / n;
    double l;
    switch (cf.lap_order) {  // tab. derivative_kernels; order 2 with the sign of its stencil
      case 2: l = -2.0 * (1.0 - std::cos(th)); break;
      case 4: l = -(std::cos(2 * th) - 16.0 * std::cos(th) + 15.0) / 6.0; break;
      case 6: l = -(-2.0 * std::cos(3 * th) + 27.0 * std::cos(2 * th) - 270.0 * std::cos(th) + 245.0) / 90.0; break;
      default: l = -th * th;
    }
    c->lap[i] = (float)l;
    double h = 0.5 * th, sinc = (h == 0.0) ? 1.0 : std::sin(h) / h;
    double wv = std::pow(sinc, cf.mak);
    c->win2[i] = cf.deconvolve ? (float)(wv * wv) : 1.0f;
    c->cic4[i] = std::pow(sinc, 4);
  }
  // NUFFT: exponential-of-semicircle table (phi at t/4096 cells, 20-bit
  // integers, round half even) and the deconvolution 1/phi_hat^2 on the modes
  // strictly below the particle Nyquist mode (truncation: 0 elsewhere).
  // Device layout: row k (k = 0 .. 4096) holds the interpolation pairs
  // (phi_t, phi_t+1) at t = k, k + 4096, k + 8192, padded to 8 ints, so the
  // three nodes on one side of a particle come from one 32-byte row.
  if (cf.force == PM_FORCE_NUFFT) {
    const int w = cf.es_width, tabn = (w / 2) * kEsTabPerCell + 2;
    std::vector<int32_t> lin(tabn);
    for (int t = 0; t < tabn; ++t) {
      double x = (double)t / kEsTabPerCell, z = x / (0.5 * w);
      double phi = z < 1.0 ? std::exp(cf.es_beta * (std::sqrt(1.0 - z * z) - 1.0)) : 0.0;
      lin[t] = (int32_t)std::nearbyint(phi * (double)(1 << kWeightBits));
    }
    c->es_tab.assign((size_t)(kEsTabPerCell + 1) * 8, 0);
    for (int k = 0; k <= kEsTabPerCell; ++k)
      for (int m = 0; m < w / 2; ++m) {
        c->es_tab[8 * k + 2 * m] = lin[k + m * kEsTabPerCell];
        c->es_tab[8 * k + 2 * m + 1] = lin[k + m * kEsTabPerCell + 1];
      }
    c->esdec.assign(n, 0.f);
    for (int i = 0; i < n; ++i) {
      int m = i < n / 2 ? i : i - n;
      if (2 * std::abs(m) < cf.n_p) {
        double ph = es_phihat(2.0 * M_PI * m / n, w, cf.es_beta);
        c->esdec[i] = (float)(1.0 / (ph * ph));
      }
    }
  } else {
    c->es_tab.assign(4, 0);
    c->esdec.assign(n, 0.f);
  }
  // second-order LPT grid of 2 n_p points per axis (<= n): the modes of the
  // particle grid strictly below its Nyquist mode
  c->lptkeep.assign(n, 0.f);
  if (2 * cf.n_p <= n)
    for (int i = 0; i < 2 * cf.n_p; ++i) {
      const int m = i < cf.n_p ? i : i - 2 * cf.n_p;
      c->lptkeep[i] = 2 * std::abs(m) < cf.n_p ? 1.f : 0.f;
    }
  // IC multiplier on the particle grid: h_c = i m_c amp[|m|^2], with
  // amp = kf sqrt(P(k) n^3/L^3) / (k^2 D_ref dq) / n^3 (the 1/n^3 of the
  // normalised inverse DFT), zero at m = 0 and for |m| > n/2
  const int np = cf.n_p;
  const long long m2max = 3ll * (np / 2) * (np / 2);
  c->amp_tab.assign(m2max + 1, 0.f);
  const double kf = 2.0 * M_PI / cf.box, dq = cf.box / np;
  const double n3 = (double)np * np * np;
  for (long long m2 = 1; m2 <= m2max; ++m2) {
    if (4 * m2 > (long long)np * np) break;
    double k2 = kf * kf * m2, k = std::sqrt(k2);
    double P = spectrum_eval(cf, c->amp, k);
    c->amp_tab[m2] = (float)(kf * std::sqrt(P * n3 / (cf.box * cf.box * cf.box)) / (k2 * c->D_ref * dq) / n3);
  }
}

Geom make_geom(int n_p, int n_g, long long part_stride, long long mesh_stride, long long spec_stride) {
  Geom g{};
  g.n_p = n_p;
  g.n_g = n_g;
  g.log2_np = ilog2(n_p);
  g.log2_ng = ilog2(n_g);
  g.log2_r = g.log2_ng - g.log2_np;
  // lattice blocks that fill one mesh tile (tile edge min(16, n_g) cells)
  g.log2_pb = std::max(0, std::min(g.log2_np, ilog2(n_g < 16 ? n_g : 16) - g.log2_r));
  g.N = (long long)n_p * n_p * n_p;
  g.M = (long long)n_g * n_g * n_g;
  g.part_stride = part_stride;
  g.mesh_stride = mesh_stride;
  g.spec_stride = spec_stride;
  return g;
}

unsigned long long all_mask(int B) { return B >= 64 ? ~0ull : ((1ull << B) - 1); }

// --------------------------------------------------------------- FFT chains

// real mesh (int64 mass or float) -> spectrum, forward 3D (or up to y only)
// prune > 0: only the modes |m| < prune/2 per axis are needed afterwards, so
// the rows keep k_z < prune/2 and the y pass writes only the kept k_y
pm_status r2c_mesh(pm_ctx* c, const void* src, int src_mode, long long src_stride, double scale,
                   double shift, float2* dst, long long dst_stride, int n, bool do_x,
                   unsigned long long active, int prune = 0) {
  RowLaunch r{};
  r.n = n;
  r.rs = spec_rs(n);
  r.kz_lim = prune / 2;
  r.n_rows = (long long)n * n;
  r.batch = c->cfg.batch;
  r.inverse = false;
  r.src_mode = src_mode;
  r.src = src;
  r.src_stride = src_stride;
  r.dst = dst;
  r.dst_stride = dst_stride;
  r.tw = c->d_tw;
  r.tws_half = c->Lmax / (n / 2);
  r.tws_full = c->Lmax / n;
  r.scale = scale;
  r.shift = shift;
  r.stream = c->stream;
  r.active = active;
  r.gate = c->g.gate;
  KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(r));
  ColArgs a{};
  a.gate = c->g.gate;
  a.sched = c->g.sched;
  a.sched_steps = c->g.sched_steps;
  a.data = dst;
  a.slot_stride = dst_stride;
  a.n = n;
  a.nh = n / 2 + 1;
  a.rs = spec_rs(n);
  a.tw = c->d_tw;
  a.tws = c->Lmax / n;
  a.active = active;
  a.axis = 1;
  a.zlim = prune / 2;
  a.keep = prune;
  a.keep_out = prune > 0;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_FWD, c->cfg.batch, c->stream));
  if (do_x) {
    if (prune) return fail(c, PM_EINVAL, "pruned transform stops after the y pass");
    a.axis = 0;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_FWD, c->cfg.batch, c->stream));
  }
  return PM_OK;
}

// spectrum after the y pass -> x pass with the PM multiplier -> y inverse -> real
pm_status poisson_to_real(pm_ctx* c, const double* s, float* out, unsigned long long active) {
  const int n = c->cfg.n_g;
  ColArgs a{};
  a.data = c->spec;
  a.slot_stride = c->g.spec_stride;
  a.n = n;
  a.nh = n / 2 + 1;
  a.rs = spec_rs(n);
  a.tw = c->d_tw;
  a.tws = c->Lmax / n;
  a.lap = c->d_lap;
  a.win2 = c->d_win2;
  a.active = active;
  a.gate = c->g.gate;
  a.sched = c->g.sched;
  a.sched_steps = c->g.sched_steps;
  const double r = (double)(1 << c->g.log2_r);
  const double n3 = (double)n * n * n;
  for (int b = 0; b < c->cfg.batch; ++b) a.coef[b] = (float)(-s[b] / (r * n3));
  a.axis = 0;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_FUSED_H, c->cfg.batch, c->stream));
  a.axis = 1;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_INV, c->cfg.batch, c->stream));
  RowLaunch rl{};
  rl.n = n;
  rl.rs = spec_rs(n);
  rl.n_rows = (long long)n * n;
  rl.batch = c->cfg.batch;
  rl.inverse = true;
  rl.dst_mode = DST_F32;
  rl.src = c->spec;
  rl.src_stride = c->g.spec_stride;
  rl.dst = out;
  rl.dst_stride = c->g.mesh_stride;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (n / 2);
  rl.tws_full = c->Lmax / n;
  rl.scale = 1.0;
  rl.stream = c->stream;
  rl.active = active;
  rl.gate = c->g.gate;
  KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  return PM_OK;
}

// deposit of `disp` (optionally drifting by tau first) into the int64 mesh
// counting sort of the particles of `disp` by the tile of their home node
// (optionally drifting them by tau first); fills key/rank/sorted/offset
TileArgs tile_args(pm_ctx* c, float* disp, unsigned long long active);

pm_status bin(pm_ctx* c, float* disp, const float* vel_pre, const double* tau, int mak,
              unsigned long long active, int home_shift = 0) {
  KLAUNCH(c, PM_K_FILL, launch_fill(c->count, (long long)sizeof(int32_t) * c->ts * c->cfg.batch, c->stream));
  BinArgs b{};
  b.g = c->g;
  b.batch = c->cfg.batch;
  b.active = active;
  b.disp = disp;
  b.vel = vel_pre;
  for (int s = 0; s < c->cfg.batch; ++s) b.tau[s] = tau ? (float)tau[s] : 0.f;
  b.log2T = c->log2T;
  b.log2nt = c->log2nt;
  b.n_tiles = c->n_tiles;
  b.ts = c->ts;
  b.key = c->key;
  b.rank = c->rank;
  b.sorted = c->sorted;
  b.count = c->count;
  b.offset = c->offset;
  b.home_shift = home_shift;
  b.scan_partial = c->scan_partial;
  b.scan_np = scan_np(c->n_tiles);
  KLAUNCH(c, PM_K_BIN, launch_binning(b, mak, c->stream));
  if (home_shift == kEsAnchor) {  // ES binning: the spreads' LDS-bank order (in the rank buffer, free by now)
    TileArgs t = tile_args(c, disp, active);
    KLAUNCH(c, PM_K_MISC, launch_es_bank_order(t, c->rank, c->stream));
  }
  return PM_OK;
}

TileArgs tile_args(pm_ctx* c, float* disp, unsigned long long active) {
  TileArgs t{};
  t.g = c->g;
  t.batch = c->cfg.batch;
  t.active = active;
  t.T = c->T;
  t.log2T = c->log2T;
  t.log2nt = c->log2nt;
  t.n_tiles = c->n_tiles;
  t.ts = c->ts;
  t.sorted = c->sorted;
  t.offset = c->offset;
  t.bank = c->rank;  // written by an ES binning
  t.disp = disp;
  t.vel = c->vel;
  t.xbar = c->xbar;
  t.vbar = c->vbar;
  t.scratch = c->scratch;
  t.u_sorted = c->u_sorted;
  t.umax = c->umax;
  t.scale = c->scale;
  t.es_beta = (float)c->cfg.es_beta;
  return t;
}

AssembleArgs assemble_args(pm_ctx* c, int Rlo, int Rhi, void* out, unsigned long long active) {
  AssembleArgs a{};
  a.g = c->g;
  a.batch = c->cfg.batch;
  a.active = active;
  a.T = c->T;
  a.Rlo = Rlo;
  a.Rhi = Rhi;
  a.log2T = c->log2T;
  a.log2nt = c->log2nt;
  a.n_tiles = c->n_tiles;
  a.scratch = c->scratch;
  a.out = out;
  a.inv_scale = c->inv_scale;
  return a;
}

// fixed-point deposit of `disp` (after binning) into the int64 mesh
pm_status deposit(pm_ctx* c, float* disp, const float* vel_pre, const double* tau, int mak,
                  long long* mesh, unsigned long long active) {
  pm_status st = bin(c, disp, vel_pre, tau, mak, active);
  if (st) return st;
  TileArgs t = tile_args(c, disp, active);
  AssembleArgs a = assemble_args(c, kernel_reach_of(mak), kernel_reach_of(mak), mesh, active);
  KLAUNCH(c, PM_K_DEPOSIT, both(launch_tile(t, TK_DEPOSIT, mak, 0, c->stream), launch_assemble(a, false, c->stream)));
  return PM_OK;
}

pm_status nufft_meshes(pm_ctx* c, float* disp, const float* vel_pre, const double* tau, const double* s,
                       unsigned long long active);
pm_status nufft_force_chain(pm_ctx* c, const float* rho, const double* s, float* out, unsigned long long active);

// potential phi of the positions `disp` for the midpoint normalisation s
// (NUFFT: the three force meshes)
pm_status potential_interlaced(pm_ctx* c, float* disp, const float* vel_pre, const double* tau, const double* s,
                               unsigned long long active);

pm_status potential(pm_ctx* c, float* disp, const float* vel_pre, const double* tau, const double* s,
                    unsigned long long active) {
  if (c->cfg.force == PM_FORCE_NUFFT) return nufft_meshes(c, disp, vel_pre, tau, s, active);
  if (c->cfg.antialias) return potential_interlaced(c, disp, vel_pre, tau, s, active);
  const double N = (double)c->g.N, n3 = (double)c->g.M;
  // the halo sum of the int64 windows writes the FP32 contrast directly
  pm_status st = bin(c, disp, vel_pre, tau, c->cfg.mak, active);
  if (st) return st;
  TileArgs t = tile_args(c, disp, active);
  float* rho = reinterpret_cast<float*>(c->mesh);
  AssembleArgs as = assemble_args(c, kernel_reach_of(c->cfg.mak), kernel_reach_of(c->cfg.mak), rho, active);
  as.inv_scale = nullptr;
  as.scale = n3 / N / 4294967296.0;
  as.shift = 1.0;
  KLAUNCH(c, PM_K_DEPOSIT, both(launch_tile(t, TK_DEPOSIT, c->cfg.mak, 0, c->stream), launch_assemble(as, true, c->stream)));
  st = r2c_mesh(c, rho, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec, c->g.spec_stride, c->cfg.n_g, false, active);
  if (st) return st;
  return poisson_to_real(c, s, c->phi, active);
}

// x pass, y inverse and C2R of a half spectrum after its y pass (the plain
// PM multiplier: mode MODE_FUSED_H; interlaced: MODE_FUSED_IL with the second
// grid's x-transformed spectrum in `other`; MODE_INV: inverse only)
pm_status spectrum_to_real(pm_ctx* c, float2* spec, int mode, const double* s, float2* other, float* out,
                           unsigned long long active) {
  const int n = c->cfg.n_g;
  ColArgs a{};
  a.data = spec;
  a.slot_stride = c->g.spec_stride;
  a.n = n;
  a.nh = n / 2 + 1;
  a.rs = spec_rs(n);
  a.tw = c->d_tw;
  a.tws = c->Lmax / n;
  a.lap = c->d_lap;
  a.win2 = c->d_win2;
  a.active = active;
  a.src3 = other;
  a.dst3 = other;
  const double r = (double)(1 << c->g.log2_r);
  const double n3 = (double)n * n * n;
  for (int b = 0; b < c->cfg.batch; ++b) a.coef[b] = s ? (float)(-s[b] / (r * n3)) : 0.f;
  a.axis = 0;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, mode, c->cfg.batch, c->stream));
  a.axis = 1;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_INV, c->cfg.batch, c->stream));
  RowLaunch rl{};
  rl.n = n;
  rl.rs = spec_rs(n);
  rl.n_rows = (long long)n * n;
  rl.batch = c->cfg.batch;
  rl.inverse = true;
  rl.dst_mode = DST_F32;
  rl.src = spec;
  rl.src_stride = c->g.spec_stride;
  rl.dst = out;
  rl.dst_stride = c->g.mesh_stride;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (n / 2);
  rl.tws_full = c->Lmax / n;
  rl.scale = 1.0;
  rl.stream = c->stream;
  rl.active = active;
  KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  return PM_OK;
}

// Interlaced grids (antialias 1): the contrast of the particles and of the
// particles half a cell up the diagonal (fixed-point coordinate + 2^19 on
// every axis; the second grid's nodes sit half a cell down the diagonal),
// both transformed; the x pass of grid 1 forms (d1 + e^{i phi} d2)/2, applies
// the multiplier and hands H delta e^{-i phi} to grid 2; each grid's inverse
// gives its potential (phi on c->phi, the second in the mesh buffer behind
// the first grid's contrast).  The binning left behind is grid 2's.
pm_status potential_interlaced(pm_ctx* c, float* disp, const float* vel_pre, const double* tau, const double* s,
                               unsigned long long active) {
  const double N = (double)c->g.N, n3 = (double)c->g.M;
  const int kr = kernel_reach_of(c->cfg.mak);
  float* rho1 = reinterpret_cast<float*>(c->mesh);
  float* rho2 = rho1 + (long long)c->cfg.batch * c->g.M;
  for (int grid = 0; grid < 2; ++grid) {
    c->g.ushift = grid ? (1ll << (kFracBits - 1)) : 0;
    pm_status st = grid ? bin(c, disp, nullptr, nullptr, c->cfg.mak, active)
                        : bin(c, disp, vel_pre, tau, c->cfg.mak, active);
    if (st) { c->g.ushift = 0; return st; }
    TileArgs t = tile_args(c, disp, active);
    AssembleArgs as = assemble_args(c, kr, kr, grid ? rho2 : rho1, active);
    as.inv_scale = nullptr;
    as.scale = n3 / N / 4294967296.0;
    as.shift = 1.0;
    KLAUNCH(c, PM_K_DEPOSIT,
            both(launch_tile(t, TK_DEPOSIT, c->cfg.mak, 0, c->stream), launch_assemble(as, true, c->stream)));
    c->g.ushift = 0;
  }
  pm_status st = r2c_mesh(c, rho1, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec, c->g.spec_stride, c->cfg.n_g, false,
                          active);
  if (st) return st;
  st = r2c_mesh(c, rho2, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec2, c->g.spec_stride, c->cfg.n_g, true, active);
  if (st) return st;
  st = spectrum_to_real(c, c->spec, MODE_FUSED_IL, s, c->spec2, c->phi, active);
  if (st) return st;
  c->phi2 = rho2;
  return spectrum_to_real(c, c->spec2, MODE_INV, nullptr, nullptr, c->phi2, active);
}

// NUFFT force meshes: ES spreading (type 1) -> R2C -> truncate, deconvolve,
// i k_c s / k^2, deconvolve -> zero-padded C2R per component (type 2 grid)
pm_status nufft_meshes(pm_ctx* c, float* disp, const float* vel_pre, const double* tau, const double* s,
                       unsigned long long active) {
  pm_status st = bin(c, disp, vel_pre, tau, 2, active, kEsAnchor);  // first stencil node floor(u) - 2
  if (st) return st;
  TileArgs t = tile_args(c, disp, active);
  t.es_tab = c->d_es_tab;
  const int n = c->cfg.n_g, np = c->cfg.n_p;
  const double N = (double)c->g.N;
  const double ph0 = es_phihat(0.0, c->cfg.es_width, c->cfg.es_beta);
  const double mean = N * ph0 * ph0 * ph0 / (double)c->g.M;  // removes most of k = 0
  // FP32 partial sums per window (the force chain is FP32 from here on)
  t.win_f32 = 1;
  t.win_scale = 1.0 / 2147483648.0;  // the ES node weight is 2^31 at phi(0)^3
  float* rho = reinterpret_cast<float*>(c->mesh);
  AssembleArgs as = assemble_args(c, kEsHaloLo, kEsHaloHi, rho, active);
  as.slab_f32 = 1;
  as.shift = mean;
  KLAUNCH(c, PM_K_DEPOSIT, both(launch_tile_es(t, TK_ES_DEPOSIT, c->stream), launch_assemble(as, true, c->stream)));
  return nufft_force_chain(c, rho, s, c->force3, active);
}

// the three NUFFT force meshes (out: [B][3][M]) of a spread density rho
// ([B][M], slot stride M): R2C -> truncation, deconvolution, i k_c s / k^2
// (x pass) -> y inverse, C2R per component
pm_status nufft_force_chain(pm_ctx* c, const float* rho, const double* s, float* out, unsigned long long active) {
  const int n = c->cfg.n_g, np = c->cfg.n_p;
  const double N = (double)c->g.N;
  pm_status st = r2c_mesh(c, rho, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec, c->g.spec_stride, n, false, active, np);
  if (st) return st;
  ColArgs a{};
  a.data = c->spec;
  a.slot_stride = c->g.spec_stride;
  a.n = n;
  a.nh = n / 2 + 1;
  a.rs = spec_rs(n);
  a.tw = c->d_tw;
  a.tws = c->Lmax / n;
  a.active = active;
  a.esdec = c->d_esdec;
  a.n_p = np;
  a.dst3 = c->spec2;
  a.zlim = np / 2;  // kept modes |m| < n_p / 2 only
  a.keep = np;
  a.keep_outer = 1;
  const double np3 = (double)np * np * np;
  for (int b = 0; b < c->cfg.batch; ++b) a.coef[b] = (float)(s[b] / np3 * (np3 / N));
  for (int comp = 0; comp < 3; ++comp) {
    a.comp = comp;
    a.axis = 0;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_NUFFT_C, c->cfg.batch, c->stream));
    ColArgs y = a;
    y.data = c->spec2;
    y.axis = 1;
    y.keep_outer = 0;
    y.keep_in = 1;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(y, MODE_INV, c->cfg.batch, c->stream));
    RowLaunch rl{};
    rl.n = n;
    rl.rs = spec_rs(n);
    rl.kz_lim = np / 2;
    rl.n_rows = (long long)n * n;
    rl.batch = c->cfg.batch;
    rl.inverse = true;
    rl.dst_mode = DST_F32;
    rl.src = c->spec2;
    rl.src_stride = c->g.spec_stride;
    rl.dst = out + comp * c->g.M;
    rl.dst_stride = 3 * c->g.M;
    rl.tw = c->d_tw;
    rl.tws_half = c->Lmax / (n / 2);
    rl.tws_full = c->Lmax / n;
    rl.scale = 1.0;
    rl.stream = c->stream;
    rl.active = active;
    KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  }
  return PM_OK;
}

// gather of the force and kick/drift (or force only into acc_out)
pm_status kick(pm_ctx* c, float* disp, const double* alpha, const double* beta, const double* tau_post,
               float* acc_out, unsigned long long active) {
  TileArgs a = tile_args(c, disp, active);
  a.acc_out = acc_out;
  for (int b = 0; b < c->cfg.batch; ++b) {
    a.alpha[b] = alpha ? (float)alpha[b] : 1.f;
    a.beta[b] = beta ? (float)beta[b] : 0.f;
    a.tau[b] = tau_post ? (float)tau_post[b] : 0.f;
  }
  if (c->cfg.force == PM_FORCE_NUFFT) {
    a.mesh_in = c->force3;
    a.comp_stride = c->g.M;
    a.es_tab = c->d_es_tab;
    KLAUNCH(c, PM_K_GATHER_KICK, launch_tile_es(a, TK_ES_KICK, c->stream));
  } else if (c->cfg.antialias) {
    // grid 2 first, on its binning (the current one): its forces alone
    c->g.ushift = 1ll << (kFracBits - 1);
    TileArgs a2 = tile_args(c, disp, active);
    c->g.ushift = 0;
    a2.mesh_in = c->phi2;
    a2.acc_out = c->accbuf;
    KLAUNCH(c, PM_K_GATHER_KICK, launch_tile(a2, TK_KICK, c->cfg.mak, c->cfg.grad_order, c->stream));
    // grid 1 on the particles' own binning: the mean of the two gathers kicks
    if (pm_status st = bin(c, disp, nullptr, nullptr, c->cfg.mak, active)) return st;
    a.mesh_in = c->phi;
    a.acc_in = c->accbuf;
    KLAUNCH(c, PM_K_GATHER_KICK, launch_tile(a, TK_KICK, c->cfg.mak, c->cfg.grad_order, c->stream));
  } else {
    a.mesh_in = c->phi;
    KLAUNCH(c, PM_K_GATHER_KICK, launch_tile(a, TK_KICK, c->cfg.mak, c->cfg.grad_order, c->stream));
  }
  return PM_OK;
}

// Second-order LPT term (Sec. "Lagrangian perturbation theory", eq. LPT_L at
// n = 2, eq. helmholtz): the six derivative fields psi_{i,j} of the
// first-order displacement are evaluated on a grid of P = 2 n_p points per
// axis from their zero-padded spectra (twice the lattice resolves every
// product of two fields of the modes |m| < n_p/2, as Orszag's 3/2 rule does),
// mu = sum_{i<j} (psi_ii psi_jj - psi_ij^2) is formed there in the C2R
// epilogues, transformed back to the kept modes, and
// psi2_c = (3/7) i k_c mu / k^2 is evaluated at the lattice points (the even
// nodes of the P grid): Psi += D0^2 psi2, V += 2 D0 psi2.  Buffers (free
// while the initial state is built): the mesh holds A = running diagonal sum
// and mu (P^3 floats each per slot), spec and the tile scratch hold P-grid
// half spectra.
pm_status lpt2_from_mu(pm_ctx* c, const float* mu, long long mu_stride, float* vel, float* disp,
                       unsigned long long act);

pm_status lpt2(pm_ctx* c, unsigned long long act) {
  const int np = c->cfg.n_p, P = 2 * np, B = c->cfg.batch;
  const long long N = c->g.N, M = c->g.M;  // M = n_g^3 >= P^3
  float* A = reinterpret_cast<float*>(c->mesh);
  float2* fspec = c->spec;
  float2* cspec = reinterpret_cast<float2*>(c->scratch);
  ColArgs a{};
  a.n = P;
  a.nh = P / 2 + 1;
  a.rs = spec_rs(P);
  a.tw = c->d_tw;
  a.tws = c->Lmax / P;
  a.amp = c->d_amp;
  a.active = act;
  a.n_p = np;
  for (int b = 0; b < B; ++b)
    a.fac[b] = (float)(c->cfg.spectrum == PM_SPEC_BBKS ? c->slot_sigma8[b] / c->cfg.sigma8 : 1.0);
  a.src3 = c->icspec + 3 * c->icspec_comp;  // noise spectrum on the particle grid
  a.src_slot_stride = c->icspec_stride;
  a.src_rs = spec_rs(np);
  a.slot_stride = c->g.spec_stride;
  a.data = fspec;
  a.dst3 = fspec;
  a.axis = 0;
  a.zlim = np / 2;
  a.keep = np;
  a.keep_outer = 1;
  RowLaunch rl{};
  rl.n = P;
  rl.rs = spec_rs(P);
  rl.kz_lim = np / 2;
  rl.n_rows = (long long)P * P;
  rl.batch = B;
  rl.inverse = true;
  rl.src = fspec;
  rl.src_stride = c->g.spec_stride;
  rl.dst = A;
  rl.dst2 = A + M;
  rl.dst_stride = 2 * M;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (P / 2);
  rl.tws_full = c->Lmax / P;
  rl.scale = 1.0;
  rl.stream = c->stream;
  rl.active = act;
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  const int epi[6] = {DST_F32, DST_MU_AB, DST_MU_ACC, DST_MU_SQ, DST_MU_SQ, DST_MU_SQ};
  for (int q = 0; q < 6; ++q) {
    a.comp = pairs[q][0];
    a.comp2 = pairs[q][1];
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_LPT_D, B, c->stream));
    ColArgs y = a;
    y.axis = 1;
    y.keep_outer = 0;
    y.keep_in = 1;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(y, MODE_INV, B, c->stream));
    rl.dst_mode = epi[q];
    KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  }
  return lpt2_from_mu(c, A + M, 2 * M, c->vel, c->disp, act);
}

// psi2 = (3/7) i k / k^2 of the source mu (padded grid, slot stride
// mu_stride) on the kept modes, read off at the lattice points: adds
// 2 D0 psi2 to vel and D0^2 psi2 to disp (lattice-block order)
pm_status lpt2_from_mu(pm_ctx* c, const float* mu, long long mu_stride, float* vel, float* disp,
                       unsigned long long act) {
  const int np = c->cfg.n_p, P = 2 * np, B = c->cfg.batch;
  const long long N = c->g.N;
  float2* fspec = c->spec;
  float2* cspec = reinterpret_cast<float2*>(c->scratch);
  pm_status st = r2c_mesh(c, mu, SRC_F32, mu_stride, 1.0, 0.0, fspec, c->g.spec_stride, P, false, act, np);
  if (st) return st;
  RowLaunch rl{};
  rl.n = P;
  rl.rs = spec_rs(P);
  rl.kz_lim = np / 2;
  rl.n_rows = (long long)P * P;
  rl.batch = B;
  rl.inverse = true;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (P / 2);
  rl.tws_full = c->Lmax / P;
  rl.stream = c->stream;
  rl.active = act;
  rl.src_stride = c->g.spec_stride;
  ColArgs x{};
  x.data = fspec;
  x.dst3 = cspec;
  x.slot_stride = c->g.spec_stride;
  x.n = P;
  x.nh = P / 2 + 1;
  x.rs = spec_rs(P);
  x.tw = c->d_tw;
  x.tws = c->Lmax / P;
  x.esdec = c->d_lptkeep;  // truncation to the kept modes (no deconvolution)
  x.n_p = np;
  x.active = act;
  x.axis = 0;
  x.zlim = np / 2;
  x.keep = np;
  x.keep_outer = 1;
  // (3/7) i k_c / k^2 in lattice units; 1/P^3 takes the P-grid transform of mu
  // to the particle grid's normalised inverse
  for (int b = 0; b < B; ++b) x.coef[b] = (float)(3.0 / 7.0 / ((double)P * P * P));
  RowLaunch r2 = rl;
  r2.src = cspec;
  r2.dst_mode = DST_IC2;
  r2.dst_stride = 3 * N;
  r2.scale = 2.0 * c->D0 * c->vfac;
  r2.scale2 = c->D0 * c->D0;
  r2.ic_log2pb = c->g.log2_pb;
  for (int comp = 0; comp < 3; ++comp) {
    x.comp = comp;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(x, MODE_NUFFT_C, B, c->stream));
    ColArgs y = x;
    y.data = cspec;
    y.axis = 1;
    y.keep_outer = 0;
    y.keep_in = 1;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(y, MODE_INV, B, c->stream));
    r2.dst = vel + comp * N;
    r2.dst2 = disp + comp * N;
    KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(r2));
  }
  return PM_OK;
}

pm_status check_bound(pm_ctx* c) {
  if (!c) return PM_EINVAL;
  if (!c->bound) return fail(c, PM_ESTATE, "context not bound to a workspace");
  return PM_OK;
}

}  // namespace

// =========================================================== public calls

extern "C" {

pm_status pm_create(const pm_config* cfg, pm_ctx** out) {
  if (!cfg || !out) return PM_EINVAL;
  *out = nullptr;
  const pm_config& c = *cfg;
  if (!pow2(c.n_p) || c.n_p < 4 || c.n_p > 1024 || !pow2(c.n_g) || c.n_g < c.n_p || c.n_g > 1024 ||
      c.n_g / c.n_p > 4)
    return PM_EINVAL;
  if (c.box <= 0 || c.n_steps < 1 || c.a_start <= 0 || c.a_end <= c.a_start || c.batch < 1 ||
      c.batch > kMaxBatch || c.omega_m <= 0 || c.omega_m > 1)
    return PM_EINVAL;
  if (c.force == PM_FORCE_PM) {
    // PCS (mak 4) runs with FD2 / FD4: its FD6 windows would not fit a workgroup's LDS
    if ((c.mak < 2 || c.mak > 4) || (c.grad_order != 2 && c.grad_order != 4 && c.grad_order != 6) ||
        (c.mak == 4 && c.grad_order == 6) ||
        (c.lap_order != 0 && c.lap_order != 2 && c.lap_order != 4 && c.lap_order != 6))
      return PM_EINVAL;
  } else if (c.force == PM_FORCE_NUFFT) {
    // exact i k gradient and -k^2 (Sec. "Force evaluation"), width-6 ES kernel on
    // a grid upsampled by 2
    // (n_p >= 8: the pruned NUFFT passes run in the register FFT kernels)
    if (c.es_width != 6 || c.n_g != 2 * c.n_p || c.n_p < 8 || c.grad_order != 0 || c.lap_order != 0 ||
        !(c.es_beta > 0))
      return PM_EINVAL;
  } else {
    return PM_EINVAL;
  }
  if (c.spectrum != PM_SPEC_BBKS && c.spectrum != PM_SPEC_POWERLAW) return PM_EINVAL;
  // second-order LPT runs its products on a 2 n_p grid held in the mesh buffers
  // (pruned register FFT passes: n_p >= 8)
  if (c.lpt_order < 0 || c.lpt_order > 2 || (c.lpt_order == 2 && (c.n_g < 2 * c.n_p || c.n_p < 8)))
    return PM_EINVAL;
  if (c.stepper < 0 || c.stepper > 2 || c.time_var < 0 || c.time_var > 3) return PM_EINVAL;
  if (c.antialias < 0 || c.antialias > 1 || (c.antialias && (c.force != PM_FORCE_PM || c.n_g < 16)))
    return PM_EINVAL;
  pm_ctx* ctx = new (std::nothrow) pm_ctx();
  if (!ctx) return PM_ENOMEM;
  ctx->cfg = c;
  ctx->growth.solve(c.omega_m);
  ctx->table = step_table(ctx->growth, c.a_start, c.a_end, c.n_steps, c.stepper, c.time_var);
  ctx->D0 = ctx->growth.D_of_a(c.a_start);
  ctx->vfac = c.stepper == 2 ? ctx->growth.zeta(c.a_start) : 1.0;
  ctx->D_ref = ctx->growth.D_of_a(1.0);
  if (c.spectrum == PM_SPEC_BBKS)
    ctx->amp = bbks_amplitude(c.omega_m, c.h, c.n_s, c.sigma8);
  else
    ctx->amp = powerlaw_amplitude(c, ctx->D0, ctx->D_ref);
  ctx->slot_steps.assign(c.batch, c.n_steps);
  ctx->slot_sigma8.assign(c.batch, c.sigma8);
  ctx->slot_table.assign(c.batch, ctx->table);
  ctx->user_mask = all_mask(c.batch);
  build_tables(ctx);
  *out = ctx;
  return PM_OK;
}

size_t pm_workspace_bytes(const pm_ctx* ctx, int32_t with_adjoint) {
  if (!ctx) return 0;
  return layout(ctx, with_adjoint != 0).total;
}

pm_status pm_bind(pm_ctx* c, void* workspace, size_t bytes, int32_t with_adjoint, void* stream) {
  if (!c) return PM_EINVAL;
  Layout L = layout(c, with_adjoint != 0);
  if (!workspace || ((uintptr_t)workspace % kAlign)) return fail(c, PM_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < L.total) return fail(c, PM_ENOMEM, "workspace too small");
  char* ws = (char*)workspace;
  c->stream = (hipStream_t)stream;
  c->with_adj = with_adjoint != 0;
  HIPCHK(c, configure_tile_kernels());
  if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  ++c->gen;
  const int B = c->cfg.batch;
  c->d_tw = (float2*)(ws + L.off_tw);
  c->d_lap = (float*)(ws + L.off_lap);
  c->d_win2 = (float*)(ws + L.off_win2);
  c->d_amp = (float*)(ws + L.off_amp);
  c->d_cic4 = (double*)(ws + L.off_cic4);
  c->disp = (float*)(ws + L.off_disp);
  c->vel = (float*)(ws + L.off_vel);
  c->w = (float*)(ws + L.off_w);
  c->xbar = with_adjoint ? (float*)(ws + L.off_xbar) : nullptr;
  c->vbar = with_adjoint ? (float*)(ws + L.off_vbar) : nullptr;
  c->mesh = (long long*)(ws + L.off_mesh);
  c->spec = (float2*)(ws + L.off_spec);
  c->phi = (float*)(ws + L.off_phi);
  c->T = tile_edge(c->cfg.n_g);
  c->log2T = ilog2(c->T);
  c->log2nt = ilog2(c->cfg.n_g / c->T);
  c->n_tiles = 1 << (3 * c->log2nt);
  c->ts = (c->n_tiles + 1 + 63) / 64 * 64;
  c->key = (int32_t*)(ws + L.off_key);
  c->rank = (int32_t*)(ws + L.off_rank);
  c->sorted = (int32_t*)(ws + L.off_sorted);
  c->count = (int32_t*)(ws + L.off_count);
  c->offset = (int32_t*)(ws + L.off_offset);
  c->scan_partial = (int32_t*)(ws + L.off_scanp);
  c->scratch = (void*)(ws + L.off_scratch);
  c->u_sorted = with_adjoint ? (float*)(ws + L.off_u) : nullptr;
  c->d_es_tab = (int32_t*)(ws + L.off_es_tab);
  c->d_esdec = (float*)(ws + L.off_esdec);
  c->d_lptkeep = (float*)(ws + L.off_lptkeep);
  c->d_gate = (int32_t*)(ws + L.off_gate);
  c->d_gsteps = (int32_t*)(ws + L.off_gsteps);
  c->d_sched = (float*)(ws + L.off_sched);
  c->sched_dirty.assign(B, 1);
  ++c->bind_gen;
  c->force3 = c->cfg.force == PM_FORCE_NUFFT ? (float*)(ws + L.off_force3) : nullptr;
  c->spec2 = (c->cfg.force == PM_FORCE_NUFFT || c->cfg.antialias) ? (float2*)(ws + L.off_spec2) : nullptr;
  c->accbuf = c->cfg.antialias ? (float*)(ws + L.off_accbuf) : nullptr;
  c->umax = (float*)(ws + L.off_umax);
  c->scale = (double*)(ws + L.off_scale);
  c->inv_scale = c->scale + kMaxBatch;
  c->icspec = (float2*)(ws + L.off_icspec);
  c->pk_partial = (double*)(ws + L.off_pk);
  c->dot_partial = (double*)(ws + L.off_dot);
  c->tdots = (double*)(ws + L.off_tdots);
  const int n = c->cfg.n_g, np = c->cfg.n_p;
  c->icspec_comp = (long long)(align_up(spec_elems(np)));
  c->icspec_stride = 4 * c->icspec_comp;
  const long long N = (long long)np * np * np, M = (long long)n * n * n;
  c->g = make_geom(np, n, 3 * N, M, spec_elems(n));
  c->gp = make_geom(np, np, 3 * N, N, c->icspec_stride);
  (void)B;
  HIPCHK(c, hipMemcpyAsync(c->d_tw, c->tw.data(), sizeof(float2) * c->tw.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_lap, c->lap.data(), sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_win2, c->win2.data(), sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_amp, c->amp_tab.data(), sizeof(float) * c->amp_tab.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_cic4, c->cic4.data(), sizeof(double) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_es_tab, c->es_tab.data(), sizeof(int32_t) * c->es_tab.size(), hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_esdec, c->esdec.data(), sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->d_lptkeep, c->lptkeep.data(), sizeof(float) * n, hipMemcpyHostToDevice, c->stream));
  {
    GateSet gs{};
    gs.batch = B;
    for (int b = 0; b < B; ++b) gs.k[b] = -1;
    HIPCHK(c, launch_set_gate(c->d_gate, gs, c->stream));
  }
  // host tables must outlive the copies: wait for them here (bind is not on the hot path)
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->bound = true;
  c->ics_done = c->ran = false;
  return PM_OK;
}

pm_status pm_schedule(const pm_ctx* c, int32_t slot, double* out) {
  if (!c || !out || slot < 0 || slot >= c->cfg.batch) return PM_EINVAL;
  const auto& T = c->slot_table[slot];
  for (size_t n = 0; n < T.size(); ++n) {
    const StepCoef& s = T[n];
    double row[8] = {s.D_n, s.D_half, s.D_np1, s.alpha, s.beta, s.tau1, s.tau2, s.s};
    std::memcpy(out + 8 * n, row, sizeof(row));
  }
  return PM_OK;
}

pm_status pm_describe(const pm_ctx* c, double* out) {
  if (!c || !out) return PM_EINVAL;
  out[0] = c->D0;
  out[1] = c->D_ref;
  out[2] = c->amp;
  return PM_OK;
}

pm_status pm_set_active(pm_ctx* c, uint64_t mask) {
  if (!c) return PM_EINVAL;
  if (!mask || (mask & ~all_mask(c->cfg.batch))) return fail(c, PM_EINVAL, "slot mask empty or beyond the batch");
  if (mask != c->user_mask) ++c->gen;
  c->user_mask = mask;
  return PM_OK;
}

pm_status pm_use_graphs(pm_ctx* c, int32_t enable) {
  if (!c) return PM_EINVAL;
  c->use_graph = enable != 0;
  return PM_OK;
}

pm_status pm_profile(pm_ctx* c, int32_t on) {
  if (!c) return PM_EINVAL;
  c->prof = on != 0;
  return PM_OK;
}

pm_status pm_kernel_times(pm_ctx* c, double* ms, int64_t* launches) {
  if (!c || !ms || !launches) return PM_EINVAL;
  if (!c->pending.empty()) HIPCHK(c, hipStreamSynchronize(c->stream));
  for (auto& p : c->pending) {
    float t = 0.f;
    if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) {
      c->prof_ms[p.cls] += t;
      c->prof_n[p.cls] += 1;
    }
    c->pool.push_back(p.a);
    c->pool.push_back(p.b);
  }
  c->pending.clear();
  for (int k = 0; k < PM_K_COUNT; ++k) {
    ms[k] = c->prof_ms[k];
    launches[k] = c->prof_n[k];
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return PM_OK;
}

pm_status pm_destroy(pm_ctx* c) {
  delete c;
  return PM_OK;
}

const char* pm_last_error(const pm_ctx* c) { return c ? c->err.c_str() : "null context"; }

pm_status pm_set_slot_params(pm_ctx* c, const int32_t* n_steps, const double* sigma8) {
  if (!c) return PM_EINVAL;
  for (int b = 0; b < c->cfg.batch; ++b) {
    if (n_steps && (n_steps[b] < 1 || n_steps[b] > c->cfg.n_steps))
      return fail(c, PM_EINVAL, "slot n_steps out of range");
    if (sigma8 && !(sigma8[b] > 0)) return fail(c, PM_EINVAL, "sigma8 must be positive");
  }
  // the run graph bakes in the per-slot schedules (not sigma8, which only the
  // initial conditions read): rebuild it only when a step count changes
  for (int b = 0; b < c->cfg.batch; ++b) {
    if (n_steps && n_steps[b] != c->slot_steps[b]) {
      if ((int)c->sched_dirty.size() == c->cfg.batch) c->sched_dirty[b] = 1;
      c->slot_steps[b] = n_steps[b];
      c->slot_table[b] = step_table(c->growth, c->cfg.a_start, c->cfg.a_end, n_steps[b], c->cfg.stepper,
                                    c->cfg.time_var);
      ++c->gen;
    }
    if (sigma8) c->slot_sigma8[b] = sigma8[b];
  }
  return PM_OK;
}

static pm_status ic_chain(pm_ctx* c, const float* w, float* disp, float* vel, unsigned long long act);

pm_status pm_init_ics(pm_ctx* c, const uint64_t* seeds, const float* w_in, float* w_out) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!seeds && !w_in) return fail(c, PM_EINVAL, "need seeds or w_in");
  const int B = c->cfg.batch, np = c->cfg.n_p;
  const long long N = c->g.N;
  const unsigned long long act = c->user_mask;
  if (w_in) {
    for (int b = 0; b < B; ++b)
      if ((act >> b) & 1ull)
        HIPCHK(c, hipMemcpyAsync(c->w + b * N, w_in + b * N, sizeof(float) * N, hipMemcpyDeviceToDevice, c->stream));
  } else
    KLAUNCH(c, PM_K_MISC, launch_white_noise(c->w, N, N, B, seeds, act, c->stream));
  if (pm_status st = ic_chain(c, c->w, c->disp, c->vel, act)) return st;
  if (c->cfg.lpt_order == 2)
    if (pm_status st2 = lpt2(c, act)) return st2;
  if (w_out)
    for (int b = 0; b < B; ++b)
      if ((act >> b) & 1ull)
        HIPCHK(c, hipMemcpyAsync(w_out + b * N, c->w + b * N, sizeof(float) * N, hipMemcpyDeviceToDevice, c->stream));
  c->ics_done = true;
  c->ran = false;
  return PM_OK;
}

// Zel'dovich state from white noise w ([B][N], lattice order): Psi = D_start
// psi into disp, V = psi into vel (lattice blocks); psi = IDFT(h_c DFT(w))
static pm_status ic_chain(pm_ctx* c, const float* w, float* disp, float* vel, unsigned long long act) {
  const int B = c->cfg.batch, np = c->cfg.n_p;
  const long long N = c->g.N;
  float2* wspec = c->icspec + 3 * c->icspec_comp;
  pm_status st = r2c_mesh(c, w, SRC_F32, N, 1.0, 0.0, wspec, c->icspec_stride, np, true, act);
  if (st) return st;
  ColArgs a{};
  a.data = wspec;
  a.slot_stride = c->icspec_stride;
  a.n = np;
  a.nh = np / 2 + 1;
  a.rs = spec_rs(np);
  a.tw = c->d_tw;
  a.tws = c->Lmax / np;
  a.amp = c->d_amp;
  a.active = act;
  for (int b = 0; b < B; ++b)
    a.fac[b] = (float)(c->cfg.spectrum == PM_SPEC_BBKS ? c->slot_sigma8[b] / c->cfg.sigma8 : 1.0);
  for (int comp = 0; comp < 3; ++comp) {
    float2* out = c->icspec + comp * c->icspec_comp;
    a.axis = 0;
    a.comp = comp;
    a.dst3 = out;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_IC_C, B, c->stream));
    ColArgs y = a;
    y.data = out;
    y.axis = 1;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(y, MODE_INV, B, c->stream));
    RowLaunch rl{};
    rl.n = np;
    rl.rs = spec_rs(np);
    rl.n_rows = (long long)np * np;
    rl.batch = B;
    rl.inverse = true;
    rl.dst_mode = DST_IC;
    rl.src = out;
    rl.src_stride = c->icspec_stride;
    rl.dst = vel + comp * N;
    rl.dst2 = disp + comp * N;
    rl.dst_stride = 3 * N;
    rl.tw = c->d_tw;
    rl.tws_half = c->Lmax / (np / 2);
    rl.tws_full = c->Lmax / np;
    rl.scale = c->vfac;  // V = vfac psi, Psi = (D0 / vfac) V
    rl.scale2 = c->D0 / c->vfac;
    rl.ic_log2pb = c->g.log2_pb;
    rl.stream = c->stream;
    rl.active = act;
    KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  }
  return PM_OK;
}

static pm_status step_common(pm_ctx* c, const double* tau_pre, bool pre_drift, const double* s,
                             const double* alpha, const double* beta, const double* tau_post,
                             unsigned long long active) {
  pm_status st = potential(c, c->disp, pre_drift ? c->vel : nullptr, tau_pre, s, active);
  if (st) return st;
  return kick(c, c->disp, alpha, beta, tau_post, nullptr, active);
}

pm_status pm_step(pm_ctx* c, const int32_t* step_index) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!c->ics_done) return fail(c, PM_ESTATE, "pm_step before pm_init_ics");
  if (!step_index) return PM_EINVAL;
  const int B = c->cfg.batch;
  std::vector<double> tp(B, 0), s(B, 1), al(B, 1), be(B, 0), tq(B, 0);
  unsigned long long act = 0;
  for (int b = 0; b < B; ++b) {
    int k = step_index[b];
    if (k < 0) continue;
    if (k >= c->slot_steps[b]) return fail(c, PM_EINVAL, "step index out of range");
    const StepCoef& sc = c->slot_table[b][k];
    tp[b] = sc.tau1; s[b] = sc.s; al[b] = sc.alpha; be[b] = sc.beta; tq[b] = sc.tau2;
    act |= 1ull << b;
  }
  act &= c->user_mask;
  if (!act) return PM_OK;
  pm_status st = step_common(c, tp.data(), true, s.data(), al.data(), be.data(), tq.data(), act);
  if (st) return st;
  c->ran = true;
  return PM_OK;
}

// ---- device-indexed steps: every slot's step index and step scalars live in
// device memory, so one captured graph advances any mix of slots
static pm_status device_steps_ok(pm_ctx* c) {
  if (pm_status st = check_bound(c)) return st;
  if (c->cfg.force != PM_FORCE_PM)
    return fail(c, PM_EUNSUPPORTED, "device-indexed steps cover the PM force");
  if (c->cfg.n_steps > kMaxSchedSteps) return fail(c, PM_EUNSUPPORTED, "device schedules hold at most 96 steps");
  if (c->cfg.antialias) return fail(c, PM_EUNSUPPORTED, "device-indexed steps cover the single-grid force");
  return PM_OK;
}

// upload the schedule rows of slots whose step count changed (stream-ordered,
// by value)
static pm_status upload_schedules(pm_ctx* c) {
  const double r = (double)(1 << c->g.log2_r), n3 = (double)c->g.M;
  for (int b = 0; b < c->cfg.batch; ++b) {
    if (!c->sched_dirty[b]) continue;
    SchedRows rows{};
    rows.n = c->slot_steps[b];
    rows.slot = b;
    rows.stride = kMaxSchedSteps;
    for (int k = 0; k < rows.n; ++k) {
      const StepCoef& sc = c->slot_table[b][k];
      float* v = rows.v + k * kSch;
      v[kSchTau1] = (float)sc.tau1;
      v[kSchAlpha] = (float)sc.alpha;
      v[kSchBeta] = (float)sc.beta;
      v[kSchTau2] = (float)sc.tau2;
      v[kSchCoef] = (float)(-sc.s / (r * n3));  // the PM multiplier's coefficient, as poisson_to_real forms it
    }
    KLAUNCH(c, PM_K_MISC, launch_set_sched(c->d_sched, c->d_gsteps, rows, c->stream));
    c->sched_dirty[b] = 0;
  }
  return PM_OK;
}

pm_status pm_set_step_index(pm_ctx* c, const int32_t* step_index) {
  if (pm_status st = device_steps_ok(c)) return st;
  if (!step_index) return PM_EINVAL;
  GateSet g{};
  g.batch = c->cfg.batch;
  for (int b = 0; b < g.batch; ++b) {
    const int k = step_index[b];
    if (k < -2 || k >= c->slot_steps[b]) return fail(c, PM_EINVAL, "step index out of range");
    g.k[b] = k;
  }
  if (pm_status st = upload_schedules(c)) return st;
  KLAUNCH(c, PM_K_MISC, launch_set_gate(c->d_gate, g, c->stream));
  return PM_OK;
}

// one step of every slot at its device step index, then the indices advance
static pm_status device_step_launches(pm_ctx* c) {
  const int B = c->cfg.batch;
  std::vector<double> unused(B, 0.0);
  c->g.gate = c->d_gate;
  c->g.sched = c->d_sched;
  c->g.sched_steps = kMaxSchedSteps;
  pm_status st = step_common(c, unused.data(), true, unused.data(), unused.data(), unused.data(), unused.data(),
                             all_mask(B));
  c->g.gate = nullptr;
  c->g.sched = nullptr;
  c->g.sched_steps = 0;
  if (st) return st;
  KLAUNCH(c, PM_K_MISC, launch_advance_gate(c->d_gate, c->d_gsteps, B, c->stream));
  return PM_OK;
}

pm_status pm_step_device(pm_ctx* c) {
  if (c) c->tangent_valid = false;
  if (pm_status st = device_steps_ok(c)) return st;
  if (!c->ics_done) return fail(c, PM_ESTATE, "pm_step_device before pm_init_ics");
  if (pm_status st = upload_schedules(c)) return st;
  if (!c->use_graph || c->prof) {
    if (pm_status st = device_step_launches(c)) return st;
  } else {
    if (!c->step_exec || c->step_bind_gen != c->bind_gen) {
      if (c->step_exec) {
        HIPCHK(c, hipGraphExecDestroy(c->step_exec));
        c->step_exec = nullptr;
      }
      hipStream_t user = c->stream;
      c->stream = c->cap;
      HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
      pm_status st = device_step_launches(c);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap, &g);
      c->stream = user;
      if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(c, PM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&c->step_exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) {
        c->step_exec = nullptr;
        return fail(c, PM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
      c->step_bind_gen = c->bind_gen;
    }
    HIPCHK(c, hipGraphLaunch(c->step_exec, c->stream));
  }
  c->ran = true;
  return PM_OK;
}

pm_status pm_get_step_index(pm_ctx* c, int32_t* step_index) {
  if (pm_status st = device_steps_ok(c)) return st;
  if (!step_index) return PM_EINVAL;
  HIPCHK(c, hipMemcpyAsync(step_index, c->d_gate, sizeof(int32_t) * c->cfg.batch, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return PM_OK;
}

static pm_status run_steps(pm_ctx* c);

pm_status pm_run(pm_ctx* c) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!c->ics_done) return fail(c, PM_ESTATE, "pm_run before pm_init_ics");
  if (!c->use_graph || c->prof) {
    pm_status st = run_steps(c);
    if (st) return st;
  } else {
    if (!c->run_exec || c->run_gen != c->gen) {
      if (c->run_exec) {
        HIPCHK(c, hipGraphExecDestroy(c->run_exec));
        c->run_exec = nullptr;
      }
      // capture on the context's own stream (the bound one may be the null
      // stream); nothing runs during capture
      hipStream_t user = c->stream;
      c->stream = c->cap;
      HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
      pm_status st = run_steps(c);
      hipGraph_t g = nullptr;
      hipError_t e = hipStreamEndCapture(c->cap, &g);
      c->stream = user;
      if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
      }
      if (e != hipSuccess) return fail(c, PM_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
      e = hipGraphInstantiate(&c->run_exec, g, nullptr, nullptr, 0);
      hipGraphDestroy(g);
      if (e != hipSuccess) {
        c->run_exec = nullptr;
        return fail(c, PM_EHIP, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
      c->run_gen = c->gen;
    }
    HIPCHK(c, hipGraphLaunch(c->run_exec, c->stream));
  }
  c->ran = true;
  return PM_OK;
}

// every step of the run: slot b stops after its own step count
static pm_status run_steps(pm_ctx* c) {
  const int B = c->cfg.batch;
  int nmax = 0;
  for (int b = 0; b < B; ++b) nmax = std::max(nmax, c->slot_steps[b]);
  for (int n = 0; n < nmax; ++n) {
    std::vector<double> tp(B, 0), s(B, 1), al(B, 1), be(B, 0), tq(B, 0);
    unsigned long long act = 0;
    for (int b = 0; b < B; ++b) {
      if (n >= c->slot_steps[b]) continue;
      const auto& T = c->slot_table[b];
      tp[b] = T[n].tau1;
      s[b] = T[n].s; al[b] = T[n].alpha; be[b] = T[n].beta;
      tq[b] = T[n].tau2;
      act |= 1ull << b;
    }
    act &= c->user_mask;
    if (!act) continue;
    // the same launches as pm_step(n): the first drift rides on the binning
    // pass, the second on the gather-kick, so a run equals its steps bit for
    // bit (and a slot served step by step equals a run)
    pm_status st = step_common(c, tp.data(), true, s.data(), al.data(), be.data(), tq.data(), act);
    if (st) return st;
  }
  return PM_OK;
}

// one reverse step of the NUFFT force after its force meshes are rebuilt at
// X^{n+1/2}: reverse kick with the direct position gradient; the mesh term
// sum_c G_c^T (spread of u_c) as one spread of u . grad phi (its transform
// is -i k_c times that of the spread of u_c), R2C, the real remainder of the
// multiplier, C2R; its gradient gather (the transposed spreading) fused with
// the reverse drift
pm_status kick_dot(pm_ctx* c, double* out, unsigned long long act);

pm_status nufft_adjoint_step(pm_ctx* c, const double* s, const double* alpha, const double* beta,
                             const double* tau, unsigned long long act, int parts, double* kdot) {
  const int B = c->cfg.batch, ng = c->cfg.n_g;
  const long long N = c->g.N, M = c->g.M;
  TileArgs k = tile_args(c, c->disp, act);
  k.mesh_in = c->force3;
  k.comp_stride = M;
  k.es_tab = c->d_es_tab;
  for (int b = 0; b < B; ++b) {
    k.alpha[b] = (float)alpha[b];
    k.beta[b] = (float)beta[b];
  }
  KLAUNCH(c, PM_K_ADJ_KICK, launch_tile_es(k, TK_ES_ADJ_KICK, c->stream));
  if (pm_status st = kick_dot(c, kdot, act)) return st;
  if (!(parts & 1))
    KLAUNCH(c, PM_K_FILL, launch_fill(c->xbar, (long long)sizeof(float) * 3 * N * B, c->stream));
  if (!(parts & 2)) return PM_OK;
  // every node value sum_c u_c d/du_c phi3 is bounded by 3 max|u| per
  // particle (|phi| <= 1, |phi'| < 1 cell^-1)
  KLAUNCH(c, PM_K_MISC, launch_dipole_scale((const unsigned int*)c->umax, c->scale, c->inv_scale, 3.0 * (double)N,
                                            3.0, B, c->stream));
  float* d = reinterpret_cast<float*>(c->mesh);
  k.win_f32 = 1;  // FP32 partial sums at the slot's inverse scale
  k.win_scale = 0.0;
  k.inv_scale = c->inv_scale;
  AssembleArgs as = assemble_args(c, kEsHaloLo, kEsHaloHi, d, act);
  as.slab_f32 = 1;
  as.shift = 0.0;
  KLAUNCH(c, PM_K_DIPOLE, both(launch_tile_es(k, TK_ES_DIPOLE, c->stream), launch_assemble(as, true, c->stream)));
  pm_status st = r2c_mesh(c, d, SRC_F32, M, 1.0, 0.0, c->spec, c->g.spec_stride, ng, false, act, c->cfg.n_p);
  if (st) return st;
  // x pass: forward, real multiplier (n_f / n_p) (s / N) / (k^2 Phi^2), inverse
  ColArgs x{};
  x.data = c->spec;
  x.dst3 = c->spec2;
  x.slot_stride = c->g.spec_stride;
  x.n = ng;
  x.nh = ng / 2 + 1;
  x.rs = spec_rs(ng);
  x.tw = c->d_tw;
  x.tws = c->Lmax / ng;
  x.active = act;
  x.esdec = c->d_esdec;
  x.n_p = c->cfg.n_p;
  x.axis = 0;
  x.zlim = c->cfg.n_p / 2;
  x.keep = c->cfg.n_p;
  x.keep_outer = 1;
  for (int b = 0; b < B; ++b) x.coef[b] = (float)(s[b] / (double)N * ((double)ng / c->cfg.n_p));
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(x, MODE_NUFFT_ADJ, B, c->stream));
  ColArgs y = x;
  y.data = c->spec2;
  y.axis = 1;
  y.keep_outer = 0;
  y.keep_in = 1;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(y, MODE_INV, B, c->stream));
  RowLaunch rl{};
  rl.n = ng;
  rl.rs = spec_rs(ng);
  rl.kz_lim = c->cfg.n_p / 2;
  rl.n_rows = (long long)ng * ng;
  rl.batch = B;
  rl.inverse = true;
  rl.dst_mode = DST_F32;
  rl.src = c->spec2;
  rl.src_stride = c->g.spec_stride;
  rl.dst = c->phi;
  rl.dst_stride = c->g.mesh_stride;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (ng / 2);
  rl.tws_full = c->Lmax / ng;
  rl.scale = 1.0;
  rl.stream = c->stream;
  rl.active = act;
  KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  TileArgs dr = tile_args(c, c->disp, act);
  dr.mesh_in = c->phi;
  dr.es_tab = c->d_es_tab;
  for (int b = 0; b < B; ++b) {
    dr.coef[b] = 1.f;
    dr.tau[b] = (float)tau[b];
  }
  KLAUNCH(c, PM_K_ADJ_DRIFT, launch_tile_es(dr, TK_ES_ADJ_DRIFT, c->stream));
  return PM_OK;
}

// One reverse step after the force of X^{n+1/2} was rebuilt (particles binned):
// reverse kick V = (V - beta A)/alpha with the direct X_bar term, V_bar =
// alpha V_bar, u = beta V_bar; the mesh path of the force VJP; the
// scatter-w.r.t.-positions term with the reverse drift by tau.  parts: bit 0
// keeps the direct term, bit 1 runs the mesh path (the force-VJP test hook
// separates them; the adjoint uses both).
// dot of V_bar and V right after the adjoint kick (temporal adjoints)
pm_status kick_dot(pm_ctx* c, double* out, unsigned long long act) {
  if (!out) return PM_OK;
  std::vector<double> ones(c->cfg.batch, 1.0);
  KLAUNCH(c, PM_K_MISC, launch_dot(c->vbar, c->vel, 3 * c->g.N, 3 * c->g.N, c->cfg.batch, c->dot_partial, out,
                                   ones.data(), act, c->stream));
  return PM_OK;
}

pm_status reverse_force_step_interlaced(pm_ctx* c, const double* s, const double* alpha, const double* beta,
                                        const double* tau, unsigned long long act, int parts, double* kdot);

pm_status reverse_force_step(pm_ctx* c, const double* s, const double* alpha, const double* beta,
                             const double* tau, unsigned long long act, int parts, double* kdot = nullptr) {
  KLAUNCH(c, PM_K_FILL, launch_fill(c->umax, (long long)sizeof(float) * kMaxBatch, c->stream));
  if (c->cfg.force == PM_FORCE_NUFFT) return nufft_adjoint_step(c, s, alpha, beta, tau, act, parts, kdot);
  if (c->cfg.antialias) return reverse_force_step_interlaced(c, s, alpha, beta, tau, act, parts, kdot);
  const int B = c->cfg.batch;
  const long long N = c->g.N, M = c->g.M;
  const double mfac = (double)M / (double)N;
  const int ord = c->cfg.grad_order, mak = c->cfg.mak;
  // sum |c_s| of the FD stencil: bounds the transposed gather per unit |u|
  const double fd_l1 = ord == 2 ? 1.0 : (ord == 4 ? 1.5 : 110.0 / 60.0);
  TileArgs k = tile_args(c, c->disp, act);
  k.mesh_in = c->phi;
  for (int b = 0; b < B; ++b) {
    k.alpha[b] = (float)alpha[b];
    k.beta[b] = (float)beta[b];
  }
  KLAUNCH(c, PM_K_ADJ_KICK, launch_tile(k, TK_ADJ_KICK, mak, ord, c->stream));
  if (pm_status st = kick_dot(c, kdot, act)) return st;
  if (!(parts & 1))
    KLAUNCH(c, PM_K_FILL, launch_fill(c->xbar, (long long)sizeof(float) * 3 * N * B, c->stream));
  if (!(parts & 2)) return PM_OK;
  // mesh cotangent of the force: transposed FD gather in fixed point
  KLAUNCH(c, PM_K_MISC, launch_dipole_scale((const unsigned int*)c->umax, c->scale, c->inv_scale,
                                            3.0 * fd_l1 * (double)N, fd_l1, B, c->stream));
  // transposed multiplier (H is real and even)
  float* d = reinterpret_cast<float*>(c->mesh);
  AssembleArgs as = assemble_args(c, dipole_halo(ord, mak), dipole_halo(ord, mak), d, act);
  KLAUNCH(c, PM_K_DIPOLE, both(launch_tile(k, TK_DIPOLE, mak, ord, c->stream), launch_assemble(as, true, c->stream)));
  pm_status st = r2c_mesh(c, d, SRC_F32, M, 1.0, 0.0, c->spec, c->g.spec_stride, c->cfg.n_g, false, act);
  if (st) return st;
  st = poisson_to_real(c, s, c->phi, act);
  if (st) return st;
  TileArgs dr = tile_args(c, c->disp, act);
  dr.mesh_in = c->phi;
  for (int b = 0; b < B; ++b) {
    dr.coef[b] = (float)mfac;
    dr.tau[b] = (float)tau[b];
  }
  KLAUNCH(c, PM_K_ADJ_DRIFT, launch_tile(dr, TK_ADJ_DRIFT, mak, ord, c->stream));
  return PM_OK;
}

// The reverse step through interlaced grids (the force averages two grids,
// the second at the positions + (1/2, 1/2, 1/2) cells): every term of the
// force VJP is the mean of the two grids' terms.  The mesh cotangents of the
// two deposits come from the transposed gathers of u on each grid through the
// same two-grid chain as the forward force (the transposed multiplier of grid
// 1 with the phase is that of grid 2 with the conjugate phase).  The passes
// that need the other grid's binning run first and leave their terms in the
// per-particle buffer; the binning left behind is the second grid's.
pm_status reverse_force_step_interlaced(pm_ctx* c, const double* s, const double* alpha, const double* beta,
                                        const double* tau, unsigned long long act, int parts, double* kdot) {
  const int B = c->cfg.batch;
  const long long N = c->g.N, M = c->g.M;
  const double mfac = (double)M / (double)N;
  const int ord = c->cfg.grad_order, mak = c->cfg.mak;
  const double fd_l1 = ord == 2 ? 1.0 : (ord == 4 ? 1.5 : 110.0 / 60.0);
  const long long half = 1ll << (kFracBits - 1);
  float* d1 = reinterpret_cast<float*>(c->mesh);
  float* d2 = d1 + (long long)B * M;  // the second grid's potential, then its cotangents
  auto args = [&](long long ushift) {
    c->g.ushift = ushift;
    TileArgs k = tile_args(c, c->disp, act);
    c->g.ushift = 0;
    for (int b = 0; b < B; ++b) {
      k.alpha[b] = (float)alpha[b];
      k.beta[b] = (float)beta[b];
      k.coef[b] = (float)mfac;
      k.tau[b] = (float)tau[b];
    }
    return k;
  };
  auto dipole = [&](const TileArgs& k, float* out) -> pm_status {
    AssembleArgs as = assemble_args(c, dipole_halo(ord, mak), dipole_halo(ord, mak), out, act);
    KLAUNCH(c, PM_K_DIPOLE,
            both(launch_tile(k, TK_DIPOLE, mak, ord, c->stream), launch_assemble(as, true, c->stream)));
    return PM_OK;
  };
  // second grid (its binning is current): force and direct term, u in its order
  TileArgs k2 = args(half);
  k2.mesh_in = c->phi2;
  k2.il_out = c->accbuf;
  KLAUNCH(c, PM_K_ADJ_KICK, launch_tile(k2, TK_ADJ_KICK, mak, ord, c->stream));
  if (parts & 2) {
    KLAUNCH(c, PM_K_MISC, launch_dipole_scale((const unsigned int*)c->umax, c->scale, c->inv_scale,
                                              3.0 * fd_l1 * (double)N, fd_l1, B, c->stream));
    if (pm_status st = dipole(k2, d2)) return st;
  }
  // first grid: the reverse kick with the means
  if (pm_status st = bin(c, c->disp, nullptr, nullptr, mak, act)) return st;
  TileArgs k1 = args(0);
  k1.mesh_in = c->phi;
  k1.il_in = c->accbuf;
  KLAUNCH(c, PM_K_ADJ_KICK, launch_tile(k1, TK_ADJ_KICK, mak, ord, c->stream));
  if (pm_status st = kick_dot(c, kdot, act)) return st;
  if (!(parts & 1))
    KLAUNCH(c, PM_K_FILL, launch_fill(c->xbar, (long long)sizeof(float) * 3 * N * B, c->stream));
  if (!(parts & 2)) return PM_OK;
  if (pm_status st = dipole(k1, d1)) return st;
  // mesh cotangents of the two deposits (cotangent 1 on c->phi, 2 on d2)
  pm_status st = r2c_mesh(c, d1, SRC_F32, M, 1.0, 0.0, c->spec, c->g.spec_stride, c->cfg.n_g, false, act);
  if (st) return st;
  st = r2c_mesh(c, d2, SRC_F32, M, 1.0, 0.0, c->spec2, c->g.spec_stride, c->cfg.n_g, true, act);
  if (st) return st;
  st = spectrum_to_real(c, c->spec, MODE_FUSED_IL, s, c->spec2, c->phi, act);
  if (st) return st;
  st = spectrum_to_real(c, c->spec2, MODE_INV, nullptr, nullptr, d2, act);
  if (st) return st;
  // scatter terms: the first grid's into the buffer, then the second grid's
  // pass takes the mean and reverses the drift
  TileArgs r1 = args(0);
  r1.mesh_in = c->phi;
  r1.il_out = c->accbuf;
  KLAUNCH(c, PM_K_ADJ_DRIFT, launch_tile(r1, TK_ADJ_DRIFT, mak, ord, c->stream));
  c->g.ushift = half;
  st = bin(c, c->disp, nullptr, nullptr, mak, act);
  c->g.ushift = 0;
  if (st) return st;
  TileArgs r2 = args(half);
  r2.mesh_in = d2;
  r2.il_in = c->accbuf;
  KLAUNCH(c, PM_K_ADJ_DRIFT, launch_tile(r2, TK_ADJ_DRIFT, mak, ord, c->stream));
  return PM_OK;
}

// Reverse pass through the second-order displacement (the transposes of
// lpt2 in reverse order): psi2_bar = D0^2 X_bar + 2 D0 V_bar on the lattice;
// mu_bar on the padded grid through the conjugate multiplier; the cotangents
// of the six derivative fields, mu_bar (S - g_ii) and -2 mu_bar g_ij
// (d mu / d g, S the diagonal sum, the fields recomputed from the noise);
// each transformed and pulled back through its real multiplier into the
// particle-grid spectrum at icspec component 3, which the Zel'dovich
// combination then adds to.
static pm_status lpt2_adjoint(pm_ctx* c, unsigned long long act) {
  const int np = c->cfg.n_p, P = 2 * np, B = c->cfg.batch;
  const long long N = c->g.N, M = c->g.M;
  float* A = reinterpret_cast<float*>(c->mesh);  // mu_bar, and S at A + M (slot stride 2M)
  float* gb = c->phi;                              // one field's cotangent (slot stride M)
  float2* fspec = c->spec;
  float2* Q = c->icspec + 3 * c->icspec_comp;
  float* psibar = c->u_sorted;
  // psi2_bar = D0^2 X_bar + 2 D0 vfac V_bar = 2 D0 vfac (D0 / (2 vfac) X_bar + V_bar);
  // the factor 2 D0 vfac rides on the multiplier
  std::vector<float> half(B, (float)(0.5 * c->D0 / c->vfac));
  KLAUNCH(c, PM_K_MISC, launch_psibar(c->xbar, c->vbar, psibar, N, 3 * N, B, half.data(), c->g.log2_np,
                                       c->g.log2_pb, act, c->stream));
  for (int comp = 0; comp < 3; ++comp) {
    pm_status st = r2c_mesh(c, psibar + comp * N, SRC_F32, 3 * N, 1.0, 0.0, c->icspec + comp * c->icspec_comp,
                            c->icspec_stride, np, true, act);
    if (st) return st;
  }
  ColArgs m{};
  m.data = fspec;
  m.slot_stride = c->g.spec_stride;
  m.n = P;
  m.nh = P / 2 + 1;
  m.rs = spec_rs(P);
  m.tw = c->d_tw;
  m.tws = c->Lmax / P;
  m.src3 = c->icspec;
  m.comp_stride = c->icspec_comp;
  m.src_slot_stride = c->icspec_stride;
  m.src_rs = spec_rs(np);
  m.n_p = np;
  m.active = act;
  m.axis = 0;
  m.zlim = np / 2;
  m.keep = np;
  m.keep_outer = 1;
  for (int b = 0; b < B; ++b) m.coef[b] = (float)(3.0 / 7.0 / ((double)P * P * P) * 2.0 * c->D0 * c->vfac);
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(m, MODE_LPT_MUBAR, B, c->stream));
  ColArgs my = m;
  my.axis = 1;
  my.keep_outer = 0;
  my.keep_in = 1;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(my, MODE_INV, B, c->stream));
  RowLaunch rl{};
  rl.n = P;
  rl.rs = spec_rs(P);
  rl.kz_lim = np / 2;
  rl.n_rows = (long long)P * P;
  rl.batch = B;
  rl.inverse = true;
  rl.src = fspec;
  rl.src_stride = c->g.spec_stride;
  rl.dst = A;
  rl.dst_stride = 2 * M;
  rl.dst_mode = DST_F32;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (P / 2);
  rl.tws_full = c->Lmax / P;
  rl.scale = 1.0;
  rl.stream = c->stream;
  rl.active = act;
  KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  // the noise spectrum again (component 0; the psi2_bar spectra are spent)
  pm_status st = r2c_mesh(c, c->w, SRC_F32, N, 1.0, 0.0, c->icspec, c->icspec_stride, np, true, act);
  if (st) return st;
  ColArgs a{};
  a.n = P;
  a.nh = P / 2 + 1;
  a.rs = spec_rs(P);
  a.tw = c->d_tw;
  a.tws = c->Lmax / P;
  a.amp = c->d_amp;
  a.active = act;
  a.n_p = np;
  for (int b = 0; b < B; ++b)
    a.fac[b] = (float)(c->cfg.spectrum == PM_SPEC_BBKS ? c->slot_sigma8[b] / c->cfg.sigma8 : 1.0);
  a.src3 = c->icspec;
  a.src_slot_stride = c->icspec_stride;
  a.src_rs = spec_rs(np);
  a.slot_stride = c->g.spec_stride;
  a.data = fspec;
  a.dst3 = fspec;
  a.axis = 0;
  a.zlim = np / 2;
  a.keep = np;
  a.keep_outer = 1;
  auto field = [&](int i, int j, int mode, float* dst, long long dst_stride, float* dst2) -> pm_status {
    a.comp = i;
    a.comp2 = j;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_LPT_D, B, c->stream));
    ColArgs y = a;
    y.axis = 1;
    y.keep_outer = 0;
    y.keep_in = 1;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(y, MODE_INV, B, c->stream));
    RowLaunch r = rl;
    r.dst_mode = mode;
    r.dst = dst;
    r.dst_stride = dst_stride;
    r.dst2 = dst2;
    KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(r));
    return PM_OK;
  };
  // S = g_00 + g_11 + g_22
  for (int i = 0; i < 3; ++i)
    if ((st = field(i, i, i ? DST_ACC : DST_F32, A + M, 2 * M, nullptr))) return st;
  for (int b = 0; b < B; ++b)
    if ((act >> b) & 1ull)
      KLAUNCH(c, PM_K_FILL, launch_fill(Q + b * c->icspec_stride, (long long)sizeof(float2) * c->icspec_comp,
                                        c->stream));
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int q = 0; q < 6; ++q) {
    const int i = pairs[q][0], j = pairs[q][1];
    if ((st = field(i, j, i == j ? DST_GBAR_DIAG : DST_GBAR_OFF, gb, M, A))) return st;
    st = r2c_mesh(c, gb, SRC_F32, M, 1.0, 0.0, fspec, c->g.spec_stride, P, false, act, np);
    if (st) return st;
    ColArgs t = a;
    t.dst3 = Q;
    t.comp = i;
    t.comp2 = j;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(t, MODE_LPT_DT, B, c->stream));
  }
  return PM_OK;
}

pm_status pm_adjoint_full(pm_ctx* c, const float* dL_ddelta, float* dL_dw, double* dL_dsigma8, double* dL_dtime);

pm_status pm_adjoint(pm_ctx* c, const float* dL_ddelta, float* dL_dw, double* dL_dsigma8) {
  return pm_adjoint_full(c, dL_ddelta, dL_dw, dL_dsigma8, nullptr);
}

pm_status pm_adjoint_full(pm_ctx* c, const float* dL_ddelta, float* dL_dw, double* dL_dsigma8, double* dL_dtime) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!c->with_adj) return fail(c, PM_ESTATE, "workspace bound without adjoint buffers");
  if (!c->ran) return fail(c, PM_ESTATE, "pm_adjoint before pm_run");
  if (!dL_ddelta || !dL_dw || !dL_dsigma8) return PM_EINVAL;
  const int B = c->cfg.batch, np = c->cfg.n_p;
  const long long N = c->g.N, M = c->g.M;
  const double mfac = (double)M / (double)N;
  KLAUNCH(c, PM_K_FILL, launch_fill(c->xbar, (long long)sizeof(float) * 3 * N * B, c->stream));
  KLAUNCH(c, PM_K_FILL, launch_fill(c->vbar, (long long)sizeof(float) * 3 * N * B, c->stream));
  int nmax = 0;
  for (int b = 0; b < B; ++b) nmax = std::max(nmax, c->slot_steps[b]);
  // loss pullback through the final CIC density and the last half drift
  const unsigned long long all = c->user_mask;
  pm_status st0 = bin(c, c->disp, nullptr, nullptr, 2, all);
  if (st0) return st0;
  TileArgs lv = tile_args(c, c->disp, all);
  lv.mesh_in = dL_ddelta;
  for (int b = 0; b < B; ++b) {
    lv.coef[b] = (float)mfac;
    lv.tau[b] = (float)c->slot_table[b][c->slot_steps[b] - 1].tau2;
  }
  KLAUNCH(c, PM_K_ADJ_DRIFT, launch_tile(lv, TK_ADJ_DRIFT, 2, c->cfg.grad_order, c->stream));
  // temporal adjoints (tab. adjoint_dkd), rows (tau1, tau2, alpha, beta) per
  // step: X_bar . V after the loss pullback gives the last tau2 of each slot;
  // after reverse step n (its merged drift leaves X_bar and V alone) it gives
  // tau1 of step n and tau2 of step n - 1; alpha and beta come from the dots
  // taken around the adjoint kick
  const int S = c->cfg.n_steps;
  std::vector<double> ones(B, 1.0);
  auto row = [&](int n, int field) {
    std::vector<long long> v(B);
    for (int b = 0; b < B; ++b) v[b] = ((long long)b * S + std::max(0, n)) * 4 + field;
    return v;
  };
  if (dL_dtime) {
    KLAUNCH(c, PM_K_FILL, launch_fill(dL_dtime, (long long)sizeof(double) * 4 * S * B, c->stream));
    std::vector<long long> last(B);
    for (int b = 0; b < B; ++b) last[b] = ((long long)b * S + c->slot_steps[b] - 1) * 4 + 1;
    KLAUNCH(c, PM_K_MISC, launch_dot(c->xbar, c->vel, 3 * N, 3 * N, B, c->dot_partial, dL_dtime, ones.data(), all,
                                     c->stream, last.data()));
  }
  for (int n = nmax - 1; n >= 0; --n) {
    std::vector<double> s(B, 1);
    unsigned long long act = 0;
    for (int b = 0; b < B; ++b)
      if (n < c->slot_steps[b]) { s[b] = c->slot_table[b][n].s; act |= 1ull << b; }
    act &= c->user_mask;
    if (!act) continue;
    // force at X^{n+1/2} (bins the particles by tile for the kernels below)
    pm_status st = potential(c, c->disp, nullptr, nullptr, s.data(), act);
    if (st) return st;
    std::vector<double> al(B, 1), be(B, 0), tau(B, 0);
    for (int b = 0; b < B; ++b) {
      if (!((act >> b) & 1)) continue;
      const auto& T = c->slot_table[b];
      al[b] = T[n].alpha;
      be[b] = T[n].beta;
      tau[b] = T[n].tau1 + (n > 0 ? T[n - 1].tau2 : 0.0);
    }
    double* d1 = c->tdots;
    double* d2 = c->tdots + kMaxBatch;
    if (dL_dtime)
      KLAUNCH(c, PM_K_MISC, launch_dot(c->vbar, c->vel, 3 * N, 3 * N, B, c->dot_partial, d1, ones.data(), act,
                                       c->stream));
    st = reverse_force_step(c, s.data(), al.data(), be.data(), tau.data(), act, 3, dL_dtime ? d2 : nullptr);
    if (st) return st;
    if (dL_dtime) {
      TimeAB t{};
      const std::vector<long long> r0 = row(n, 0);
      for (int b = 0; b < B; ++b) {
        t.alpha[b] = al[b];
        t.beta[b] = be[b];
        t.idx[b] = r0[b];
      }
      KLAUNCH(c, PM_K_MISC, launch_time_ab(d1, d2, dL_dtime, t, act, c->stream));
      KLAUNCH(c, PM_K_MISC, launch_dot(c->xbar, c->vel, 3 * N, 3 * N, B, c->dot_partial, dL_dtime, ones.data(), act,
                                       c->stream, r0.data()));
      if (n > 0)
        KLAUNCH(c, PM_K_MISC, launch_dot(c->xbar, c->vel, 3 * N, 3 * N, B, c->dot_partial, dL_dtime, ones.data(),
                                         act, c->stream, row(n - 1, 1).data()));
    }
  }
  // initial conditions: psi_bar = D0 X_bar + V_bar, w_bar = sum_c T_c^T psi_bar_c
  // (plus the second-order term's pullback, gathered first)
  if (c->cfg.lpt_order == 2)
    if (pm_status st = lpt2_adjoint(c, c->user_mask)) return st;
  // with the canonical momentum V = vfac psi: psi_bar = vfac (D0 / vfac X_bar + V_bar)
  std::vector<float> d0(B, (float)(c->D0 / c->vfac));
  float* psibar = c->u_sorted;
  KLAUNCH(c, PM_K_MISC, launch_psibar(c->xbar, c->vbar, psibar, N, 3 * N, B, d0.data(), c->g.log2_np, c->g.log2_pb,
                                       c->user_mask, c->stream));
  const unsigned long long act = c->user_mask;
  for (int comp = 0; comp < 3; ++comp) {
    pm_status st = r2c_mesh(c, psibar + comp * N, SRC_F32, 3 * N, 1.0, 0.0,
                            c->icspec + comp * c->icspec_comp, c->icspec_stride, np, true, act);
    if (st) return st;
  }
  float2* comb = c->icspec + 3 * c->icspec_comp;
  ColArgs ca{};
  ca.src3 = c->icspec;
  ca.comp_stride = c->icspec_comp;
  ca.data = comb;
  ca.slot_stride = c->icspec_stride;
  ca.n = np;
  ca.nh = np / 2 + 1;
  ca.rs = spec_rs(np);
  ca.tw = c->d_tw;
  ca.tws = c->Lmax / np;
  ca.amp = c->d_amp;
  ca.active = act;
  ca.axis = 0;
  for (int b = 0; b < B; ++b)
    ca.fac[b] = (float)((c->cfg.spectrum == PM_SPEC_BBKS ? c->slot_sigma8[b] / c->cfg.sigma8 : 1.0) * c->vfac);
  ca.combine_add = c->cfg.lpt_order == 2;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(ca, MODE_COMBINE_IC, B, c->stream));
  ca.axis = 1;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(ca, MODE_INV, B, c->stream));
  RowLaunch rl{};
  rl.n = np;
  rl.rs = spec_rs(np);
  rl.n_rows = (long long)np * np;
  rl.batch = B;
  rl.inverse = true;
  rl.dst_mode = DST_F32;
  rl.src = comb;
  rl.src_stride = c->icspec_stride;
  rl.dst = dL_dw;
  rl.dst_stride = N;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (np / 2);
  rl.tws_full = c->Lmax / np;
  rl.scale = 1.0;
  rl.stream = c->stream;
  rl.active = act;
  KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  // dL/dsigma8 = <psi_bar, psi>/sigma8 = <w_bar, w>/sigma8 (psi is linear in w and
  // sigma8).  The power-law spectrum is normalised by its rms displacement, so
  // there psi does not depend on sigma8 and the derivative is 0.
  std::vector<double> inv(B);
  for (int b = 0; b < B; ++b) inv[b] = c->cfg.spectrum == PM_SPEC_BBKS ? 1.0 / c->slot_sigma8[b] : 0.0;
  KLAUNCH(c, PM_K_MISC, launch_dot(dL_dw, c->w, N, N, B, c->dot_partial, dL_dsigma8, inv.data(), act, c->stream));
  c->ran = false;
  return PM_OK;
}

pm_status pm_power_spectrum(pm_ctx* c, int32_t n_bins, int32_t deconvolve_cic, double* k_mean,
                            double* pk, int64_t* n_modes) {
  if (pm_status st = check_bound(c)) return st;
  if (!c->ics_done) return fail(c, PM_ESTATE, "no particles yet");
  const int n = c->cfg.n_g;
  if (n_bins < 1 || n_bins > n || n_bins > 512 || !k_mean || !pk || !n_modes)
    return fail(c, PM_EINVAL, "n_bins must be in [1, min(n_g, 512)]");
  const unsigned long long act = c->user_mask;
  pm_status st = deposit(c, c->disp, nullptr, nullptr, 2, c->mesh, act);
  if (st) return st;
  const double N = (double)c->g.N, n3 = (double)c->g.M;
  st = r2c_mesh(c, c->mesh, SRC_I64, c->g.mesh_stride, n3 / N / 4294967296.0, 1.0, c->spec,
                c->g.spec_stride, n, true, act);
  if (st) return st;
  const double L = c->cfg.box;
  KLAUNCH(c, PM_K_MISC, launch_pk(c->spec, c->g.spec_stride, n, c->cfg.batch, n_bins, 2.0 * M_PI / L,
                      L * L * L / (n3 * n3), c->d_cic4, deconvolve_cic, c->pk_partial, k_mean, pk,
                      (long long*)n_modes, act, spec_rs(n), c->stream));
  return PM_OK;
}

// ------------------------------------------------------------ forward mode

// tangent of the contrast at the current binning for the tangent positions
// in xbar (max |xdot| already reduced into umax): out = r n_g^3 / N
// sum_i grad W . xdot_i, as FP32 [B][M]
static pm_status tangent_contrast(pm_ctx* c, int mak, float* out, unsigned long long act) {
  const int B = c->cfg.batch;
  const double N = (double)c->g.N, coef = (double)(1 << c->g.log2_r) * (double)c->g.M / N;
  KLAUNCH(c, PM_K_MISC, launch_dipole_scale((const unsigned int*)c->umax, c->scale, c->inv_scale, 3.0 * coef * N,
                                            3.0 * coef, B, c->stream));
  TileArgs t = tile_args(c, c->disp, act);
  for (int b = 0; b < B; ++b) t.coef[b] = (float)coef;
  const int kr = kernel_reach_of(mak);
  AssembleArgs as = assemble_args(c, kr, kr, out, act);
  KLAUNCH(c, PM_K_DIPOLE,
          both(launch_tile(t, TK_TAN_SPREAD, mak, 0, c->stream), launch_assemble(as, true, c->stream)));
  return PM_OK;
}

static pm_status absmax_tangent(pm_ctx* c, const SlotCoef& tau, unsigned long long act) {
  const long long N = c->g.N;
  KLAUNCH(c, PM_K_FILL, launch_fill(c->umax, (long long)sizeof(float) * kMaxBatch, c->stream));
  KLAUNCH(c, PM_K_MISC, launch_tan_drift(c->xbar, c->vbar, 3 * N, 3 * N, tau, (unsigned int*)c->umax,
                                         c->cfg.batch, act, c->stream));
  return PM_OK;
}

// Tangent of the second-order term along the noise w_eff (whose spectrum
// is at icspec component 3, left there by its IC chain): with g the six
// derivative fields of w and gd those of w_eff, S and Sd their traces,
//   mu_dot = S Sd - sum_i g_ii gd_ii - 2 sum_{i<j} g_ij gd_ij,
// then the same multiplier as the primal term, added to (xbar, vbar).
static pm_status lpt2_tangent(pm_ctx* c, unsigned long long act) {
  const int np = c->cfg.n_p, P = 2 * np, B = c->cfg.batch;
  const long long N = c->g.N, M = c->g.M, P3 = (long long)P * P * P;
  float* F = reinterpret_cast<float*>(c->mesh);  // Sd, then -c g_ij (slot stride 2M)
  float* mud = F + M;                             // mu_dot (slot stride 2M)
  float* S = c->phi;                              // trace of g (slot stride M)
  pm_status st = r2c_mesh(c, c->w, SRC_F32, N, 1.0, 0.0, c->icspec, c->icspec_stride, np, true, act);
  if (st) return st;
  ColArgs a{};
  a.n = P;
  a.nh = P / 2 + 1;
  a.rs = spec_rs(P);
  a.tw = c->d_tw;
  a.tws = c->Lmax / P;
  a.amp = c->d_amp;
  a.active = act;
  a.n_p = np;
  for (int b = 0; b < B; ++b)
    a.fac[b] = (float)(c->cfg.spectrum == PM_SPEC_BBKS ? c->slot_sigma8[b] / c->cfg.sigma8 : 1.0);
  a.src_slot_stride = c->icspec_stride;
  a.src_rs = spec_rs(np);
  a.slot_stride = c->g.spec_stride;
  a.data = c->spec;
  a.dst3 = c->spec;
  a.axis = 0;
  a.zlim = np / 2;
  a.keep = np;
  a.keep_outer = 1;
  RowLaunch rl{};
  rl.n = P;
  rl.rs = spec_rs(P);
  rl.kz_lim = np / 2;
  rl.n_rows = (long long)P * P;
  rl.batch = B;
  rl.inverse = true;
  rl.src = c->spec;
  rl.src_stride = c->g.spec_stride;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (P / 2);
  rl.tws_full = c->Lmax / P;
  rl.stream = c->stream;
  rl.active = act;
  const float2* wspec = c->icspec;                           // the primal noise
  const float2* dspec = c->icspec + 3 * c->icspec_comp;      // the tangent noise
  auto field = [&](const float2* src, int i, int j, int mode, double scale, float* dst, long long stride,
                   float* dst2) -> pm_status {
    a.src3 = src;
    a.comp = i;
    a.comp2 = j;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_LPT_D, B, c->stream));
    ColArgs y = a;
    y.axis = 1;
    y.keep_outer = 0;
    y.keep_in = 1;
    KLAUNCH(c, PM_K_FFT_COLS, fft_cols(y, MODE_INV, B, c->stream));
    RowLaunch r = rl;
    r.dst_mode = mode;
    r.scale = scale;
    r.dst = dst;
    r.dst_stride = stride;
    r.dst2 = dst2;
    KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(r));
    return PM_OK;
  };
  for (int i = 0; i < 3; ++i) {
    if ((st = field(wspec, i, i, i ? DST_ACC : DST_F32, 1.0, S, M, nullptr))) return st;
    if ((st = field(dspec, i, i, i ? DST_ACC : DST_F32, 1.0, F, 2 * M, nullptr))) return st;
  }
  KLAUNCH(c, PM_K_MISC, launch_mul(S, M, F, 2 * M, mud, 2 * M, P3, B, act, c->stream));
  const int pairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {0, 1}, {0, 2}, {1, 2}};
  for (int q = 0; q < 6; ++q) {
    const int i = pairs[q][0], j = pairs[q][1];
    if ((st = field(wspec, i, j, DST_F32, i == j ? -1.0 : -2.0, F, 2 * M, nullptr))) return st;
    if ((st = field(dspec, i, j, DST_MU_ACC, 1.0, F, 2 * M, mud))) return st;
  }
  return lpt2_from_mu(c, mud, 2 * M, c->vbar, c->xbar, act);
}

// NUFFT tangent kick at X^{n+1/2} (the primal force meshes in force3, the
// binning current): the spread's tangent (the ES gradient spread of
// r Xdot, fixed point at the scale of max |Xdot|), the force chain to three
// tangent meshes (in the scratch slab, free between spreads: 3M <= 8 W^3
// n_tiles / 4 floats per slot), then the ES tangent kick and drift
static pm_status nufft_tangent_kick(pm_ctx* c, const double* s, const double* al, const double* be,
                                    const double* tau, unsigned long long act) {
  const int B = c->cfg.batch;
  const long long N = c->g.N;
  const double r = (double)(1 << c->g.log2_r);
  KLAUNCH(c, PM_K_MISC, launch_dipole_scale((const unsigned int*)c->umax, c->scale, c->inv_scale,
                                            3.0 * r * (double)N, 3.0 * r, B, c->stream));
  TileArgs k = tile_args(c, c->disp, act);
  k.es_tab = c->d_es_tab;
  k.tan_xbar = 1;
  k.win_f32 = 1;  // FP32 partial sums at the slot's inverse scale
  k.win_scale = 0.0;
  k.inv_scale = c->inv_scale;
  for (int b = 0; b < B; ++b) k.coef[b] = (float)r;
  float* d = reinterpret_cast<float*>(c->mesh);
  AssembleArgs as = assemble_args(c, kEsHaloLo, kEsHaloHi, d, act);
  as.slab_f32 = 1;
  as.shift = 0.0;
  KLAUNCH(c, PM_K_DIPOLE, both(launch_tile_es(k, TK_ES_DIPOLE, c->stream), launch_assemble(as, true, c->stream)));
  float* tmesh = reinterpret_cast<float*>(c->scratch);
  if (pm_status st = nufft_force_chain(c, d, s, tmesh, act)) return st;
  TileArgs q = tile_args(c, c->disp, act);
  q.es_tab = c->d_es_tab;
  q.mesh_in = c->force3;
  q.mesh_in2 = tmesh;
  q.comp_stride = c->g.M;
  q.acc_out = c->u_sorted;
  for (int b = 0; b < B; ++b) {
    q.alpha[b] = (float)al[b];
    q.beta[b] = (float)be[b];
    q.tau[b] = (float)tau[b];
  }
  KLAUNCH(c, PM_K_GATHER_KICK, launch_tile_es(q, TK_ES_TAN_KICK, c->stream));
  return PM_OK;
}

// Interlaced tangent kick at X^{n+1/2} (primal potentials phi_1 on c->phi,
// phi_2 on c->phi2; the second grid's binning current): every term of J_A
// Xdot is the mean of the two grids' terms.  The tangent contrasts of both
// grids go through the same two-grid chain as the force; the grid passes
// that need the other binning leave their terms in the per-particle buffer
// ([B][3][N] views of its two halves); the second grid's binning and both
// primal potentials are left for the primal kick.
static pm_status interlaced_tangent_kick(pm_ctx* c, const double* s, const double* al, const double* be,
                                         const double* tau, unsigned long long act) {
  const int B = c->cfg.batch, mak = c->cfg.mak, ord = c->cfg.grad_order;
  const long long N = c->g.N;
  const long long half = 1ll << (kFracBits - 1);
  float* d1 = reinterpret_cast<float*>(c->mesh);      // tangent contrast, then tangent potential 1
  float* d2 = c->phi2;                                 // primal potential 2 (the primal kick reads it too)
  float* t2 = reinterpret_cast<float*>(c->scratch);    // tangent potential 2 (the slab is free after the spreads)
  float* dir2 = c->accbuf;                             // grid 2's direct term
  float* j1 = c->accbuf + 3 * N * B;                   // grid 1's J
  auto args = [&](long long ushift) {
    c->g.ushift = ushift;
    TileArgs k = tile_args(c, c->disp, act);
    c->g.ushift = 0;
    for (int b = 0; b < B; ++b) {
      k.alpha[b] = (float)al[b];
      k.beta[b] = (float)be[b];
      k.tau[b] = (float)tau[b];
    }
    return k;
  };
  // grid 2: direct term, then its tangent contrast to the spectrum (full transform)
  TileArgs k2 = args(half);
  k2.mesh_in = d2;
  k2.acc_out = dir2;
  KLAUNCH(c, PM_K_ADJ_KICK, launch_tile(k2, TK_TAN_DIRECT, mak, ord, c->stream));
  c->g.ushift = half;
  pm_status st = tangent_contrast(c, mak, d1, act);
  c->g.ushift = 0;
  if (st) return st;
  st = r2c_mesh(c, d1, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec2, c->g.spec_stride, c->cfg.n_g, true, act);
  if (st) return st;
  // grid 1: its tangent contrast, the two-grid chain to both tangent potentials
  if ((st = bin(c, c->disp, nullptr, nullptr, mak, act))) return st;
  if ((st = tangent_contrast(c, mak, d1, act))) return st;
  st = r2c_mesh(c, d1, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec, c->g.spec_stride, c->cfg.n_g, false, act);
  if (st) return st;
  if ((st = spectrum_to_real(c, c->spec, MODE_FUSED_IL, s, c->spec2, d1, act))) return st;
  if ((st = spectrum_to_real(c, c->spec2, MODE_INV, nullptr, nullptr, t2, act))) return st;
  TileArgs k1 = args(0);
  k1.mesh_in = c->phi;
  k1.acc_out = c->u_sorted;
  KLAUNCH(c, PM_K_ADJ_KICK, launch_tile(k1, TK_TAN_DIRECT, mak, ord, c->stream));
  TileArgs q1 = args(0);
  q1.mesh_in = d1;
  q1.acc_in = c->u_sorted;
  q1.il_out = j1;
  KLAUNCH(c, PM_K_GATHER_KICK, launch_tile(q1, TK_TAN_KICK, mak, ord, c->stream));
  // grid 2 again: its J, the mean, the tangent kick and drift
  c->g.ushift = half;
  st = bin(c, c->disp, nullptr, nullptr, mak, act);
  c->g.ushift = 0;
  if (st) return st;
  TileArgs q2 = args(half);
  q2.mesh_in = t2;
  q2.acc_in = dir2;
  q2.il_in = j1;
  KLAUNCH(c, PM_K_GATHER_KICK, launch_tile(q2, TK_TAN_KICK, mak, ord, c->stream));
  return PM_OK;
}

pm_status pm_jvp(pm_ctx* c, const float* w_dot, const double* sigma8_dot, float* delta_dot_out) {
  if (pm_status st = check_bound(c)) return st;
  if (!c->with_adj) return fail(c, PM_ESTATE, "workspace bound without adjoint buffers (the tangents live there)");
  if (!c->ics_done) return fail(c, PM_ESTATE, "pm_jvp before pm_init_ics");
  if (!w_dot || !delta_dot_out) return PM_EINVAL;
  const bool nufft = c->cfg.force == PM_FORCE_NUFFT;
  const int B = c->cfg.batch, mak = c->cfg.mak, ord = c->cfg.grad_order;
  const long long N = c->g.N;
  const unsigned long long all = c->user_mask;
  // primal initial state again from the stored white noise; tangent initial
  // state psi(w_dot + (sigma8_dot / sigma8) w): psi is linear in w and, with
  // the BBKS spectrum, proportional to sigma8
  if (pm_status st = ic_chain(c, c->w, c->disp, c->vel, all)) return st;
  if (c->cfg.lpt_order == 2)
    if (pm_status st = lpt2(c, all)) return st;
  SlotCoef k{};
  for (int b = 0; b < B; ++b)
    k.v[b] = (sigma8_dot && c->cfg.spectrum == PM_SPEC_BBKS) ? (float)(sigma8_dot[b] / c->slot_sigma8[b]) : 0.f;
  float* weff = c->u_sorted;  // [B][N] of the [B][3][N] adjoint buffer, idle here
  KLAUNCH(c, PM_K_MISC, launch_lincomb(w_dot, c->w, weff, N, k, B, all, c->stream));
  if (pm_status st = ic_chain(c, weff, c->xbar, c->vbar, all)) return st;
  if (c->cfg.lpt_order == 2)
    if (pm_status st = lpt2_tangent(c, all)) return st;
  int nmax = 0;
  for (int b = 0; b < B; ++b) nmax = std::max(nmax, c->slot_steps[b]);
  float* dd = reinterpret_cast<float*>(c->mesh);  // tangent contrast, then tangent potential
  for (int n = 0; n < nmax; ++n) {
    std::vector<double> tp(B, 0), s(B, 1), al(B, 1), be(B, 0), tq(B, 0);
    SlotCoef t1{};
    unsigned long long act = 0;
    for (int b = 0; b < B; ++b) {
      if (n >= c->slot_steps[b]) continue;
      const StepCoef& sc = c->slot_table[b][n];
      tp[b] = sc.tau1; s[b] = sc.s; al[b] = sc.alpha; be[b] = sc.beta; tq[b] = sc.tau2;
      t1.v[b] = (float)sc.tau1;
      act |= 1ull << b;
    }
    act &= all;
    if (!act) continue;
    // Xdot += tau1 Vdot (and max |Xdot|); the primal drift rides on the binning
    if (pm_status st = absmax_tangent(c, t1, act)) return st;
    pm_status st = potential(c, c->disp, c->vel, tp.data(), s.data(), act);
    if (st) return st;
    if (nufft || c->cfg.antialias) {
      st = nufft ? nufft_tangent_kick(c, s.data(), al.data(), be.data(), tq.data(), act)
                 : interlaced_tangent_kick(c, s.data(), al.data(), be.data(), tq.data(), act);
      if (st) return st;
      if ((st = kick(c, c->disp, al.data(), be.data(), tq.data(), nullptr, act))) return st;
      continue;
    }
    // J_A Xdot at X^{n+1/2}: the tangent contrast through the same multiplier,
    // gathered like the force, plus the gather's position term
    if ((st = tangent_contrast(c, mak, dd, act))) return st;
    st = r2c_mesh(c, dd, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec, c->g.spec_stride, c->cfg.n_g, false, act);
    if (st) return st;
    if ((st = poisson_to_real(c, s.data(), dd, act))) return st;
    TileArgs d = tile_args(c, c->disp, act);
    d.mesh_in = c->phi;
    d.acc_out = c->u_sorted;
    KLAUNCH(c, PM_K_ADJ_KICK, launch_tile(d, TK_TAN_DIRECT, mak, ord, c->stream));
    TileArgs q = tile_args(c, c->disp, act);
    q.mesh_in = dd;
    q.acc_in = c->u_sorted;
    for (int b = 0; b < B; ++b) {
      q.alpha[b] = (float)al[b];
      q.beta[b] = (float)be[b];
      q.tau[b] = (float)tq[b];
    }
    KLAUNCH(c, PM_K_GATHER_KICK, launch_tile(q, TK_TAN_KICK, mak, ord, c->stream));
    // the primal kick and drift
    if ((st = kick(c, c->disp, al.data(), be.data(), tq.data(), nullptr, act))) return st;
  }
  // tangent of the final CIC contrast
  if (pm_status st = absmax_tangent(c, SlotCoef{}, all)) return st;
  if (pm_status st = bin(c, c->disp, nullptr, nullptr, 2, all)) return st;
  if (pm_status st = tangent_contrast(c, 2, delta_dot_out, all)) return st;
  c->ran = true;
  c->tangent_valid = true;
  return PM_OK;
}


pm_status pm_power_spectrum_jvp(pm_ctx* c, const float* delta_dot, int32_t n_bins, int32_t deconvolve_cic,
                                double* k_mean, double* pk, double* pk_dot, int64_t* n_modes) {
  if (!delta_dot || !pk_dot) return PM_EINVAL;
  if (pm_status st = pm_power_spectrum(c, n_bins, deconvolve_cic, k_mean, pk, n_modes)) return st;
  // the tangent's spectrum in the (now free) mesh buffer: n^2 rs <= n^3
  const int n = c->cfg.n_g;
  const unsigned long long act = c->user_mask;
  float2* spec2 = reinterpret_cast<float2*>(c->mesh);
  pm_status st = r2c_mesh(c, delta_dot, SRC_F32, c->g.mesh_stride, 1.0, 0.0, spec2, c->g.spec_stride, n, true, act);
  if (st) return st;
  const double L = c->cfg.box, n3 = (double)c->g.M;
  KLAUNCH(c, PM_K_MISC, launch_pk(c->spec, c->g.spec_stride, n, c->cfg.batch, n_bins, 2.0 * M_PI / L,
                                  L * L * L / (n3 * n3), c->d_cic4, deconvolve_cic, c->pk_partial, k_mean, pk_dot,
                                  (long long*)n_modes, act, spec_rs(n), c->stream, spec2));
  return PM_OK;
}

pm_status pm_density(pm_ctx* c, float* delta_out, int64_t* fixed_out) {
  if (pm_status st = check_bound(c)) return st;
  if (!c->ics_done) return fail(c, PM_ESTATE, "no particles yet");
  const unsigned long long act = c->user_mask;
  pm_status st = deposit(c, c->disp, nullptr, nullptr, 2, c->mesh, act);
  if (st) return st;
  const double scale = (double)c->g.M / (double)c->g.N / 4294967296.0;
  if (delta_out)
    KLAUNCH(c, PM_K_MISC, launch_i64_to_delta(c->mesh, delta_out, c->g.M, c->g.mesh_stride, c->cfg.batch, scale, act, c->stream));
  if (fixed_out)
    for (int b = 0; b < c->cfg.batch; ++b)
      if ((act >> b) & 1ull)
        HIPCHK(c, hipMemcpyAsync(fixed_out + b * c->g.M, c->mesh + b * c->g.mesh_stride, sizeof(long long) * c->g.M,
                                 hipMemcpyDeviceToDevice, c->stream));
  return PM_OK;
}

// particle arrays [B][3][N]: row-major lattice order at the boundary,
// lattice-block order inside (mak.h)
static pm_status to_user_order(pm_ctx* c, const float* internal, float* user) {
  KLAUNCH(c, PM_K_MISC, launch_reorder(internal, user, c->g.N, 3 * c->g.N, 3, c->cfg.batch, c->g.log2_np,
                                       c->g.log2_pb, false, all_mask(c->cfg.batch), c->stream));
  return PM_OK;
}

static pm_status from_user_order(pm_ctx* c, const float* user, float* internal) {
  KLAUNCH(c, PM_K_MISC, launch_reorder(user, internal, c->g.N, 3 * c->g.N, 3, c->cfg.batch, c->g.log2_np,
                                       c->g.log2_pb, true, all_mask(c->cfg.batch), c->stream));
  return PM_OK;
}

pm_status pm_get_state(pm_ctx* c, float* disp, float* vel) {
  if (pm_status st = check_bound(c)) return st;
  if (disp)
    if (pm_status st = to_user_order(c, c->disp, disp)) return st;
  if (vel)
    if (pm_status st = to_user_order(c, c->vel, vel)) return st;
  return PM_OK;
}

pm_status pm_get_tangent(pm_ctx* c, float* disp_dot, float* vel_dot) {
  if (pm_status st = check_bound(c)) return st;
  if (!c->tangent_valid) return fail(c, PM_ESTATE, "no tangents: pm_jvp was not the last call that moved the state");
  if (disp_dot)
    if (pm_status st = to_user_order(c, c->xbar, disp_dot)) return st;
  if (vel_dot)
    if (pm_status st = to_user_order(c, c->vbar, vel_dot)) return st;
  return PM_OK;
}

pm_status pm_set_state(pm_ctx* c, const float* disp, const float* vel) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!disp || !vel) return PM_EINVAL;
  if (pm_status st = from_user_order(c, disp, c->disp)) return st;
  if (pm_status st = from_user_order(c, vel, c->vel)) return st;
  c->ics_done = true;
  c->ran = true;  // any state may be pulled back by pm_adjoint after a run
  return PM_OK;
}

pm_status pm_deposit(pm_ctx* c, const float* disp, int32_t mak, int64_t* mesh_out) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!disp || !mesh_out || (mak != 2 && mak != 3 && mak != 4 && mak != 6)) return PM_EINVAL;
  if (mak == 6 && c->cfg.force != PM_FORCE_NUFFT)
    return fail(c, PM_EINVAL, "ES spreading needs a NUFFT context");
  if (mak == 4 && c->cfg.mak != 4) return fail(c, PM_EINVAL, "the PCS deposit needs a PCS context (its windows)");
  if (pm_status st = from_user_order(c, disp, c->disp)) return st;  // the hooks use the particle state
  float* x = c->disp;
  const unsigned long long act = all_mask(c->cfg.batch);
  if (mak != 6) return deposit(c, x, nullptr, nullptr, mak, (long long*)mesh_out, act);
  pm_status st = bin(c, x, nullptr, nullptr, 2, act, kEsAnchor);
  if (st) return st;
  TileArgs t = tile_args(c, x, act);
  t.es_tab = c->d_es_tab;
  AssembleArgs as = assemble_args(c, kEsHaloLo, kEsHaloHi, mesh_out, act);
  KLAUNCH(c, PM_K_DEPOSIT, both(launch_tile_es(t, TK_ES_DEPOSIT, c->stream), launch_assemble(as, false, c->stream)));
  return PM_OK;
}

pm_status pm_force(pm_ctx* c, const float* disp, double s, float* acc_out) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!disp || !acc_out) return PM_EINVAL;
  const int B = c->cfg.batch;
  std::vector<double> sv(B, s);
  const unsigned long long act = all_mask(B);
  if (pm_status st = from_user_order(c, disp, c->disp)) return st;  // the hooks use the particle state
  pm_status st = potential(c, c->disp, nullptr, nullptr, sv.data(), act);
  if (st) return st;
  st = kick(c, c->disp, nullptr, nullptr, nullptr, c->vel, act);
  if (st) return st;
  return to_user_order(c, c->vel, acc_out);
}

pm_status pm_force_vjp(pm_ctx* c, const float* disp, double s, const float* u, int32_t parts, float* xbar_out) {
  if (c) c->tangent_valid = false;
  if (pm_status st = check_bound(c)) return st;
  if (!c->with_adj) return fail(c, PM_ESTATE, "workspace bound without adjoint buffers");
  if (!disp || !u || !xbar_out || parts < 1 || parts > 3) return PM_EINVAL;
  const int B = c->cfg.batch;
  const long long N = c->g.N;
  const size_t bytes = sizeof(float) * 3 * N * B;
  const unsigned long long act = all_mask(B);
  if (pm_status st = from_user_order(c, disp, c->disp)) return st;
  if (pm_status st = from_user_order(c, u, c->vbar)) return st;
  KLAUNCH(c, PM_K_FILL, launch_fill(c->vel, (long long)bytes, c->stream));
  KLAUNCH(c, PM_K_FILL, launch_fill(c->xbar, (long long)bytes, c->stream));
  std::vector<double> sv(B, s), one(B, 1.0), zero(B, 0.0);
  pm_status st = potential(c, c->disp, nullptr, nullptr, sv.data(), act);
  if (st) return st;
  // alpha = beta = 1, tau = 0: X_bar = J_A^T u, the drift is the identity
  st = reverse_force_step(c, sv.data(), one.data(), one.data(), zero.data(), act, parts);
  if (st) return st;
  if (pm_status st = to_user_order(c, c->xbar, xbar_out)) return st;
  c->ics_done = true;
  c->ran = false;
  return PM_OK;
}

pm_status pm_fft(pm_ctx* c, const void* in, void* out, int32_t inverse) {
  if (pm_status st = check_bound(c)) return st;
  if (!in || !out) return PM_EINVAL;
  const int n = c->cfg.n_g, B = c->cfg.batch;
  const unsigned long long act = all_mask(B);
  const long long nh = n / 2 + 1, cn = (long long)n * n * nh;  // compact user layout
  if (!inverse) {
    pm_status st = r2c_mesh(c, in, SRC_F32, c->g.mesh_stride, 1.0, 0.0, c->spec, c->g.spec_stride, n, true, act);
    if (st) return st;
    for (int b = 0; b < B; ++b)
      HIPCHK(c, hipMemcpy2DAsync((float2*)out + b * cn, sizeof(float2) * nh, c->spec + b * c->g.spec_stride,
                                 sizeof(float2) * spec_rs(n), sizeof(float2) * nh, (size_t)n * n,
                                 hipMemcpyDeviceToDevice, c->stream));
    return PM_OK;
  }
  for (int b = 0; b < B; ++b)
    HIPCHK(c, hipMemcpy2DAsync(c->spec + b * c->g.spec_stride, sizeof(float2) * spec_rs(n),
                               (const float2*)in + b * cn, sizeof(float2) * nh, sizeof(float2) * nh,
                               (size_t)n * n, hipMemcpyDeviceToDevice, c->stream));
  ColArgs a{};
  a.data = c->spec;
  a.slot_stride = c->g.spec_stride;
  a.n = n;
  a.nh = n / 2 + 1;
  a.rs = spec_rs(n);
  a.tw = c->d_tw;
  a.tws = c->Lmax / n;
  a.active = act;
  a.axis = 0;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_INV, B, c->stream));
  a.axis = 1;
  KLAUNCH(c, PM_K_FFT_COLS, fft_cols(a, MODE_INV, B, c->stream));
  RowLaunch rl{};
  rl.n = n;
  rl.rs = spec_rs(n);
  rl.n_rows = (long long)n * n;
  rl.batch = B;
  rl.inverse = true;
  rl.dst_mode = DST_F32;
  rl.src = c->spec;
  rl.src_stride = c->g.spec_stride;
  rl.dst = out;
  rl.dst_stride = c->g.mesh_stride;
  rl.tw = c->d_tw;
  rl.tws_half = c->Lmax / (n / 2);
  rl.tws_full = c->Lmax / n;
  rl.scale = 1.0;
  rl.stream = c->stream;
  rl.active = act;
  KLAUNCH(c, PM_K_FFT_ROWS, fft_rows(rl));
  return PM_OK;
}

}  // extern "C"
