// Launch interface of the particle/mesh and auxiliary kernels.
#pragma once
#include "pm_internal.h"

namespace pm {

// ------------------------------------------------ tile-binned kernels (binned.hip)
struct BinArgs {
  Geom g;
  int batch;
  unsigned long long active;
  float* disp;             // [B][3][N]; drifted in place when vel != null
  const float* vel;
  float tau[kMaxBatch];
  int log2T, log2nt, n_tiles;
  long long ts;            // ints per slot of count / offset
  int32_t* key;            // [B][N] tile of each particle
  int32_t* rank;           // [B][N] rank inside its tile
  int32_t* sorted;         // [B][N] particle indices grouped by tile
  int32_t* count;          // [B][ts], zero on entry
  int32_t* offset;         // [B][ts], n_tiles + 1 entries used
  int home_shift;          // bin by home node - home_shift (ES: the first stencil node)
  int32_t* scan_partial;   // [B][scan_np] block totals of the count scan
  int scan_np;
};

enum { TK_DEPOSIT = 0, TK_KICK = 1, TK_ADJ_KICK = 2, TK_ADJ_DRIFT = 3, TK_DIPOLE = 4, TK_ES_DEPOSIT = 5,
       TK_ES_KICK = 6, TK_ES_ADJ_KICK = 7, TK_ES_DIPOLE = 8, TK_ES_ADJ_DRIFT = 9, TK_TAN_SPREAD = 10,
       TK_TAN_DIRECT = 11, TK_TAN_KICK = 12, TK_ES_TAN_KICK = 13 };

struct TileArgs {
  Geom g;
  int batch;
  unsigned long long active;
  int T, log2T, log2nt, n_tiles;
  long long ts;
  const int32_t* sorted;
  const int32_t* offset;
  const int32_t* bank;     // ES spreads: positions into sorted, per tile in LDS-bank order
  float* disp;
  float* vel;
  float* xbar;
  float* vbar;
  const float* mesh_in;    // potential (kicks) or mesh cotangent (adjoint drift)
  const float* mesh_in2;   // ES tangent kick: the tangent force meshes
  int tan_xbar;            // ES gradient spread of the tangent positions (xbar, times coef)
  void* scratch;           // window slab [B][n_tiles][W^3] int64
  float* acc_out;          // force-only output
  const float* acc_in;     // interlaced grids: the other grid's forces, averaged in the kick
  // interlaced grids, reverse pass ([B][6][N]): the second grid's adjoint kick
  // writes its force (3) and direct position term (3) to il_out, the adjoint
  // drift of the first grid writes its scatter term (3); the other grid's
  // pass averages its own with il_in
  float* il_out;
  const float* il_in;
  float* u_sorted;         // [B][3][N] u = beta V_bar in sorted order
  float* umax;             // [B] max |u| (as uint bits)
  const double* scale;     // [B] fixed-point scale of the cotangent scatter
  const int32_t* es_tab;   // integer exponential-of-semicircle table (NUFFT)
  // ES spreads into a force chain: the window is stored as FP32 partial
  // sums, acc * win_scale (or acc * inv_scale[slot] when win_scale is 0),
  // instead of int64 (the exact path for the deposited mesh itself)
  int win_f32;
  double win_scale;
  const double* inv_scale;
  float es_beta;           // its shape parameter (closed-form derivative)
  long long comp_stride;   // floats between the 3 force meshes (NUFFT kick)
  float alpha[kMaxBatch];
  float beta[kMaxBatch];
  float tau[kMaxBatch];
  float coef[kMaxBatch];
};

struct AssembleArgs {
  Geom g;
  int batch;
  unsigned long long active;
  int T, Rlo, Rhi, log2T, log2nt, n_tiles;  // window halo below / above
  const void* scratch;
  void* out;               // int64 mesh, or float mesh (below)
  // float output: acc * inv_scale[slot] when inv_scale is set (fixed-point
  // dipole meshes), else (double)acc * scale - shift (mass meshes)
  const double* inv_scale;
  double scale, shift;
  int slab_f32;            // the windows are FP32 partial sums: out = sum - shift
};

hipError_t launch_binning(const BinArgs& a, int mak, hipStream_t s);
hipError_t launch_tile(const TileArgs& a, int kind, int mak, int fd_order, hipStream_t s);
hipError_t launch_assemble(const AssembleArgs& a, bool out_f32, hipStream_t s);
hipError_t launch_tile_es(const TileArgs& a, int kind, hipStream_t s);
// the ES spreads' order of each tile's entries of `sorted` (bank, [B][N]
// positions into sorted), which spreads a wave's window bases over the LDS
// banks
hipError_t launch_es_bank_order(const TileArgs& a, int32_t* bank, hipStream_t s);
hipError_t configure_tile_kernels();
hipError_t launch_dipole_scale(const unsigned int* umax_bits, double* scale, double* inv_scale,
                               double bound_per_u, double node_per_u, int batch, hipStream_t s);

// auxiliary kernels (misc.hip)
hipError_t launch_fill(void* p, long long bytes, hipStream_t s);
struct SlotCoef {
  float v[kMaxBatch];
};
// out = a + coef[slot] x over n floats per slot (slot stride n)
hipError_t launch_lincomb(const float* a, const float* x, float* out, long long n, const SlotCoef& coef, int batch,
                          unsigned long long active, hipStream_t s);
// out = a b elementwise over n floats per slot (slot strides sa, sb, so)
hipError_t launch_mul(const float* a, long long sa, const float* b, long long sb, float* out, long long so,
                      long long n, int batch, unsigned long long active, hipStream_t s);
// xd += tau[slot] vd over n floats per slot (stride `stride`), then
// amax[slot] = max(amax[slot], max |xd|) as float bits (amax starts at 0)
hipError_t launch_tan_drift(float* xd, const float* vd, long long n, long long stride, const SlotCoef& tau,
                            unsigned int* amax, int batch, unsigned long long active, hipStream_t s);
// device-indexed step state (by-value uploads, no host buffers in flight)
constexpr int kMaxSchedSteps = 96;   // steps per slot a device schedule holds
struct GateSet {
  int32_t k[kMaxBatch];
  int batch;
};
struct SchedRows {
  float v[kMaxSchedSteps * kSch];
  int n, slot, stride;
};
hipError_t launch_set_gate(int32_t* gate, const GateSet& g, hipStream_t s);
hipError_t launch_advance_gate(int32_t* gate, const int32_t* nsteps, int batch, hipStream_t s);
hipError_t launch_set_sched(float* sched, int32_t* nsteps, const SchedRows& r, hipStream_t s);
hipError_t launch_white_noise(float* w, long long N, long long slot_stride, int batch,
                              const uint64_t* seeds_host, unsigned long long active, hipStream_t s);
hipError_t launch_psibar(const float* xbar, const float* vbar, float* out, long long N,
                         long long part_stride, int batch, const float* d0, int log2_np, int log2_pb,
                         unsigned long long active, hipStream_t s);
hipError_t launch_reorder(const float* src, float* dst, long long N, long long stride, int ncomp, int batch,
                          int log2_np, int log2_pb, bool to_blocked, unsigned long long active, hipStream_t s);
hipError_t launch_dot(const float* a, const float* b, long long n, long long stride, int batch,
                      double* partial, double* out, const double* scale, unsigned long long active,
                      hipStream_t s, const long long* out_idx = nullptr);
struct TimeAB {
  double alpha[kMaxBatch], beta[kMaxBatch];
  long long idx[kMaxBatch];  // first element of the slot's (tau1, tau2, alpha, beta) row
};
hipError_t launch_time_ab(const double* d1, const double* d2, double* out, const TimeAB& t,
                          unsigned long long active, hipStream_t s);
hipError_t launch_i64_to_delta(const long long* m, float* delta, long long M, long long stride,
                               int batch, double scale, unsigned long long active, hipStream_t s);
hipError_t launch_pk(const float2* spec, long long slot_stride, int n, int batch, int n_bins,
                     double kf, double norm, const double* cic4, int deconv, double* partial,
                     double* k_mean, double* pk, long long* n_modes, unsigned long long active,
                     int rs, hipStream_t s, const float2* spec2 = nullptr);

}  // namespace pm
