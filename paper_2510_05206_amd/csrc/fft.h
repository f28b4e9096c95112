// Launch interface of the FFT passes (fft.hip).
#pragma once
#include "pm_internal.h"

namespace pm {

enum { SRC_I64 = 0, SRC_F32 = 1 };
// row epilogues: DST_F32 real rows; DST_IC the Zel'dovich state; on the
// second-order LPT grid (twice the lattice per axis) DST_MU_AB / DST_MU_ACC /
// DST_MU_SQ accumulate the source mu from the derivative fields (dst = A, the
// running diagonal sum, dst2 = mu), DST_IC2 adds the second-order term at the
// lattice points (even nodes) to the state.  Reverse pass through the second
// order: DST_ACC adds the row to dst; DST_GBAR_DIAG / DST_GBAR_OFF write the
// cotangent of a derivative field g (the row) into dst: mu_bar (S - g) for a
// diagonal field, -2 mu_bar g for an off-diagonal one, with mu_bar and the
// diagonal sum S read from dst2 and dst2 + dst_stride (slot stride
// 2 dst_stride there)
enum { DST_F32 = 0, DST_IC = 1, DST_MU_AB = 2, DST_MU_ACC = 3, DST_MU_SQ = 4, DST_IC2 = 5, DST_ACC = 6,
       DST_GBAR_DIAG = 7, DST_GBAR_OFF = 8 };
enum { MODE_FWD = 0, MODE_INV = 1, MODE_FUSED_H = 2, MODE_IC_C = 3, MODE_COMBINE_IC = 4, MODE_NUFFT_C = 5,
       MODE_NUFFT_ADJ = 6, MODE_LPT_D = 7, MODE_FUSED_IL = 8, MODE_LPT_MUBAR = 9, MODE_LPT_DT = 10 };

// z-row pass: real rows of n <-> half-spectrum rows of n/2+1
struct RowLaunch {
  int n;                 // row length of the real mesh
  long long n_rows;      // rows per slot (n^2)
  int batch;
  bool inverse;
  int src_mode, dst_mode;
  const void* src;
  long long src_stride;  // elements between slots
  void* dst;
  long long dst_stride;
  void* dst2;            // DST_IC: displacement output
  const float2* tw;
  int tws_half, tws_full;  // twiddle strides for the n/2 FFT and for exp(-2 pi i k/n)
  double scale, shift, scale2;
  unsigned long long active;  // bit b set: slot b takes part
  int rs;                     // row stride of the half spectrum (float2), >= n/2 + 1
  // pruning (truncated spectra): R2C writes and C2R reads only k < kz_lim
  // (the rest is zero); 0 = the whole half row
  int kz_lim;
  int ic_log2pb;         // DST_IC: particle arrays in lattice blocks of 2^ic_log2pb (mak.h)
  const int32_t* gate;   // device-indexed steps: slot b takes part while gate[b] >= 0 (null: all)
  hipStream_t stream;
};

// strided complex pass along y (axis 1) or x (axis 0) of a half spectrum
struct ColArgs {
  float2* data;        // in-place spectrum (MODE_COMBINE_IC: output)
  const float2* src3;  // MODE_COMBINE_IC: 3 input spectra, spaced by comp_stride
  float2* dst3;        // MODE_IC_C: output spectrum
  long long slot_stride, comp_stride;
  int n, nh, axis;
  int rs;              // row stride of the half spectrum (float2), >= nh
  const float2* tw;
  int tws;             // Lmax / n
  // PM multiplier H = coef / ((lap[ix]+lap[iy]+lap[iz]) win2[ix] win2[iy] win2[iz]), 0 at k = 0
  // (MODE_FUSED_IL, interlaced grids: the x pass of grid 1 averages its
  // spectrum with the x-transformed spectrum of grid 2 in src3, phase
  // e^{i phi}, phi = (theta_x + theta_y + theta_z)/2, applies H, writes
  // H delta e^{-i phi} to dst3 (the same array) for grid 2 and inverts x for
  // grid 1)
  const float* lap;
  const float* win2;
  float coef[kMaxBatch];
  // IC multiplier h_c = i m_c amp[|m|^2] fac
  const float* amp;
  float fac[kMaxBatch];
  int comp;
  // NUFFT multiplier for component comp (x pass): i theta_c / |theta|^2 * coef *
  // esdec[ix] esdec[iy] esdec[iz], theta = 2 pi m / n_p; esdec is 1/phi_hat^2 on
  // the kept modes |m| < n_p/2 and 0 elsewhere (truncation)
  const float* esdec;
  int n_p;
  // MODE_LPT_D (x pass on the padded second-order grid, n = 2 n_p): the
  // derivative field psi_{comp, comp2} = -(2 pi / n_p) m_comp m_comp2 amp fac w
  // of the particle-grid noise spectrum src3 (row stride src_rs, slot stride
  // src_slot_stride), zero-padded to the modes |m| < n_p / 2, into dst3
  int comp2, src_rs;
  long long src_slot_stride;
  // MODE_LPT_MUBAR (x pass on the padded grid): sum_c conj(h_c) S_c of the
  // three particle-grid spectra S_c in src3 (comp_stride apart), h_c = i coef
  // k_c / |k|^2 on the kept modes (the transpose of the second-order
  // multiplier), zero-padded, then the inverse x transform
  // MODE_LPT_DT (x pass on the padded grid, forward): the transpose of
  // MODE_LPT_D, its real multiplier for (comp, comp2) times the transformed
  // field, added into the particle-grid spectrum dst3 on the kept modes
  // MODE_COMBINE_IC with combine_add: the combination is added to the
  // spectrum already in data
  int combine_add;
  unsigned long long active;  // bit b set: slot b takes part
  // pruning for spectra truncated to |m| < keep/2 per axis (keep = 0: none):
  // only columns iz < zlim (0 = all nh); keep_in: indices along the pass
  // outside the kept set are zero and not read; keep_out: they are not
  // written; keep_outer: whole lines whose outer index is not kept are skipped
  int zlim, keep, keep_in, keep_out, keep_outer;
  // device-indexed steps (Geom): gate, and MODE_FUSED_H's coef from sched
  const int32_t* gate;
  const float* sched;
  int sched_steps;
};

hipError_t fft_rows(const RowLaunch& r);
hipError_t fft_cols(const ColArgs& a, int mode, int batch, hipStream_t s);

}  // namespace pm
