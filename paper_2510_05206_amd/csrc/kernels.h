// Launch interface of the particle/mesh and auxiliary kernels.
#pragma once
#include "pm_internal.h"

namespace pm {

struct DepositArgs {
  Geom g;
  int batch;
  float* disp;             // [B][3][N]
  const float* vel;        // non-null: drift X += tau V first and write X back
  long long* mesh;         // [B][M] int64 (must be zero on entry)
  float tau[kMaxBatch];
  unsigned long long active;  // bit b set: slot b takes part
};

enum { GK_KICK = 0, GK_ADJ_KICK = 1, GK_ADJ_DRIFT = 2 };

struct GatherArgs {
  Geom g;
  int batch;
  float* disp;
  float* vel;
  float* xbar;
  float* vbar;
  const float* phi;        // potential (kick) or mesh cotangent (adjoint drift)
  float* gbar;             // [B][3][M] cotangent meshes (adjoint kick)
  float* acc_out;          // force-only output (test hook)
  float alpha[kMaxBatch];
  float beta[kMaxBatch];
  float tau[kMaxBatch];
  float coef[kMaxBatch];
  unsigned long long active;  // bit b set: slot b takes part
};

hipError_t launch_deposit(const DepositArgs& a, int mak, hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, int kind, int mak, int fd_order, hipStream_t s);
hipError_t launch_fd_div(const float* gbar, float* d, const Geom& g, int batch, int fd_order,
                         unsigned long long active, hipStream_t s);

// auxiliary kernels (misc.hip)
hipError_t launch_fill(void* p, long long bytes, hipStream_t s);
hipError_t launch_white_noise(float* w, long long N, long long slot_stride, int batch,
                              const uint64_t* seeds_host, hipStream_t s);
hipError_t launch_psibar(const float* xbar, const float* vbar, float* out, long long N,
                         long long part_stride, int batch, const float* d0, hipStream_t s);
hipError_t launch_dot(const float* a, const float* b, long long n, long long stride, int batch,
                      double* partial, double* out, const double* scale, hipStream_t s);
hipError_t launch_i64_to_delta(const long long* m, float* delta, long long M, long long stride,
                               int batch, double scale, hipStream_t s);
hipError_t launch_pk(const float2* spec, long long slot_stride, int n, int batch, int n_bins,
                     double kf, double norm, const double* cic4, int deconv, double* partial,
                     double* k_mean, double* pk, long long* n_modes, hipStream_t s);

// ES / NUFFT kernels (nufft.hip)
struct EsArgs {
  Geom g;                  // n_g = fine grid n_f
  int batch;
  int width;
  float* disp;
  float* vel;
  const float* vel_pre;    // deposit: merged drift
  long long* mesh;
  const float* force3;     // [B][3][M] interpolation meshes
  float* acc_out;
  const int32_t* tab;      // integer ES table
  float alpha[kMaxBatch], beta[kMaxBatch], tau[kMaxBatch];
  unsigned long long active;  // bit b set: slot b takes part
};
hipError_t launch_es_deposit(const EsArgs& a, hipStream_t s);
hipError_t launch_es_gather(const EsArgs& a, hipStream_t s);

}  // namespace pm
