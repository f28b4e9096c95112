// Internal declarations shared by the host tables, the kernels and the C ABI
// of libpm.so.  Not part of the public interface (include/pm.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pm.h"

namespace pm {

constexpr int kMaxBatch = 64;    // slots per context (per-step scalars travel by value)
constexpr int kFracBits = 20;    // fixed-point fraction bits of a mesh coordinate
constexpr int kWeightBits = 20;  // bits of a 1D integer weight (sums to 2^20)
constexpr int kMassBits = 32;    // mass unit per particle: 2^32
constexpr int kEsTabPerCell = 4096;
// width-6 ES stencil: nodes floor(u) - 2 .. floor(u) + 3.  Particles are
// binned by the first node (anchor shift 2), so the tile window covers the
// tile and 5 cells above it on each axis
constexpr int kEsAnchor = 2;
constexpr int kEsHaloLo = 0, kEsHaloHi = 5;

// ---------------------------------------------------------------- host FP64
struct StepCoef {          // one drift-kick-drift step (Sec. "Time stepping")
  double D_n, D_half, D_np1, alpha, beta, tau1, tau2, s;
};

struct Growth {            // D(a), E(a) of the growth ODEs (D ~ a normalisation)
  double omega_m = 1.0;
  bool eds = true;
  std::vector<double> lna, D, dD, E, dE;  // dX = dX/dln a
  void solve(double om);
  double D_of_a(double a) const;
  double a_of_D(double D) const;
  void at_D(double Dv, double* E, double* dEdD) const;
  double zeta(double a) const;  // H a^3 dD/da (FastPM)
};

// stepper 0 BullFrog, 1 FastPM, 2 leapfrog in the canonical momentum;
// time_var 0 uniform in D, 1 in a, 2 in ln a, 3 in superconformal time
std::vector<StepCoef> step_table(const Growth& g, double a_start, double a_end, int n_steps, int stepper,
                                 int time_var);
double bbks_amplitude(double omega_m, double h, double n_s, double sigma8);
double spectrum_eval(const pm_config& c, double amp, double k);
double powerlaw_amplitude(const pm_config& c, double D_start, double D_ref);
double es_phihat(double theta, int width, double beta);

// ------------------------------------------------------------- device args
struct SlotStep {          // per-slot scalars of one launch, passed by value
  float alpha[kMaxBatch];
  float beta[kMaxBatch];
  float tau_pre[kMaxBatch];   // drift applied before the deposit (merged)
  float tau_post[kMaxBatch];  // drift applied after the kick
  float s[kMaxBatch];         // 1/D_{n+1/2}^2
  int32_t active[kMaxBatch];
};

struct Geom {
  int n_p, n_g, log2_np, log2_ng, log2_r;  // r = n_g / n_p
  int log2_pb;                // particle storage: lattice blocks of 2^log2_pb per axis
  long long N, M;             // particles, mesh cells (per slot)
  long long part_stride;      // floats between slots of a [3][N] array
  long long mesh_stride;      // elements between slots of a mesh
  long long spec_stride;      // float2 between slots of a half spectrum
  // device-indexed steps (pm_step_device): when gate is set, slot b takes
  // part only while gate[b] >= 0, and its step scalars come from
  // sched[(b sched_steps + gate[b]) kSch + field] instead of the by-value
  // arrays of the launch
  const int32_t* gate;
  const float* sched;
  int sched_steps;
  // interlaced grids: added to every fixed-point mesh coordinate of the PM
  // tile kernels (half a cell, 2^19, for the second grid; 0 otherwise)
  long long ushift;
};

// fields of one device schedule row (the same floats the by-value path passes)
enum { kSchTau1 = 0, kSchAlpha = 1, kSchBeta = 2, kSchTau2 = 3, kSchCoef = 4, kSch = 5 };

__host__ __device__ __forceinline__ bool slot_on(const int32_t* gate, unsigned long long active, int slot) {
  return ((active >> slot) & 1ull) && (gate == nullptr || gate[slot] >= 0);
}
__host__ __device__ __forceinline__ float slot_f(const int32_t* gate, const float* sched, int sched_steps,
                                                 const float* byval, int slot, int field) {
  return gate ? sched[((long long)slot * sched_steps + gate[slot]) * kSch + field] : byval[slot];
}

}  // namespace pm
