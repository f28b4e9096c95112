/* pm.h - C ABI of the MI355X particle-mesh hot path (libpm.so).
 *
 * Differentiable particle-mesh N-body step of DISCO-DJ II (arXiv:2510.05206):
 * Zel'dovich initial conditions, BullFrog drift-kick-drift steps with a PM
 * (CIC/TSC) or exponential-of-semicircle NUFFT force, the binned power
 * spectrum, and the adjoint (reverse-in-time) gradient of a loss on the final
 * density with respect to the white-noise field and sigma8.
 *
 * Conventions shared by every call
 * --------------------------------
 * Memory.   The library never allocates device memory.  The caller passes a
 *           device workspace (pm_bind) of at least pm_workspace_bytes() bytes
 *           and owns every device buffer; the context keeps raw pointers only
 *           between pm_bind and pm_destroy.  Host arrays are copied during
 *           the call.  Device pointers must be 256-byte aligned.
 * Streams.  All device work is enqueued on the stream given to pm_bind and is
 *           asynchronous; calls return after enqueueing.  pm_power_spectrum
 *           and pm_adjoint write device outputs only.
 * Errors.   Every call returns a pm_status; pm_last_error(ctx) gives a message.
 *           Arguments are validated before any launch, so a failed call leaves
 *           the state unchanged.  Launch failures return PM_EHIP.  Calls made
 *           out of order (for example pm_adjoint before pm_run) return
 *           PM_ESTATE.  Nothing aborts and no C++ exception crosses the ABI.
 * Threads.  A context is not thread-safe; distinct contexts on distinct
 *           streams are independent.
 * Batch.    A context holds B same-shape slots ("batch").  Per-slot arrays
 *           ([B]...) are laid out slot-major.  Slots share the cosmology and
 *           the mesh, and each has its own seed, sigma8 and number of steps.
 * Units.    Particle state is exchanged in lattice units: the displacement
 *           Psi from the Lagrangian lattice point q_j = j L/n_p in units of
 *           dq = L/n_p, and V = dPsi/dD in dq per unit of the growth factor D
 *           (D ~ a at early times).  Layout [B][3][N], N = n_p^3, lattice
 *           index j = (jx n_p + jy) n_p + jz at every call (inside, the
 *           context keeps particles in lattice blocks that match its mesh
 *           tiles).  Meshes are [B][n_g][n_g][n_g] with z fastest.
 * Determinism.  The forward deposit accumulates int64 fixed point (2^32 per
 *           particle) and the adjoint's cotangent scatter int64 fixed point
 *           at a power-of-two scale, so results are bit-identical run to run
 *           and slot to slot.
 */
#ifndef PM_H
#define PM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm_ctx pm_ctx;

typedef enum {
  PM_OK = 0,
  PM_EINVAL = -1,       /* invalid argument or configuration                   */
  PM_ENOMEM = -2,       /* workspace smaller than pm_workspace_bytes()         */
  PM_EHIP = -3,         /* a HIP call or kernel launch failed                  */
  PM_ESTATE = -4,       /* call out of order (e.g. step before init_ics)       */
  PM_EUNSUPPORTED = -5  /* valid but not implemented combination               */
} pm_status;

enum { PM_FORCE_PM = 0, PM_FORCE_NUFFT = 1 };
enum { PM_SPEC_POWERLAW = 0, PM_SPEC_BBKS = 1 };

/* Run configuration (Sec. "Validation and performance", tab. default_parameters
 * for the knobs; Sec. "Time stepping" for the schedule).
 *   n_p            particles per dimension (power of two, 4..1024)
 *   n_g            PM mesh per dimension; NUFFT: fine grid n_f = sigma n_p.
 *                  n_g / n_p must be a power of two (1, 2 or 4)
 *   box            L in Mpc/h
 *   omega_m, h, n_s, sigma8   flat LCDM (omega_m = 1 is EdS, D = a)
 *   spectrum       PM_SPEC_BBKS: P = A k^n_s T_BBKS^2 normalised to sigma8;
 *                  PM_SPEC_POWERLAW: P = A k^-2 exp(-(k/k_c)^2), k_c half the
 *                  particle Nyquist wavenumber, A from pl_rms_cells (expected
 *                  3D rms displacement at a_start in PM-mesh cells)
 *   a_start, a_end, n_steps   uniform steps in D between D(a_start), D(a_end)
 *   force          PM_FORCE_PM or PM_FORCE_NUFFT
 *   mak            2 = CIC, 3 = TSC, 4 = PCS with grad_order 2 or 4
 *                  (tab. interpolation_kernels; PM force; the final density and P(k) are
 *                  always CIC)
 *   deconvolve     divide the PM multiplier by the squared window
 *   grad_order     0 exact i k (NUFFT only), 2/4/6 finite differences (PM)
 *   lap_order      0 exact -k^2, 2/4/6 finite differences
 *   es_width, es_beta   NUFFT exponential-of-semicircle kernel (width 6);
 *                  NUFFT needs n_g = 2 n_p and n_p >= 8
 *   batch          number of same-shape slots B >= 1
 *   lpt_order      initial state from the LPT series of Sec. "Lagrangian
 *                  perturbation theory" (eq. LPT, D^n approximation): 1 (or
 *                  0) Zel'dovich, 2 adds D^2 psi^(2) (eq. LPT_L at n = 2,
 *                  eq. helmholtz; de-aliased products).  2 needs
 *                  n_g >= 2 n_p and n_p >= 8; pm_adjoint and pm_jvp
 *                  differentiate through the second-order term as well
 *   stepper        0 BullFrog, 1 FastPM (velocity V = dX/dD); 2 the
 *                  symplectic leapfrog in the canonical momentum V = a^2 dX/dt
 *                  (H0 = 1, lengths in lattice units; the initial V is
 *                  zeta(a_start) = H a^3 dD/da times dX/dD) (Sec. "Time
 *                  stepping")
 *   time_var       step spacing: 0 uniform in D, 1 in a, 2 in ln a, 3 in
 *                  superconformal time (dt / a^2)
 *   antialias      1: interlaced grids for the PM force (Sec. "Discreteness
 *                  suppression"; antialias of tab. default_parameters), a
 *                  second deposit half a cell down the diagonal, the two
 *                  spectra averaged with the shift's phase and the two
 *                  gathers averaged (the adjoint and pm_force_vjp average
 *                  the two grids' terms likewise); PM force with n_g >= 16
 *                  only; the device-indexed steps return PM_EUNSUPPORTED
 *                  for it
 */
typedef struct {
  int32_t n_p, n_g;
  double box;
  double omega_m, h, n_s, sigma8;
  int32_t spectrum;
  double pl_rms_cells;
  double a_start, a_end;
  int32_t n_steps;
  int32_t force, mak, deconvolve, grad_order, lap_order;
  int32_t es_width;
  double es_beta;
  int32_t batch;
  int32_t lpt_order;
  int32_t stepper;
  int32_t time_var;
  int32_t antialias;
} pm_config;

/* Lifecycle ------------------------------------------------------------- */

/* Validate cfg and build the host tables in FP64 (growth functions, BullFrog
 * coefficients, spectrum normalisation, FFT twiddles, Fourier multipliers).
 * Host only; *out receives the context, or NULL on error. */
pm_status pm_create(const pm_config* cfg, pm_ctx** out);

/* Device workspace needed by this context: particle state for B slots plus
 * one set of meshes per slot.  with_adjoint != 0 adds the cotangent state
 * and the adjoint meshes.  This number is what admission control uses. */
size_t pm_workspace_bytes(const pm_ctx* ctx, int32_t with_adjoint);

/* Attach a device workspace (256-byte aligned, owned by the caller) and a
 * hipStream_t (NULL = default stream), upload the tables (asynchronously on
 * that stream).  with_adjoint must match the size passed. */
pm_status pm_bind(pm_ctx* ctx, void* workspace, size_t bytes, int32_t with_adjoint,
                  void* hip_stream);

pm_status pm_destroy(pm_ctx* ctx);

/* Last error message of this context (never NULL; "" if none). */
const char* pm_last_error(const pm_ctx* ctx);

/* Host-side schedule of one slot: n_steps rows of 8 doubles
 * (D_n, D_{n+1/2}, D_{n+1}, alpha, beta, tau1, tau2, s = 1/D_{n+1/2}^2), the
 * BullFrog coefficients of Sec. "Time stepping" computed in FP64. */
pm_status pm_schedule(const pm_ctx* ctx, int32_t slot, double* out);

/* out[0] = D(a_start), out[1] = D(1) (D ~ a normalisation), out[2] = the
 * linear-spectrum amplitude A (P = A k^n_s T^2, or A k^-2 exp(-(k/k_c)^2)). */
pm_status pm_describe(const pm_ctx* ctx, double* out);

/* Kernel classes timed by pm_profile (HIP events on the bound stream). */
enum {
  PM_K_FILL = 0,        /* zeroing of counters and cotangents            */
  PM_K_DEPOSIT = 1,     /* fixed-point mass assignment: tile windows + halo sum into the mesh */
  PM_K_FFT_ROWS = 2,    /* z-row real<->complex FFT passes               */
  PM_K_FFT_COLS = 3,    /* y/x strided passes (incl. the fused multiplier) */
  PM_K_GATHER_KICK = 4, /* force gather + kick + drift                   */
  PM_K_ADJ_KICK = 5,    /* adjoint kick: reverse kick, direct X_bar       */
  PM_K_DIPOLE = 6,      /* transposed force gather of the cotangent: tile windows + halo sum */
  PM_K_ADJ_DRIFT = 7,   /* scatter-position VJP + reverse drifts          */
  PM_K_MISC = 8,        /* RNG, P(k), reductions, conversions            */
  PM_K_BIN = 9,         /* counting sort of particles by mesh tile        */
  PM_K_COUNT = 10
};

/* Enable (on != 0) or disable per-launch event timing of the kernel classes
 * above.  Adds two event records per launch; off by default. */
pm_status pm_profile(pm_ctx* ctx, int32_t on);

/* Synchronise the bound stream, then return and reset the accumulated time
 * (ms[PM_K_COUNT], milliseconds) and launch count (launches[PM_K_COUNT]) per
 * kernel class since the previous call.  Host arrays. */
pm_status pm_kernel_times(pm_ctx* ctx, double* ms, int64_t* launches);

/* Restrict pm_init_ics, pm_step, pm_run, pm_adjoint, pm_power_spectrum and
 * pm_density to the slots whose bit is set in mask (default: all B slots);
 * the other slots' state and outputs are left untouched.  This is how a
 * serving loop refills and reads out single slots of a running batch.
 * PM_EINVAL for an empty mask or bits beyond the batch. */
pm_status pm_set_active(pm_ctx* ctx, uint64_t mask);

/* Change the per-slot number of steps (1..n_steps_max of pm_create) and
 * sigma8 before pm_init_ics; NULL keeps the current values. */
pm_status pm_set_slot_params(pm_ctx* ctx, const int32_t* n_steps, const double* sigma8);

/* The spec calls -------------------------------------------------- */

/* Zel'dovich initial conditions (Sec. "Lagrangian perturbation theory",
 * first order; Sec. "Time stepping" for V = dX/dD):
 *   w ~ N(0,1) on the particle lattice from Philox-4x32-10 keyed by seeds[b]
 *   (or copied from w_in, device [B][N], when non-NULL),
 *   psi_c = IDFT( i k_c / (k^2 D(1)) sqrt(P(k) n_p^3 / L^3) DFT(w) ), with
 *   k = 0, the Nyquist plane of component c and |k| > k_Nyq zeroed,
 *   Psi = D(a_start) psi, V = psi.
 * seeds: host [B].  w_out: optional device [B][N] copy of w. */
pm_status pm_init_ics(pm_ctx* ctx, const uint64_t* seeds, const float* w_in, float* w_out);

/* One BullFrog drift-kick-drift step (eq. dkd) per slot:
 *   X += tau1 V;  V = alpha V + beta A(X);  X += tau2 V
 * step_index: host [B], the step each slot takes (< its n_steps); a negative
 * entry leaves that slot idle. */
pm_status pm_step(pm_ctx* ctx, const int32_t* step_index);

/* All n_steps steps for every slot: bit-identical to pm_step(0 .. n-1).
 * Unless profiling is on or graphs are disabled (pm_use_graphs), the whole
 * launch sequence is captured once into a HIP graph and replayed on later
 * calls; the graph is rebuilt after pm_bind, pm_set_slot_params or a change
 * of pm_set_active.  Results are bit-identical to the eager launches. */
pm_status pm_run(pm_ctx* ctx);

/* Enable (default) or disable the HIP-graph replay of pm_run. */
pm_status pm_use_graphs(pm_ctx* ctx, int32_t enable);

/* Adjoint of the whole run (Sec. "Adjoint method", tab. adjoint_dkd): from
 * the final state, integrate primal and cotangents backwards in time with
 * memory independent of n_steps, then pull back through the initial
 * conditions.  dL_ddelta: device [B][n_g^3] cotangent of the final CIC
 * density contrast.  Outputs: dL_dw device [B][N], dL_dsigma8 device [B]
 * (double; 0 with PM_SPEC_POWERLAW, whose amplitude is set by its rms
 * displacement and not by sigma8).  Leaves the particle state at the
 * initial conditions. */
pm_status pm_adjoint(pm_ctx* ctx, const float* dL_ddelta, float* dL_dw, double* dL_dsigma8);

/* pm_adjoint plus the adjoints of the step scalars of tab. adjoint_dkd:
 * dL_dtime (device doubles [B][n_steps][4], n_steps of the configuration)
 * receives per slot and step n the row (dL/dtau1, dL/dtau2, dL/dalpha,
 * dL/dbeta) of V^{n+1} = alpha V^n + beta A, X^{n+1/2} = X^n + tau1 V^n,
 * X^{n+1} = X^{n+1/2} + tau2 V^{n+1}; rows beyond a slot's own step count are
 * zero.  FP64 dot products over the particles of the reverse pass's states;
 * dL/dbeta is formed as (V_bar . V^{n+1} - alpha V_bar . V^n) / beta, with
 * V_bar the cotangent of the kick's output.  dL_dtime = NULL is pm_adjoint. */
pm_status pm_adjoint_full(pm_ctx* ctx, const float* dL_ddelta, float* dL_dw, double* dL_dsigma8,
                          double* dL_dtime);

/* Device-indexed steps for continuous batching (serving): each slot's next
 * step index lives in device memory, so slots at different steps, admitted
 * at different times, advance together through one captured graph with no
 * per-step capture or argument upload.  pm_set_step_index sets the device
 * index of every slot from step_index[B] (host): k >= 0 runs step k of that
 * slot's schedule next, -1 makes it idle, -2 keeps its current value.
 * pm_step_device advances every slot whose index is >= 0 by one step of eq.
 * dkd (the same launches and scalars as pm_step) and then increments its
 * index, which returns to -1 after the slot's last step; idle slots cost a
 * launch but no work.  pm_get_step_index copies the indices to the host
 * (synchronising the stream).  The slot mask of pm_set_active does not apply
 * to these calls.  PM force contexts with n_steps <= 96 only
 * (PM_EUNSUPPORTED otherwise). */
pm_status pm_set_step_index(pm_ctx* ctx, const int32_t* step_index);
pm_status pm_step_device(pm_ctx* ctx);
pm_status pm_get_step_index(pm_ctx* ctx, int32_t* step_index);

/* Binned power spectrum of the CIC density of the current positions:
 * P(k_b) = (L^3/n_g^6) sum_{m in b} w_m |delta_m|^2 / W^2 / sum w_m, bin b
 * (1-based) holding (2b-1)^2 <= 4|m|^2 < (2b+1)^2, W the CIC window when
 * deconvolve_cic != 0.  FP64 sums in a fixed order (bit-reproducible).
 * Outputs are device [B][n_bins] arrays (k_mean in h/Mpc, pk in (Mpc/h)^3,
 * n_modes = sum of half-spectrum multiplicities). */
pm_status pm_power_spectrum(pm_ctx* ctx, int32_t n_bins, int32_t deconvolve_cic,
                            double* k_mean, double* pk, int64_t* n_modes);

/* Forward mode (Sec. "Automatic differentiation", forward mode; App.
 * "Custom VJP and JVP", subsection "VJP and JVP derivations"): the tangent
 * of the run along the direction (w_dot, sigma8_dot) of the white noise and
 * sigma8.  Reruns the forward from the white noise of the last pm_init_ics
 * while carrying the tangent positions and velocities (the JVP of a scatter
 * w.r.t. the positions is a scatter with the gradient kernel; of a gather,
 * a gather of the tangent mesh plus a gather with the gradient kernel), and
 * leaves the context at the run's final state (as pm_run).  w_dot: device
 * [B][N] in lattice order; sigma8_dot: host [B] or NULL (0; no effect with
 * the power-law spectrum, whose amplitude is not set by sigma8);
 * delta_dot_out: device [B][n_g^3], the tangent of the final CIC contrast.
 * Needs a workspace bound with adjoint buffers (the tangents use them;
 * PM_ESTATE otherwise); PM (single or interlaced grids) or NUFFT force.  With second-order initial conditions the tangent of psi2 is
 * its bilinear form in (psi, psi_dot). */
pm_status pm_jvp(pm_ctx* ctx, const float* w_dot, const double* sigma8_dot, float* delta_dot_out);

/* The tangent displacement and velocity of the final state after pm_jvp
 * (device [B][3][N], lattice order; either may be NULL).  PM_ESTATE unless
 * pm_jvp was the last call that moved the state. */
pm_status pm_get_tangent(pm_ctx* ctx, float* disp_dot, float* vel_dot);

/* pm_power_spectrum of the current state plus pk_dot (device [B][n_bins]),
 * the tangent of P(k_b) when the contrast moves along delta_dot (device
 * [B][n_g^3], e.g. from pm_jvp): the same bins of 2 Re(conj(delta_m)
 * delta_dot_m) / W^2. */
pm_status pm_power_spectrum_jvp(pm_ctx* ctx, const float* delta_dot, int32_t n_bins, int32_t deconvolve_cic,
                                double* k_mean, double* pk, double* pk_dot, int64_t* n_modes);

/* State access and single-kernel entry points (tests, loss, resume) ------- */

/* Final CIC density contrast delta = m n_g^3/N - 1 of the current positions
 * into delta_out (device [B][n_g^3] float), and optionally the raw int64
 * fixed-point mass mesh (2^32 per particle) into fixed_out. */
pm_status pm_density(pm_ctx* ctx, float* delta_out, int64_t* fixed_out);

/* Copy the particle state out of / into the context (device [B][3][N]). */
pm_status pm_get_state(pm_ctx* ctx, float* disp, float* vel);
pm_status pm_set_state(pm_ctx* ctx, const float* disp, const float* vel);

/* Deposit the given displacements (device [B][3][N]) with kernel order
 * mak (2 CIC, 3 TSC, 4 PCS in a PCS context, 6 = ES of the NUFFT grid) into
 * the int64 mesh mesh_out (device [B][n^3], n = n_g).  Bit-exact fixed-point
 * spec: CIC, TSC and PCS put 2^32 per particle; the ES spreading (Sec. "Force evaluation",
 * NUFFT paragraphs) puts floor(floor(w_x w_y / 2^17) w_z / 2^12) on each of
 * its 6^3 nodes from 20-bit 1D table weights, 2^31 at the kernel's peak.
 * This and the two hooks below load disp as the context's particle
 * positions (the previous state is overwritten). */
pm_status pm_deposit(pm_ctx* ctx, const float* disp, int32_t mak, int64_t* mesh_out);

/* PM (or NUFFT) acceleration A(X) at the given displacements for the
 * midpoint normalisation s = 1/D^2 (device in [B][3][N], out [B][3][N]).
 * Overwrites the context's particle state. */
pm_status pm_force(pm_ctx* ctx, const float* disp, double s, float* acc_out);

/* Vector-Jacobian product of that acceleration (App. "Custom VJP and JVP":
 * gather w.r.t. positions, gather w.r.t. the mesh, transposed multiplier,
 * scatter w.r.t. positions): xbar_out = J_A(disp)^T u, all device
 * [B][3][N].  parts: 1 = the direct term (the gather differentiated w.r.t.
 * the positions) only, 2 = the term through the mesh only, 3 = both.  Needs
 * a workspace bound with adjoint buffers (PM_ESTATE otherwise); overwrites
 * the context's particle state (positions = disp, velocities = 0). */
pm_status pm_force_vjp(pm_ctx* ctx, const float* disp, double s, const float* u, int32_t parts,
                       float* xbar_out);

/* 3D FFT of a real mesh (n = n_g): inverse == 0: real [B][n^3] -> half
 * spectrum [B][n][n][n/2+1] complex64 (unnormalised, exp(-i k x));
 * inverse != 0: half spectrum -> real, unnormalised (exp(+i k x)). */
pm_status pm_fft(pm_ctx* ctx, const void* in, void* out, int32_t inverse);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * binned power spectrum of pm_power_spectrum, computed from a given int64
 * fixed-point CIC mass mesh (device [n^3], 2^32 per particle, as pm_density's
 * fixed_out writes it) of n_particles particles in a box of side box, with
 * no context and no allocation.  Every intermediate (FFT twiddles, window
 * table, the half spectrum, partial bin sums) lives in one static device
 * array of about 11 MB per GPU, held until the process ends, which bounds the
 * mesh to n <= 128 cells per axis.  Outputs: device k_mean, pk, n_modes
 * [n_bins] as in pm_power_spectrum; asynchronous on hip_stream (NULL = the
 * default stream).  Errors: PM_EINVAL for null pointers, n not a power of
 * two >= 4, n_bins outside [1, n], n_particles < 1 or box <= 0; PM_ENOMEM for
 * n > 128 (beyond the static array); PM_EHIP for a launch failure.  Nothing
 * is launched on an error.  All calls on one GPU share its array: calls that
 * overlap on one GPU (other streams or threads) race and must be ordered by
 * the caller. */
pm_status pm_power_spectrum_mesh_noalloc(const int64_t* mesh, int32_t n, int64_t n_particles, double box,
                                         int32_t n_bins, int32_t deconvolve_cic, double* k_mean, double* pk,
                                         int64_t* n_modes, void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
