"""FP64 CPU oracle for the differentiable particle-mesh (PM) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the serving loop) may import, call or link anything here; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code, table or constant generator with the
HIP path: every formula is re-derived from the paper (DISCO-DJ II,
arXiv:2510.05206) and written out plainly in numpy/scipy FP64.

Modules
-------
cosmo    growth ODEs (App. "Exact vs approximate growth", eq. growth_odes),
         BBKS / power-law spectra, sigma8, BullFrog coefficients (Sec. "Time
         stepping").
philox   Philox-4x32-10 counter RNG (Salmon et al. 2011) + Box-Muller white
         noise.  The paper's N-GenIC generator is not reproduced.
ics      Zel'dovich initial conditions (Sec. "Lagrangian perturbation theory").
mesh     CIC/TSC mass assignment (tab. interpolation_kernels): float FP64
         deposit / gather / gradient-gather, and the integer fixed-point
         deposit whose bits the GPU must reproduce.
force    PM force (Sec. "Force evaluation"): Fourier multipliers of
         tab. derivative_kernels, window deconvolution, Poisson solve.
nufft    exponential-of-semicircle NUFFT force and the direct NUDFT
         (eq. NUDFTII).
nbody    BullFrog drift-kick-drift run (eq. dkd).
pk       binned power spectrum.
adjoint  store-all reverse mode through the run (tab. adjoint_dkd, App.
         "Custom VJP and JVP") and the IC adjoint.

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
closed form, an invariant, a brute-force sum or a value the paper prints,
except where a docstring says "parity unpinned".
"""
