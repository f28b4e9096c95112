"""Seeded synthetic inputs shared by the oracle and the HIP path in tests.

Holds none of the method's arithmetic: only random displacements, fields and
the parameter sets of the workloads.  The white noise of the method itself is
drawn by each side's own Philox implementation.
"""
from __future__ import annotations

import numpy as np

# Workloads (the same numbers feed oracle.force.PMConfig / oracle.nbody.Problem
# and paper_2510_05206_amd.Config)
C1 = dict(n_p=32, n_g=64, box=100.0, omega_m=1.0, spectrum="powerlaw", pl_rms_cells=0.2,
          a_start=0.02, a_end=1.0, n_steps=6, mak=2, deconvolve=False, grad_order=4, lap_order=0)
C2 = dict(n_p=256, n_g=512, box=500.0, omega_m=0.31, h=0.68, n_s=0.965, sigma8=0.81,
          spectrum="bbks", a_start=0.02, a_end=1.0, n_steps=10, mak=3, deconvolve=True,
          grad_order=4, lap_order=0)
C2_SMALL = dict(C2, n_p=32, n_g=64, box=62.5)          # C2 physics at 32^3 (same resolution)
C4 = dict(n_p=128, n_g=256, box=250.0, omega_m=0.31, h=0.68, n_s=0.965, sigma8=0.81,
          spectrum="bbks", a_start=0.02, a_end=1.0, n_steps=10, mak=2, deconvolve=False,
          grad_order=4, lap_order=0)
C4_SMALL = dict(C4, n_p=32, n_g=64, box=62.5)
SEED_W, SEED_TARGET, SEED_NOISE, SEED_DIRS = 54321, 54322, 54323, 54324


def gpu_config(d, **kw):
    from paper_2510_05206_amd import Config
    d = dict(d, **kw)
    return Config(**{k: v for k, v in d.items()})


def oracle_problem(d, **kw):
    from oracle.force import PMConfig
    from oracle.nbody import Problem
    d = dict(d, **kw)
    extra = {}
    if d.get("force") == "nufft":
        extra = dict(force="nufft", es_width=d["es_width"], es_beta=d["es_beta"])
    pm = PMConfig(d["n_p"], d["n_g"], d["box"], order=d.get("mak", 2),
                  deconvolve=d.get("deconvolve", False), grad_order=d.get("grad_order", 4),
                  lap_order=d.get("lap_order", 0), interlace=bool(d.get("antialias", 0)))
    return Problem(pm, omega_m=d.get("omega_m", 0.31), h=d.get("h", 0.68), n_s=d.get("n_s", 0.965),
                   sigma8=d.get("sigma8", 0.81), spectrum=d.get("spectrum", "bbks"),
                   rms_cells=d.get("pl_rms_cells", 0.2), a_start=d.get("a_start", 0.02),
                   a_end=d.get("a_end", 1.0), n_steps=d.get("n_steps", 6),
                   lpt_order=d.get("lpt_order", 1), stepper=d.get("stepper", "bullfrog"),
                   time_var=d.get("time_var", "D"), **extra)


def displacements(n_p, seed, scale=1.5, kind="gauss"):
    """FP32 displacements (3, N) in lattice units."""
    rng = np.random.default_rng(seed)
    N = n_p ** 3
    if kind == "gauss":
        psi = rng.normal(0.0, scale, (3, N))
    elif kind == "clustered":
        # particles pulled towards a few centres (dense cells, many per cell)
        q = np.stack(np.unravel_index(np.arange(N), (n_p,) * 3)).astype(float)
        centres = rng.uniform(0, n_p, (4, 3))
        k = rng.integers(0, 4, N)
        pull = rng.uniform(0.5, 0.98, N)
        psi = (centres[k].T - q) * pull + rng.normal(0, 0.05, (3, N))
    elif kind == "boundary":
        # on mesh nodes, faces, TSC midpoints and across the periodic seam
        choices = np.array([0.0, 0.25, 0.5, -0.25, -0.5, 0.75, 1.0, -1.0, n_p, -n_p, 0.125])
        psi = rng.choice(choices, (3, N)) + rng.choice([0.0, 2.0 ** -22, -(2.0 ** -22)], (3, N))
    else:
        raise ValueError(kind)
    return psi.astype(np.float32)


def random_mesh(n, seed):
    return np.random.default_rng(seed).normal(size=(n, n, n)).astype(np.float32)


def cotangent(n_g, seed):
    return np.random.default_rng(seed).normal(size=n_g ** 3).astype(np.float32)

# NUFFT force (ES width 6 at 2x upsampling, exact i k and -k^2)
C3 = dict(n_p=512, n_g=1024, box=1000.0, omega_m=0.31, h=0.68, n_s=0.965, sigma8=0.81,
          spectrum="bbks", a_start=0.02, a_end=1.0, n_steps=6, force="nufft", es_width=6,
          es_beta=13.8, grad_order=0, lap_order=0, mak=2, deconvolve=False)
C3_SUB = dict(C3, n_p=128, n_g=256, box=250.0)      # the 128^3 sub-problem (same resolution)
C3_SMALL = dict(C3, n_p=32, n_g=64, box=62.5)
# the PM path at the headline size: 512^3 particles on a 1024^3 mesh, TSC + deconvolution
PM_512_TSC = dict(C2, n_p=512, n_g=1024, box=1000.0, n_steps=6)
