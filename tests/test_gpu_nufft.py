"""GPU parity of the NUFFT force path (exponential-of-semicircle spreading,
truncated/deconvolved spectrum with the exact i k gradient, interpolation)
against the FP64 oracle."""
import sys
import time

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
from oracle import nbody as onbody
from oracle import nufft as onufft
from oracle import philox as ophilox
from oracle import pk as opk

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_05206_amd as P
    P.load()


def make_sim(d, **kw):
    from paper_2510_05206_amd import PMSim
    return PMSim(synth.gpu_config(d, **kw), with_adjoint=False)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n_p,kind", [(16, "gauss"), (16, "clustered"), (16, "boundary"), (32, "gauss")])
def test_es_spreading_bit_exact(n_p, kind):
    say("es spreading", n_p, kind)
    sim = make_sim(synth.C3_SMALL, n_p=n_p, n_g=2 * n_p)
    psi = synth.displacements(n_p, 200 + n_p, 1.5, kind)
    m = sim.deposit(torch.from_numpy(psi), 6).cpu().numpy()[0]
    ref = onufft.deposit_fixedpoint_es(psi, n_p, 2 * n_p)
    assert np.array_equal(m, ref)


@pytest.mark.parametrize("n_p", [16, 32])
def test_nufft_force_matches_oracle(n_p):
    say("nufft force", n_p)
    sim = make_sim(synth.C3_SMALL, n_p=n_p, n_g=2 * n_p)
    psi = synth.displacements(n_p, 300 + n_p, 1.0)
    a = sim.force(torch.from_numpy(psi), 2.0).cpu().numpy()[0]
    ref = onufft.nufft_force(n_p, 2 * n_p, psi.astype(np.float64), 2.0, 6, 13.8)
    err = rel_l2(a, ref)
    say(f"nufft force rel L2 {err:.3e}")
    assert err < 2e-5


def test_nufft_force_against_direct_nudft():
    n_p = 8
    sim = make_sim(synth.C3_SMALL, n_p=n_p, n_g=16)
    psi = synth.displacements(n_p, 5, 0.7)
    a = sim.force(torch.from_numpy(psi), 1.0).cpu().numpy()[0]
    ref = onufft.nudft_force_direct(n_p, 16, psi.astype(np.float64), 1.0)
    assert rel_l2(a, ref) < 3e-5


@pytest.mark.parametrize("wl", ["C3_SMALL", pytest.param("C3_SUB", marks=pytest.mark.slow)])
def test_nufft_run_matches_oracle(wl):
    d = getattr(synth, wl)
    say("nufft run", wl)
    sim = make_sim(d)
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density().cpu().numpy()[0]
    k, p, cnt = (t.cpu().numpy()[0] for t in sim.power_spectrum(d["n_g"] // 2))
    t0 = time.time()
    prob = synth.oracle_problem(d)
    psi, _ = onbody.run(prob, w=ophilox.white_noise(synth.SEED_W, d["n_p"]))
    dref = oadj.final_density(prob, psi)
    kr, pr, cr = opk.power_spectrum(dref, d["box"], d["n_g"] // 2)
    err = rel_l2(delta, dref)
    sel = kr < np.pi * d["n_p"] / d["box"] / 2
    perr = np.abs(p[sel] / pr[sel] - 1).max()
    say(f"{wl}: density rel L2 {err:.3e}, P(k<kNyq/2) max rel {perr:.3e} (oracle {time.time() - t0:.0f} s)")
    assert err < 1e-4 and perr < 1e-5
