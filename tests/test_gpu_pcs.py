"""GPU parity of the PCS (piecewise cubic, order-4 B-spline) mass assignment
of tab. interpolation_kernels against the FP64 oracle, through the C ABI:
the fixed-point deposit bit for bit, the force and its VJP on identical
positions, a whole run and its gradient."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
from oracle import force as oforce
from oracle import mesh as omesh
from oracle import nbody as onbody
from oracle import philox as ophilox

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_05206_amd as P
    P.load()


def make_sim(d, adj=False, **kw):
    from paper_2510_05206_amd import PMSim
    return PMSim(synth.gpu_config(d, **kw), with_adjoint=adj)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


PCS = dict(synth.C2_SMALL, mak=4, deconvolve=True, grad_order=4)


@pytest.mark.parametrize("kind,n_p,r", [("gauss", 16, 2), ("clustered", 16, 2), ("boundary", 16, 2),
                                        ("gauss", 32, 1), ("gauss", 8, 4), ("gauss", 64, 2)])
def test_pcs_deposit_bit_exact(kind, n_p, r):
    say("pcs deposit", kind, n_p, r)
    sim = make_sim(PCS, n_p=n_p, n_g=r * n_p, box=62.5 * n_p / 32)
    psi = synth.displacements(n_p, 400 + n_p + r, 2.0, kind)
    m = sim.deposit(torch.from_numpy(psi), 4).cpu().numpy()[0]
    ref = omesh.deposit_fixedpoint(psi, n_p, r * n_p, 4)
    assert int(m.sum()) == n_p ** 3 << 32
    assert np.array_equal(m, ref)


@pytest.mark.parametrize("dec,g", [(True, 4), (False, 2), (True, 2)])
def test_pcs_force_matches_oracle(dec, g):
    d = dict(PCS, deconvolve=dec, grad_order=g)
    sim = make_sim(d)
    psi = synth.displacements(32, 41, 1.5)
    a = sim.force(torch.from_numpy(psi), 3.0).cpu().numpy()[0]
    ref = oforce.pm_force(synth.oracle_problem(d).pm, psi.astype(np.float64), 3.0)
    err = rel_l2(a, ref)
    say(f"pcs force dec {dec} FD{g}: rel L2 {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("parts", [1, 2, 3])
def test_pcs_force_vjp_matches_oracle(parts):
    sim = make_sim(PCS, adj=True)
    psi = synth.displacements(32, 42, 1.5)
    u = synth.displacements(32, 43, 1.0)
    a = sim.force_vjp(torch.from_numpy(psi), 2.0, torch.from_numpy(u), parts).cpu().numpy()[0]
    ref = oadj.force_vjp(synth.oracle_problem(PCS).pm, psi.astype(np.float64), 2.0, u.astype(np.float64), parts)
    err = rel_l2(a, ref)
    say(f"pcs force VJP parts {parts}: rel L2 {err:.2e}")
    assert err < 1e-4


def test_pcs_run_and_gradient_match_oracle():
    sim = make_sim(PCS, adj=True)
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density()
    prob = synth.oracle_problem(PCS)
    w = ophilox.white_noise(synth.SEED_W, PCS["n_p"]).astype(np.float64)
    psi, _ = onbody.run(prob, w=w)
    dref = oadj.final_density(prob, psi)
    err = rel_l2(delta.cpu().numpy()[0], dref)
    say(f"pcs run density rel L2 {err:.2e}")
    assert err < 1e-4
    dw, ds = sim.adjoint(2.0 * delta)
    gw, gs, _ = oadj.gradient(prob, w, lambda dd: 2.0 * dd)
    a = dw.cpu().numpy()[0].astype(np.float64)
    cos = a @ gw / np.linalg.norm(a) / np.linalg.norm(gw)
    say(f"pcs gradient cosine {cos:.6f} rel {rel_l2(a, gw):.2e} dsigma8 {float(ds[0]):.5e} vs {gs:.5e}")
    assert cos > 0.999 and rel_l2(a, gw) < 1e-2 and abs(float(ds[0]) / gs - 1) < 1e-2


def test_pcs_rejects_fd6_and_foreign_deposits():
    from paper_2510_05206_amd import PMError
    with pytest.raises(PMError):
        make_sim(dict(PCS, grad_order=6))
    sim = make_sim(synth.C2_SMALL)
    with pytest.raises(PMError, match="PM_EINVAL"):
        sim.deposit(torch.zeros(3, 32 ** 3), 4)
