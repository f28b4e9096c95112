"""GPU parity of interlaced grids (antialias 1, Sec. "Discreteness
suppression") against the FP64 oracle, through the C ABI: the force of two
deposits half a cell apart, phase-averaged spectra and averaged gathers, for
every mass assignment kernel, a whole run, the force VJP and the gradient of
a run; the device-indexed steps refuse it."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
from oracle import force as oforce
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


IL = dict(synth.C2_SMALL, antialias=1)


@pytest.mark.parametrize("mak,dec,g,kind", [(2, False, 4, "gauss"), (2, True, 2, "clustered"),
                                            (3, True, 4, "gauss"), (3, False, 6, "boundary"),
                                            (4, True, 4, "gauss"), (4, False, 2, "clustered")])
def test_interlaced_force_matches_oracle(mak, dec, g, kind):
    say("interlaced force", mak, dec, g, kind)
    d = dict(IL, mak=mak, deconvolve=dec, grad_order=g)
    sim = make_sim(d)
    psi = synth.displacements(32, 500 + mak + 10 * g, 1.5, kind)
    a = sim.force(torch.from_numpy(psi), 3.0).cpu().numpy()[0]
    ref = oforce.pm_force(synth.oracle_problem(d).pm, psi.astype(np.float64), 3.0)
    err = rel_l2(a, ref)
    say(f"  rel L2 {err:.2e}")
    assert err < 1e-5
    # the second grid changes the force (aliases of odd image order removed)
    plain = oforce.pm_force(synth.oracle_problem(dict(d, antialias=0)).pm, psi.astype(np.float64), 3.0)
    assert rel_l2(plain, ref) > 1e3 * err


@pytest.mark.parametrize("n_p,r", [(8, 2), (16, 1), (16, 4)])
def test_interlaced_force_small_and_ragged_meshes(n_p, r):
    say("interlaced force mesh", n_p, r)
    d = dict(IL, n_p=n_p, n_g=r * n_p, box=62.5 * n_p / 32, mak=3, deconvolve=True)
    sim = make_sim(d)
    psi = synth.displacements(n_p, 600 + n_p + r, 1.0)
    a = sim.force(torch.from_numpy(psi), 1.5).cpu().numpy()[0]
    ref = oforce.pm_force(synth.oracle_problem(d).pm, psi.astype(np.float64), 1.5)
    err = rel_l2(a, ref)
    say(f"  rel L2 {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("mak", [2, 3])
def test_interlaced_run_matches_oracle(mak):
    say("interlaced run", mak)
    d = dict(IL, mak=mak, deconvolve=mak == 3)
    sim = make_sim(d)
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density().cpu().numpy()[0]
    prob = synth.oracle_problem(d)
    assert prob.pm.interlace
    w = ophilox.white_noise(synth.SEED_W, d["n_p"]).astype(np.float64)
    psi, _ = onbody.run(prob, w=w)
    dref = oadj.final_density(prob, psi)
    err = rel_l2(delta, dref)
    say(f"  density rel L2 {err:.2e}")
    assert err < 1e-4


def test_interlaced_batch_slots_are_independent():
    d = dict(IL, batch=2, mak=3, deconvolve=True)
    sim = make_sim(d)
    sim.init_ics([11, 12])
    sim.run()
    both = sim.density().cpu().numpy()
    for b, seed in enumerate((11, 12)):
        one = make_sim(dict(d, batch=1))
        one.init_ics([seed])
        one.run()
        assert np.array_equal(both[b], one.density().cpu().numpy()[0])


@pytest.mark.parametrize("mak,dec,g,parts", [(2, False, 4, 3), (2, False, 4, 1), (2, False, 4, 2),
                                             (3, True, 2, 3), (4, True, 4, 3)])
def test_interlaced_force_vjp_matches_oracle(mak, dec, g, parts):
    say("interlaced force VJP", mak, dec, g, parts)
    d = dict(IL, mak=mak, deconvolve=dec, grad_order=g)
    sim = make_sim(d, adj=True)
    psi = synth.displacements(32, 700 + mak, 1.5)
    u = synth.displacements(32, 710 + mak, 1.0)
    a = sim.force_vjp(torch.from_numpy(psi), 2.0, torch.from_numpy(u), parts).cpu().numpy()[0]
    ref = oadj.force_vjp(synth.oracle_problem(d).pm, psi.astype(np.float64), 2.0, u.astype(np.float64), parts)
    err = rel_l2(a, ref)
    say(f"  rel L2 {err:.2e}")
    assert err < 1e-4


@pytest.mark.parametrize("mak", [2, 3])
def test_interlaced_gradient_matches_oracle(mak):
    say("interlaced gradient", mak)
    d = dict(IL, mak=mak, deconvolve=mak == 3)
    sim = make_sim(d, adj=True)
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density()
    dw, ds, dt = sim.adjoint(2.0 * delta, temporal=True)
    prob = synth.oracle_problem(d)
    w = ophilox.white_noise(synth.SEED_W, d["n_p"]).astype(np.float64)
    temporal = []
    gw, gs, _ = oadj.gradient(prob, w, lambda dd: 2.0 * dd, temporal=temporal)
    a = dw.cpu().numpy()[0].astype(np.float64)
    cos = a @ gw / np.linalg.norm(a) / np.linalg.norm(gw)
    say(f"  cosine {cos:.6f} rel {rel_l2(a, gw):.2e} dsigma8 {float(ds[0]):.5e} vs {gs:.5e}")
    assert cos > 0.999 and rel_l2(a, gw) < 1e-2 and abs(float(ds[0]) / gs - 1) < 1e-2
    ref = np.array(temporal)
    got = dt.cpu().numpy()[0]
    for j, name in enumerate(("tau1", "tau2", "alpha", "beta")):
        rel = np.linalg.norm(got[:, j] - ref[:, j]) / np.linalg.norm(ref[:, j])
        say(f"  {name}_bar rel L2 {rel:.2e}")
        assert rel < 5e-3


def test_interlaced_refusals():
    from paper_2510_05206_amd import PMError
    with pytest.raises(PMError, match="PM_EINVAL"):
        make_sim(dict(IL, n_p=4, n_g=8, box=10.0))
    with pytest.raises(PMError, match="PM_EINVAL"):
        make_sim(dict(synth.C3_SMALL, antialias=1))
    sim = make_sim(IL)
    sim.init_ics([synth.SEED_W])
    with pytest.raises(PMError, match="PM_EUNSUPPORTED"):
        sim.set_step_index([0])
