"""Oracle parity at the full sizes of the bench workloads, and the adjoint
against the oracle's store-all gradient at 64^3.

A displacement field that repeats a 64^3 (or 32^3) lattice tile R times per
axis has a density that repeats with period L/R, so only the modes that are
multiples of R are nonzero.  Those are the modes of the tile's own problem
(box L/R, the same cell size), the multipliers take the same values there
(same theta = 2 pi m / n per cell), and the NUFFT truncation |m| < n_p/2 keeps
exactly the tile's kept modes.  Each particle of the full-size launch must
then see the force (and, run from the replicated initial state, follow the
trajectory) of its counterpart in the tile, which the FP64 oracle computes at
the tile's size.  This reaches the 1024-point pruned row and column passes
of the headline workload and the 512/1024-point passes of the PM workloads.
"""
import sys
import time

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
from oracle import mesh as omesh
from oracle import nbody as onbody
from oracle import nufft as onufft
from oracle import philox as ophilox
from oracle.force import pm_force

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_05206_amd as P
    P.load()


def make_sim(d, adj=False):
    from paper_2510_05206_amd import PMSim
    return PMSim(synth.gpu_config(d), with_adjoint=adj)


def tile_of(d, n_tile):
    """The tile's own problem: n_tile^3 particles at the same resolution."""
    R = d["n_p"] // n_tile
    return dict(d, n_p=n_tile, n_g=d["n_g"] // R, box=d["box"] / R), R


def replicate(x, n_tile, R):
    """(3, n_tile^3) lattice-ordered particle array -> (1, 3, (R n_tile)^3) on
    the GPU, tile repeated R times per axis."""
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda().view(3, 1, n_tile, 1, n_tile, 1, n_tile)
    return t.expand(3, R, n_tile, R, n_tile, R, n_tile).reshape(1, 3, -1).contiguous()


def replica_rel_l2(a, ref, n_tile, R):
    """rel L2 of a full-size particle array against the replicated tile
    reference, over every particle (FP64 sums per component)."""
    ref = torch.from_numpy(np.asarray(ref, dtype=np.float64)).cuda().view(3, 1, n_tile, 1, n_tile, 1, n_tile)
    num = den = 0.0
    for c in range(3):
        ac = a[0, c].view(R, n_tile, R, n_tile, R, n_tile).double()
        num += float(((ac - ref[c]) ** 2).sum())
        den += float((ref[c] ** 2).sum()) * R ** 3
    return (num / den) ** 0.5


@pytest.mark.parametrize("wl,n_tile", [("C3", 64), ("C2", 32), ("PM_512_TSC", 64)])
def test_full_size_force_equals_tile_oracle(wl, n_tile):
    d = synth.PM_512_TSC if wl == "PM_512_TSC" else getattr(synth, wl)
    td, R = tile_of(d, n_tile)
    say(f"full-size force {wl}: {d['n_p']}^3 on {d['n_g']}^3 from a {n_tile}^3 tile x {R}^3")
    psi = synth.displacements(n_tile, 40 + n_tile, 1.5)
    t0 = time.time()
    if d.get("force") == "nufft":
        ref = onufft.nufft_force(n_tile, td["n_g"], psi.astype(np.float64), 2.0, d["es_width"], d["es_beta"])
    else:
        ref = pm_force(synth.oracle_problem(td).pm, psi.astype(np.float64), 2.0)
    sim = make_sim(d)
    a = sim.force(replicate(psi, n_tile, R), 2.0)
    err = replica_rel_l2(a, ref, n_tile, R)
    say(f"{wl}: every particle against the tile oracle, rel L2 {err:.3e} (oracle {time.time() - t0:.0f} s)")
    assert err < 2e-5 if d.get("force") == "nufft" else err < 1e-5


@pytest.fixture(scope="module")
def nufft64():
    """The oracle's 64^3 NUFFT problem at the C3 resolution (L = 125): initial
    state, store-all gradient of an L2 loss and the final density."""
    d = dict(synth.C3, n_p=64, n_g=128, box=125.0)
    prob = synth.oracle_problem(d)
    w = ophilox.white_noise(synth.SEED_W, 64).astype(np.float64)
    psi0, vel0, _ = onbody.initial_state(prob, w)
    t0 = time.time()
    # the observed field: a seeded Gaussian field at half the rms of the final density
    dobs = {}

    def cot(dd):
        dobs["v"] = 0.5 * dd.std() * np.random.default_rng(synth.SEED_NOISE).normal(size=dd.size)
        return 2.0 * (dd - dobs["v"])

    gw, gs, delta = oadj.gradient(prob, w, cot, progress=say)
    say(f"oracle 64^3 NUFFT gradient {time.time() - t0:.0f} s")
    return dict(d=d, psi0=psi0, vel0=vel0, gw=gw.reshape(-1), gs=gs, delta=delta, dobs=dobs["v"])


def test_full_size_nufft_run_equals_tile_oracle(nufft64):
    """The headline workload's whole run (512^3 particles, 1024^3 fine grid,
    6 steps) from the 64^3 tile's initial state replicated 8^3 times: the
    final density is the tile's oracle density repeated."""
    d = synth.C3
    R = 8
    sim = make_sim(d)
    sim.set_state(replicate(nufft64["psi0"], 64, R), replicate(nufft64["vel0"], 64, R))
    sim.run()
    delta = sim.density()[0].view(R, 128, R, 128, R, 128).double()
    ref = torch.from_numpy(nufft64["delta"]).cuda().view(1, 128, 1, 128, 1, 128)
    err = (float(((delta - ref) ** 2).sum()) / (float((ref ** 2).sum()) * R ** 3)) ** 0.5
    say(f"full-size NUFFT run from the replicated 64^3 state: density rel L2 {err:.3e}")
    assert err < 1e-4


def test_nufft_gradient_matches_oracle_store_all_64(nufft64):
    """Reverse-in-time adjoint against the oracle's store-all gradient at 64^3
    (128^3 fine grid, C3 resolution)."""
    d = nufft64["d"]
    sim = make_sim(d, adj=True)
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density()
    g = 2.0 * (delta.double() - torch.from_numpy(nufft64["dobs"]).cuda()).float()
    dw, ds = sim.adjoint(g)
    a = dw.cpu().numpy()[0].astype(np.float64)
    gw, gs = nufft64["gw"], nufft64["gs"]
    cos = a @ gw / np.linalg.norm(a) / np.linalg.norm(gw)
    rel = np.linalg.norm(a - gw) / np.linalg.norm(gw)
    srel = abs(float(ds[0]) / gs - 1)
    say(f"nufft 64^3: cosine {cos:.6f} rel L2 {rel:.3e} dsigma8 {float(ds[0]):.6e} vs {gs:.6e}")
    assert cos > 0.999 and rel < 1e-2 and srel < 1e-2


def test_gradient_matches_oracle_store_all_c4_resolution():
    """The differentiation workload's physics at 64^3 particles on a 128^3
    mesh (L = 125, the C4 resolution), 10 steps, against the store-all oracle."""
    d = dict(synth.C4, n_p=64, n_g=128, box=125.0)
    prob = synth.oracle_problem(d)
    w = ophilox.white_noise(synth.SEED_W, 64).astype(np.float64)
    dobs = {}

    def cot(dd):
        dobs["v"] = 0.5 * dd.std() * np.random.default_rng(synth.SEED_NOISE).normal(size=dd.size)
        return 2.0 * (dd - dobs["v"])

    t0 = time.time()
    gw, gs, _ = oadj.gradient(prob, w, cot, progress=say)
    say(f"oracle 64^3 C4 gradient {time.time() - t0:.0f} s")
    sim = make_sim(d, adj=True)
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density()
    g = 2.0 * (delta.double() - torch.from_numpy(dobs["v"]).cuda()).float()
    dw, ds = sim.adjoint(g)
    a = dw.cpu().numpy()[0].astype(np.float64)
    gw = gw.reshape(-1)
    cos = a @ gw / np.linalg.norm(a) / np.linalg.norm(gw)
    rel = np.linalg.norm(a - gw) / np.linalg.norm(gw)
    srel = abs(float(ds[0]) / gs - 1)
    say(f"C4 64^3: cosine {cos:.6f} rel L2 {rel:.3e} dsigma8 {float(ds[0]):.6e} vs {gs:.6e}")
    assert cos > 0.999 and rel < 1e-2 and srel < 1e-2
