"""GPU parity of the NUFFT force path (exponential-of-semicircle spreading,
truncated/deconvolved spectrum with the exact i k gradient, interpolation)
against the FP64 oracle."""
import sys
import time

import numpy as np
import pytest
import torch

import synth
from fdcheck import check_fd
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


@pytest.mark.parametrize("n_p,kind", [(8, "gauss"), (8, "boundary"), (16, "gauss"), (16, "clustered"),
                                        (16, "boundary"), (32, "gauss")])
def test_es_spreading_bit_exact(n_p, kind):
    say("es spreading", n_p, kind)
    sim = make_sim(synth.C3_SMALL, n_p=n_p, n_g=2 * n_p)
    psi = synth.displacements(n_p, 200 + n_p, 1.5, kind)
    m = sim.deposit(torch.from_numpy(psi), 6).cpu().numpy()[0]
    ref = onufft.deposit_fixedpoint_es(psi, n_p, 2 * n_p)
    assert np.array_equal(m, ref)


@pytest.mark.parametrize("n_p", [8, 16, 32, 64])
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


# the FP64 oracle takes minutes over the 128^3 run
@pytest.mark.parametrize("wl", ["C3_SMALL", pytest.param("C3_SUB", marks=pytest.mark.timeout(900))])
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
    psi, _ = onbody.run(prob, w=ophilox.white_noise(synth.SEED_W, d["n_p"]), progress=say)
    dref = oadj.final_density(prob, psi)
    kr, pr, cr = opk.power_spectrum(dref, d["box"], d["n_g"] // 2)
    err = rel_l2(delta, dref)
    sel = kr < np.pi * d["n_p"] / d["box"] / 2
    perr = np.abs(p[sel] / pr[sel] - 1).max()
    say(f"{wl}: density rel L2 {err:.3e}, P(k<kNyq/2) max rel {perr:.3e} (oracle {time.time() - t0:.0f} s)")
    assert err < 1e-4 and perr < 1e-5


def _adj_sim(d):
    from paper_2510_05206_amd import PMSim
    return PMSim(synth.gpu_config(d), with_adjoint=True)


def test_nufft_gradient_matches_oracle_store_all():
    """Reverse-in-time adjoint of the NUFFT force run against the oracle's
    store-all reverse mode (L2 loss on the final CIC density)."""
    d = synth.C3_SMALL
    say("nufft adjoint vs oracle", d["n_p"])
    prob = synth.oracle_problem(d)
    psi_t, _ = onbody.run(prob, w=ophilox.white_noise(synth.SEED_TARGET, d["n_p"]))
    dt = oadj.final_density(prob, psi_t)
    dobs = dt + 0.1 * dt.std() * np.random.default_rng(synth.SEED_NOISE).normal(size=dt.size)
    sim = _adj_sim(d)
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density()
    g = 2.0 * (delta.double() - torch.from_numpy(dobs).to(delta.device)).float()
    dw, ds = sim.adjoint(g)
    w = ophilox.white_noise(synth.SEED_W, d["n_p"]).astype(np.float64)
    gw, gs, _ = oadj.gradient(prob, w, lambda dd: 2.0 * (dd - dobs))
    gw = gw.reshape(-1)
    a = dw.cpu().numpy()[0].astype(np.float64)
    cos = a @ gw / np.linalg.norm(a) / np.linalg.norm(gw)
    rel = np.linalg.norm(a - gw) / np.linalg.norm(gw)
    srel = abs(float(ds[0]) / gs - 1)
    say(f"nufft: cosine {cos:.6f} rel L2 {rel:.3e} dsigma8 {float(ds[0]):.6e} vs {gs:.6e}")
    assert cos > 0.999 and rel < 1e-2 and srel < 1e-2


def test_nufft_adjoint_returns_to_initial_state():
    d = synth.C3_SMALL
    sim = _adj_sim(d)
    sim.init_ics([synth.SEED_W])
    x0, v0 = (t.clone() for t in sim.get_state())
    sim.run()
    sim.adjoint(torch.zeros(1, d["n_g"] ** 3, device="cuda"))
    x1, v1 = sim.get_state()
    ex = float((x1 - x0).norm() / x0.norm())
    ev = float((v1 - v0).norm() / v0.norm())
    say(f"nufft reverse integration: X rel {ex:.2e}, V rel {ev:.2e}")
    assert ex < 1e-3 and ev < 1e-3


def test_nufft_gradient_matches_finite_differences():
    """64^3 particles on the 128^3 fine grid (the C3 resolution, L = 125),
    central differences of the GPU forward along random unit directions."""
    d = dict(synth.C3, n_p=64, n_g=128, box=125.0)
    say("nufft adjoint vs FD at", d["n_p"])
    sim = _adj_sim(d)
    w = sim.init_ics([synth.SEED_W], return_w=True)
    tgt = make_sim(d)
    tgt.init_ics([synth.SEED_TARGET])
    tgt.run()
    dt = tgt.density()
    gen = torch.Generator(device="cpu").manual_seed(synth.SEED_NOISE)
    dobs = dt + 0.1 * dt.std() * torch.randn(dt.shape, generator=gen).to(dt.device)
    del tgt

    def loss(wv):
        sim.init_ics(w=wv)
        sim.run()
        return float(((sim.density().double() - dobs.double()) ** 2).sum())

    sim.init_ics(w=w)
    sim.run()
    dw, _ = sim.adjoint(2.0 * (sim.density() - dobs))
    gen = torch.Generator(device="cpu").manual_seed(synth.SEED_DIRS)
    preds, fdv, spread = [], [], []
    for k in range(16):
        v = torch.randn(w.shape, generator=gen).to(w.device)
        v /= v.norm()
        pred = float((dw.double() * v.double()).sum())
        fds = [(loss(w + eps * v) - loss(w - eps * v)) / (2 * eps) for eps in (0.05, 0.1, 0.2)]
        fd = float(np.median(fds))
        preds.append(pred)
        fdv.append(fd)
        spread.append(float(np.max(np.abs(np.array(fds) - fd))))
        say(f"dir {k}: adjoint {pred:.6e} fd {fd:.6e} ({fds}) rel {abs(pred - fd) / abs(fd):.2e}")
    check_fd(preds, fdv, spread)


def test_es_spreading_full_size_sampled_cells():
    """The 512^3 / 1024^3 launch of the headline workload: 64 sampled cells of
    the fixed-point ES spreading against the oracle, which evaluates only the
    particles whose 6^3 stencil can reach them; total mass and determinism."""
    d = synth.C3
    n_p, n_f = d["n_p"], d["n_g"]
    say("ES spreading full size", n_p, n_f)
    sim = make_sim(d)
    psi = synth.displacements(n_p, 31, 1.5)
    m = sim.deposit(torch.from_numpy(psi), 6)
    rng = np.random.default_rng(1)
    cells = np.unique(rng.integers(0, n_f ** 3, 64))
    got = m[0, torch.from_numpy(cells).to(m.device)].cpu().numpy()
    # fixed-point coordinates of every particle, in chunks; keep the ones
    # whose home node lies within the stencil reach of a sampled cell
    cx, cy, cz = cells // (n_f * n_f), (cells // n_f) % n_f, cells % n_f
    # home nodes h whose stencil h-2 .. h+3 reaches a sampled cell
    o = np.arange(-3, 3)
    reach = np.unique((((cx[:, None, None, None] + o[None, :, None, None]) % n_f * n_f
                        + (cy[:, None, None, None] + o[None, None, :, None]) % n_f) * n_f
                       + (cz[:, None, None, None] + o[None, None, None, :]) % n_f).ravel())
    acc = {int(c): 0 for c in cells}
    chunk = 1 << 22
    N = n_p ** 3
    for s in range(0, N, chunk):
        idx = np.arange(s, min(s + chunk, N))
        lat = np.stack([idx // (n_p * n_p), (idx // n_p) % n_p, idx % n_p])
        r = n_f // n_p
        frac = np.rint(psi[:, idx].astype(np.float64) * (r * 2.0 ** 20)).astype(np.int64)
        U = np.mod(lat * (r << 20) + frac, n_f << 20)
        h = U >> 20
        near = np.isin((h[0] * n_f + h[1]) * n_f + h[2], reach)
        if not near.any():
            continue
        for lin, w3 in onufft.es_fixed_stencil(U[:, near], n_f):
            for c, wv in zip(lin, w3):
                if int(c) in acc:
                    acc[int(c)] += int(wv)
    ref = np.array([acc[int(c)] for c in cells])
    assert np.array_equal(got, ref)
    # total mass: every particle's ES weights summed in the fixed-point spec
    # is not N 2^32 (the kernel is not a partition of unity), so compare two
    # launches bit for bit instead
    m2 = sim.deposit(torch.from_numpy(psi), 6)
    assert torch.equal(m, m2)


def test_nufft_force_full_size_conserves_momentum():
    """512^3 particles on the 1024^3 fine grid: the net NUFFT force vanishes
    (the multiplier is odd and spreading/interpolation share one kernel)."""
    d = synth.C3
    sim = make_sim(d)
    psi = synth.displacements(d["n_p"], 32, 1.5)
    a = sim.force(torch.from_numpy(psi), 1.0)[0].double()
    net = a.sum(dim=1).abs().max().item()
    scale = a.abs().sum(dim=1).max().item()
    say(f"full-size NUFFT net force {net:.3e} of {scale:.3e}")
    assert net < 1e-6 * scale and torch.isfinite(a).all()
