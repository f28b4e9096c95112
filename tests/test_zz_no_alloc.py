"""The allocation-free P(k) entry point (pm_power_spectrum_mesh_noalloc)
against pm_power_spectrum of the same particles, through the C ABI: two
calls in a row, the second on a smaller mesh, and the size limit."""
import sys

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_05206_amd as P
    P.load()


def _reference(d):
    """(mesh, k, pk, counts) of a short run: the fixed-point CIC mesh and
    pm_power_spectrum of the same final positions."""
    from paper_2510_05206_amd import PMSim
    sim = PMSim(synth.gpu_config(d))
    sim.init_ics([synth.SEED_W])
    sim.run()
    _, fixed = sim.density(fixed=True)
    k, p, c = sim.power_spectrum(d["n_g"] // 2)
    return fixed[0].contiguous(), k[0], p[0], c[0]


def test_noalloc_pk_matches_context_pk_twice():
    from paper_2510_05206_amd.sim import power_spectrum_of_mesh_noalloc
    # first call on a 128^3 mesh, then a smaller 64^3 one (the shared array
    # keeps the first call's contents)
    for d in (dict(synth.C2_SMALL, n_p=64, n_g=128, box=125.0), dict(synth.C1)):
        say("noalloc pk", d["n_p"], d["n_g"])
        mesh, k0, p0, c0 = _reference(d)
        nb = d["n_g"] // 2
        k1, p1, c1 = power_spectrum_of_mesh_noalloc(mesh, d["n_p"] ** 3, d["box"], nb)
        torch.cuda.synchronize()
        k0, p0, c0, k1, p1, c1 = (t.cpu().numpy() for t in (k0, p0, c0, k1, p1, c1))
        assert np.array_equal(c0, c1)
        ok = c0 > 0
        assert np.allclose(k1[ok], k0[ok], rtol=1e-12)
        assert np.abs(p1[ok] / p0[ok] - 1).max() < 1e-6


def test_noalloc_pk_rejects_meshes_beyond_its_scratch():
    from paper_2510_05206_amd import PMError
    from paper_2510_05206_amd.sim import power_spectrum_of_mesh_noalloc
    mesh = torch.zeros(256 ** 3, dtype=torch.int64, device="cuda")
    with pytest.raises(PMError, match="PM_ENOMEM"):
        power_spectrum_of_mesh_noalloc(mesh, 128 ** 3, 250.0, 16)
