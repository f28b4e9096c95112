"""GPU runs with the other steppers and step spacings of Sec. "Time
stepping" (FastPM, steps uniform in a or ln a) against the FP64 oracle,
through the C ABI.  Only the host tables differ from the BullFrog runs; the
runs check that they reach the kernels."""
import sys

import numpy as np
import pytest
import torch

import synth
from oracle import adjoint as oadj
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


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("stepper,tv", [("fastpm", "D"), ("bullfrog", "a"), ("fastpm", "lna")])
def test_run_with_stepper_and_time_variable(stepper, tv):
    from paper_2510_05206_amd import PMSim
    d = dict(synth.C2_SMALL, stepper=stepper, time_var=tv)
    say("run", stepper, tv)
    sim = PMSim(synth.gpu_config(d))
    sim.init_ics([synth.SEED_W])
    sim.run()
    delta = sim.density().cpu().numpy()[0]
    prob = synth.oracle_problem(d)
    psi, _ = onbody.run(prob, w=ophilox.white_noise(synth.SEED_W, d["n_p"]))
    err = rel_l2(delta, oadj.final_density(prob, psi))
    say(f"{stepper}/{tv}: density rel L2 {err:.2e}")
    assert err < 1e-4
