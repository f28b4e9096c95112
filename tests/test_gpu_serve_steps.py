"""Device-indexed steps (pm_set_step_index / pm_step_device), the serving
path of continuous batching: slots admitted at different times and running
different step counts through one replayed graph end bit-identical to the
same requests run alone with pm_run."""
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


def test_device_steps_equal_runs_alone():
    from paper_2510_05206_amd import PMSim
    d = dict(synth.C2_SMALL, n_steps=12, mak=2, deconvolve=False)
    reqs = [(101, 0.7, 4, 0), (102, 0.9, 7, 2), (103, 0.81, 6, 5), (104, 0.65, 5, 5)]  # seed, sigma8, steps, join
    B = 3
    sim = PMSim(synth.gpu_config(d, batch=B))
    slot_of, free, k_host = {}, list(range(B)), [-1] * B
    steps = [12] * B
    sig = [0.81] * B
    pending, done, t = list(reqs), {}, 0
    final = {}
    while pending or any(k >= 0 for k in k_host):
        # admit the requests whose join time has come, into free slots
        for r in [r for r in pending if r[3] <= t and free]:
            if not free:
                break
            b = free.pop(0)
            pending.remove(r)
            slot_of[r[0]] = b
            steps[b], sig[b] = r[2], r[1]
            sim.set_slot_params(n_steps=steps, sigma8=sig)
            sim.set_active([b])
            sim.init_ics([r[0] if i == b else 0 for i in range(B)])
            sim.set_active(None)
            sim.set_step_index([0 if i == b else -2 for i in range(B)])
            k_host[b] = 0
        if any(k >= 0 for k in k_host):
            sim.step_device()
            for b in range(B):
                if k_host[b] >= 0:
                    k_host[b] = k_host[b] + 1 if k_host[b] + 1 < steps[b] else -1
                    if k_host[b] == -1:
                        x, v = sim.get_state()
                        seed = [s for s, bb in slot_of.items() if bb == b and s not in final][0]
                        final[seed] = (x[b].cpu().numpy().copy(), v[b].cpu().numpy().copy())
                        free.append(b)
        assert sim.get_step_index() == k_host
        t += 1
    assert len(final) == len(reqs)
    for seed, s8, n, _ in reqs:
        one = PMSim(synth.gpu_config(d, batch=1))
        one.set_slot_params(n_steps=[n], sigma8=[s8])
        one.init_ics([seed])
        one.run()
        x, v = (a.cpu().numpy()[0] for a in one.get_state())
        say(f"seed {seed}: max |dx| {np.abs(x - final[seed][0]).max():.3e}")
        assert np.array_equal(x, final[seed][0]) and np.array_equal(v, final[seed][1])


def test_device_steps_reject_nufft_and_bad_indices():
    from paper_2510_05206_amd import PMError, PMSim
    sim = PMSim(synth.gpu_config(synth.C3_SMALL))
    with pytest.raises(PMError, match="PM_EUNSUPPORTED"):
        sim.set_step_index([0])
    sim = PMSim(synth.gpu_config(dict(synth.C2_SMALL, n_steps=4)))
    with pytest.raises(PMError, match="PM_EINVAL"):
        sim.set_step_index([4])
