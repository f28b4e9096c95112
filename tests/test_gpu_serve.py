"""Serving: every result is the same alone (sequential, one-slot contexts)
and in the continuously batched mix (device-indexed steps for P(k) buckets,
cohorts for gradient buckets), element by element, and the loop completes
every request."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2510_05206_amd as P
    P.load()


def test_results_identical_alone_and_in_the_mix():
    from paper_2510_05206_amd import serve
    reqs = serve.make_trace(40, rate=200.0, seed=7)
    reqs = [r for r in reqs if r.n_p <= 64][:24]
    t_mid = reqs[len(reqs) // 2].arrival
    # two 128^3 requests arriving mid-trace
    reqs += [serve.Request(1000, 128, 0.75, 5, 10 ** 6 + 1000, "grad", t_mid),
             serve.Request(1001, 128, 0.95, 6, 10 ** 6 + 1001, "pk", t_mid)]
    targets = serve.Targets()
    seq, _ = serve.serve_sequential(reqs, targets, keep_arrays=True)
    bat, stats = serve.serve_batched(reqs, hbm_budget_gb=8.0, max_batch=4, targets=targets, keep_arrays=True)
    assert len(bat) == len(reqs) == len(seq)
    a = {r.rid: r for r in seq}
    n_grad = 0
    for r in bat:
        s = a[r.rid]
        if r.kind == "pk":
            assert np.array_equal(r.pk, s.pk), r.rid
        else:
            n_grad += 1
            assert r.dsigma8 == s.dsigma8, r.rid
            assert r.dw.shape == s.dw.shape and np.array_equal(r.dw, s.dw), r.rid
    assert n_grad >= 2
    assert stats["mean_occupancy"] > 0
