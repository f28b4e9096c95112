"""Serving: every result is the same alone (sequential, one-slot contexts)
and in the continuously batched mix, and the loop completes every request."""
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
    targets = serve.Targets()
    seq, _ = serve.serve_sequential(reqs, targets)
    bat, stats = serve.serve_batched(reqs, hbm_budget_gb=8.0, max_batch=4, targets=targets)
    assert len(bat) == len(reqs) == len(seq)
    a = {r.rid: r for r in seq}
    for r in bat:
        s = a[r.rid]
        if r.kind == "pk":
            assert np.array_equal(r.pk, s.pk), r.rid
        else:
            # dL/dw bit for bit (order-free integer sum of its bit patterns)
            assert r.dsigma8 == s.dsigma8 and r.dw_bits == s.dw_bits, r.rid
            assert abs(r.dw_norm / s.dw_norm - 1) < 1e-12, r.rid
    assert stats["mean_occupancy"] > 0
