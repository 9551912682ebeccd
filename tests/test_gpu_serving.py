"""Serving on the GPU: continuous batching through the C ABI (sdm_batch),
each request's result bit-identical alone and in the mix."""
import numpy as np
import pytest

from paper_2103_17238_amd import inputs as I

from sdm_testutil import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_17238_amd import binding

    return binding


def _alone(B, req):
    st = I.request_state(req)
    st.seed = req.seed
    sim = B.Sim(st)
    sim.step(req.n_steps)
    xi, v, _ = sim.state()
    sim.close()
    return xi, v


@pytest.mark.parametrize("tight,k", [(False, 7), (True, 5)])
def test_served_alone_equals_in_mix(B, tight, k):
    from paper_2103_17238_amd.serving import GpuExecutor, Server

    reqs = I.serving_requests(40, rate_per_s=4000.0, log2_min=7, log2_max=13, n_steps=33,
                              rng_seed=11)
    ex = GpuExecutor(keep_state=True)
    fps = [ex.footprint(r, I.request_state(r)) for r in reqs]
    # tight: room for about two of the largest requests, so admission queues
    budget = int(2.2 * max(fps)) if tight else 4 * 2 ** 30
    say(f"serving 40 requests budget={budget} B k={k}")
    srv = Server(ex, budget_bytes=budget, steps_per_tick=k)
    stats = srv.run(reqs, I.request_state)
    ex.close()
    s = stats.summary()
    say(f"  summary {s}")
    assert s["done"] == len(reqs)
    if tight:
        assert s["max_resident"] < len(reqs)
    for r in reqs:
        o = stats.outcomes[r.rid]
        assert o.result["steps"] == r.n_steps
        xi, v = _alone(B, r)
        assert np.array_equal(o.result["xi"], xi), r.rid
        assert np.array_equal(o.result["v"], v), r.rid
