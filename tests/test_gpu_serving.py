"""Serving on the GPU: continuous batching through the C ABI (sdm_batch),
each request's result bit-identical alone and in the mix, where "alone" is
the request's own solo GPU run and its CPU oracle run."""
import numpy as np
import pytest

from oracle import closed_form as cf
from paper_2103_17238_amd import inputs as I

from sdm_testutil import ocfg, rel_close, say

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


def test_served_mix_equals_oracle(B, orc):
    """A mix spanning the serving range of SD counts (2^10..2^16), with
    requests of every size range (1024..16384 slots: the mid-size kernel up
    to 4096, the big-cell path above under the default automatic route) and
    above 16384 slots, both kernels, under a budget that forces queueing.  Every served result equals the request's oracle run: the
    multiplicities bit for bit, volumes within 1e-12 relative (Golovin
    requests bit-exact), and the mass spectrum within 1 %."""
    from paper_2103_17238_amd.serving import GpuExecutor, Server

    reqs = I.serving_requests(16, rate_per_s=2000.0, log2_min=10, log2_max=16, n_steps=24,
                              rng_seed=17)
    # make sure each path is in the batch at least twice, with both kernels
    for r, (n, k) in zip(reqs, [(1100, 0), (5000, 1), (9000, 0), (12000, 1), (16384, 0),
                                (16385, 1), (40000, 0), (65536, 1)]):
        r.n_sd, r.kernel = n, k
    sizes = sorted(r.n_sd for r in reqs)
    assert sizes[0] >= 2 ** 10 and sizes[-1] <= 2 ** 16
    assert sum(8192 < n <= 16384 for n in sizes) >= 2 and sum(n > 16384 for n in sizes) >= 2
    ex = GpuExecutor(keep_state=True)
    fps = [ex.footprint(r, I.request_state(r)) for r in reqs]
    budget = int(2.5 * max(fps))
    say(f"serving mix vs oracle: sizes {sizes}, budget {budget} B")
    srv = Server(ex, budget_bytes=budget, steps_per_tick=5)
    stats = srv.run(reqs, I.request_state)
    ex.close()
    s = stats.summary()
    say(f"  summary {s}")
    assert s["done"] == len(reqs)
    assert s["max_resident"] < len(reqs)
    ev = cf.volume_of_radius(cf.radius_edges(1e-6, 5e-3, 48))
    exact = 0
    for r in reqs:
        o = stats.outcomes[r.rid]
        st = I.request_state(r)
        st.seed = r.seed
        cfg = ocfg(orc, st)
        for k in range(r.n_steps):
            orc.step(cfg, st.xi, st.v, st.attrs, st.cell_off, k)
        assert o.result["steps"] == r.n_steps
        assert np.array_equal(o.result["xi"], st.xi), (r.rid, r.n_sd, r.kernel)
        assert rel_close(o.result["v"], st.v, 1e-12), (r.rid, r.n_sd, r.kernel)
        if r.kernel == I.GOLOVIN:
            assert np.array_equal(o.result["v"], st.v), (r.rid, r.n_sd)
        exact += int(np.array_equal(o.result["v"], st.v))
        sg = orc.moments(cfg, o.result["xi"], o.result["v"], st.attrs, st.cell_off, ev)
        so = orc.moments(cfg, st.xi, st.v, st.attrs, st.cell_off, ev)
        l1 = np.abs(sg["spectrum"] - so["spectrum"]).sum() / so["spectrum"].sum()
        assert l1 <= 0.01, (r.rid, l1)
    say(f"  {exact} of {len(reqs)} served results bit-identical to the oracle")
