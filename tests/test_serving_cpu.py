"""The serving scheduler on the CPU, with the oracle standing in for the device
(the idea of a CPU stand-in for the GPU backend that the PySDM v1 paper
describes for testing, "Dependencies and supported platforms").  A virtual
clock makes admission and latency bookkeeping deterministic."""
import numpy as np
import pytest

from paper_2103_17238_amd import inputs as I
from paper_2103_17238_amd.serving import Server


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class OracleExecutor:
    """Runs every simulation on the CPU oracle; a step costs 1 ms of virtual time."""

    def __init__(self, orc, clock, per_step_s=1e-3):
        self.orc = orc
        self.clock = clock
        self.per_step_s = per_step_s
        self.admitted = []
        self.released = 0
        self.batches = 0

    def footprint(self, req, state):
        return state.n_slots * (16 + 8 * state.n_attr) + 4096

    def admit(self, req, state):
        st = state.copy()
        st.seed = req.seed
        cfg = self.orc.OracleConfig(n_slots=st.n_slots, n_cells=st.n_cells, n_attr=st.n_attr,
                                    dt=st.dt, dv=st.dv, b=st.b, kernel=st.kernel,
                                    adaptive=st.adaptive, seed=st.seed)
        h = {"req": req, "st": st, "cfg": cfg, "step": 0, "sd_steps": 0}
        self.admitted.append(req.rid)
        return h

    def batch(self, handles):
        self.batches += 1
        return list(handles)

    def step(self, batch, k):
        for h in batch:
            for _ in range(k):
                if h["step"] >= h["req"].n_steps:
                    break
                st = h["st"]
                out = self.orc.step(h["cfg"], st.xi, st.v, st.attrs, st.cell_off, h["step"])
                h["sd_steps"] += int(out["tallies"][0])
                h["step"] += 1
        self.clock.t += k * self.per_step_s

    def step_of(self, h):
        return h["step"]

    def sync(self):
        pass

    def collect(self, handles):
        out = []
        for h in handles:
            st = h["st"]
            m = self.orc.moments(h["cfg"], st.xi, st.v, st.attrs, st.cell_off)
            out.append({"m0": m["m0"], "xi": st.xi.copy(), "v": st.v.copy(),
                        "sd_steps": h["sd_steps"], "steps": h["step"]})
        return out

    def release(self, h):
        self.released += 1


def small_requests(n=24, seed=3):
    reqs = I.serving_requests(n, rate_per_s=400.0, log2_min=5, log2_max=9, n_steps=30,
                              rng_seed=seed)
    return reqs


def alone(orc, req):
    st = I.request_state(req)
    st.seed = req.seed
    cfg = orc.OracleConfig(n_slots=st.n_slots, n_cells=st.n_cells, dt=st.dt, dv=st.dv, b=st.b,
                           kernel=st.kernel, seed=st.seed)
    for s in range(req.n_steps):
        orc.step(cfg, st.xi, st.v, st.attrs, st.cell_off, s)
    return st


def test_all_served_and_each_equals_its_solo_run(orc):
    clock = Clock()
    ex = OracleExecutor(orc, clock)
    reqs = small_requests()
    srv = Server(ex, budget_bytes=10 ** 9, steps_per_tick=7, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs, I.request_state)
    s = stats.summary()
    assert s["done"] == len(reqs) and s["failed"] == s["rejected"] == 0
    assert ex.released == len(reqs)
    for r in reqs:
        o = stats.outcomes[r.rid]
        assert o.result["steps"] == r.n_steps
        ref = alone(orc, r)
        assert np.array_equal(o.result["xi"], ref.xi) and np.array_equal(o.result["v"], ref.v)
        assert o.latency_s >= 0 and o.admit_s >= r.arrival_s
    assert s["p50_s"] <= s["p99_s"]
    assert s["max_resident"] > 1  # requests overlapped on the "device"


def test_budget_back_pressure_and_fifo(orc):
    clock = Clock()
    ex = OracleExecutor(orc, clock)
    reqs = small_requests(16)
    fps = [ex.footprint(r, I.request_state(r)) for r in reqs]
    budget = int(max(fps) * 1.5)  # at most one large (or two small) requests at once
    resident_bytes = []
    srv = Server(ex, budget_bytes=budget, steps_per_tick=5, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs, I.request_state, on_tick=lambda st, res, used: resident_bytes.append(used))
    assert stats.summary()["done"] == len(reqs)
    assert max(resident_bytes) <= budget
    # FIFO: admission order is arrival order
    assert ex.admitted == [r.rid for r in sorted(reqs, key=lambda r: (r.arrival_s, r.rid))]
    waited = [stats.outcomes[r.rid].admit_s - r.arrival_s for r in reqs]
    assert max(waited) > 0


def test_too_large_rejected_others_served(orc):
    clock = Clock()
    ex = OracleExecutor(orc, clock)
    reqs = small_requests(10)
    big = max(reqs, key=lambda r: r.n_sd)
    budget = ex.footprint(big, I.request_state(big)) - 1
    srv = Server(ex, budget_bytes=budget, steps_per_tick=10, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs, I.request_state)
    assert stats.outcomes[big.rid].status == "rejected"
    assert "exceeds budget" in stats.outcomes[big.rid].error
    assert all(stats.outcomes[r.rid].status == "done" for r in reqs if r.n_sd < big.n_sd)


def test_failure_isolated(orc):
    clock = Clock()
    ex = OracleExecutor(orc, clock)
    reqs = small_requests(8)
    bad = reqs[3].rid

    def state_of(req):
        if req.rid == bad:
            raise ValueError("corrupt initial state")
        return I.request_state(req)

    srv = Server(ex, budget_bytes=10 ** 9, steps_per_tick=10, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs, state_of)
    assert stats.outcomes[bad].status == "failed" and "corrupt" in stats.outcomes[bad].error
    assert stats.summary()["done"] == len(reqs) - 1


def test_cancellation(orc):
    clock = Clock()
    ex = OracleExecutor(orc, clock)
    reqs = small_requests(12)
    srv = Server(ex, budget_bytes=10 ** 9, max_resident=2, steps_per_tick=3, clock=clock,
                 sleep=clock.sleep)
    first, last = reqs[0].rid, reqs[-1].rid
    calls = {"n": 0}

    def on_tick(st, resident, used):
        calls["n"] += 1
        if calls["n"] == 2:
            srv.cancel(first)  # resident by now
            srv.cancel(last)  # still queued
    stats = srv.run(reqs, I.request_state, on_tick=on_tick)
    assert stats.outcomes[first].status == "cancelled"
    assert stats.outcomes[last].status == "cancelled"
    assert stats.summary()["done"] == len(reqs) - 2
    assert stats.summary()["max_resident"] <= 2


def test_latency_accounting_virtual_clock(orc):
    clock = Clock()
    ex = OracleExecutor(orc, clock, per_step_s=0.0)
    req = small_requests(1)[0]
    srv = Server(ex, budget_bytes=10 ** 9, steps_per_tick=req.n_steps, clock=clock,
                 sleep=clock.sleep)
    stats = srv.run([req], I.request_state)
    o = stats.outcomes[req.rid]
    assert o.status == "done" and o.latency_s == pytest.approx(0.0, abs=0.011)


class PreparingExecutor(OracleExecutor):
    """Also builds the next tick's batch while a tick "runs" (prepare/adopt)."""

    def __init__(self, orc, clock):
        super().__init__(orc, clock)
        self.prepared = 0
        self.adopted = 0
        self.current = None
        self.pending = None

    def batch(self, handles):
        self.current, self.pending = list(handles), None
        self.batches += 1
        return self.current

    def prepare(self, handles):
        self.prepared += 1
        self.pending = list(handles)
        return self.pending

    def adopt(self, b):
        assert b is self.pending  # only the batch prepared last is adopted
        self.adopted += 1
        self.current, self.pending = b, None
        return b


def test_prepared_batches_are_adopted_and_results_unchanged(orc):
    """When the next tick's membership is known while a tick runs (finishers
    out, admissions in), the server has the executor build that batch then,
    and uses it if nothing changed meanwhile; results equal the solo runs."""
    clock = Clock()
    ex = PreparingExecutor(orc, clock)
    reqs = small_requests(20, seed=5)
    srv = Server(ex, budget_bytes=10 ** 9, steps_per_tick=4, clock=clock, sleep=clock.sleep)
    stats = srv.run(reqs, I.request_state)
    assert stats.summary()["done"] == len(reqs)
    assert ex.prepared > 0 and ex.adopted > 0
    assert ex.adopted <= ex.prepared
    for r in reqs:
        ref = alone(orc, r)
        o = stats.outcomes[r.rid]
        assert np.array_equal(o.result["xi"], ref.xi) and np.array_equal(o.result["v"], ref.v)
