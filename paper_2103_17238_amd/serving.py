"""Continuous batching of SDM box simulations.

A request is one Box simulation (an SD count, a collision kernel, a seed and a
number of steps), in the sense of the PySDM v1 paper's "API in brief"
(Builder + Box + Coalescence, then run(n_steps)).  The server keeps a queue of
arrived requests and a set of resident simulations:

  * admission: a request is admitted when a resident slot is free and its
    device footprint (state + workspace) fits in what is left of the HBM
    budget; its state stays resident on the device until it finishes;
  * every tick, ONE shared launch per step advances all resident simulations
    (sdm_batch_step), each by its own counter-based random numbers, so a
    simulation's result does not depend on what it is batched with;
  * requests that arrive while a tick runs on the device are admitted while
    it runs (their upload and validation go on a second stream, and the
    library's set-up calls synchronise only that stream), and the next tick's
    shared-launch tables are built and uploaded then too, so the host work of
    a membership change overlaps the device work;
  * finished simulations are read back (moments), their slot and bytes freed,
    and their latency (completion - arrival) recorded.

The scheduler talks to an executor (``GpuExecutor`` here: the C ABI through
``binding``), so the same logic can be driven by any object with the same
methods.  Errors of one request (bad state, too large for the budget,
cancellation) are recorded for that request only.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Outcome:
    rid: int
    arrival_s: float
    admit_s: float | None = None
    done_s: float | None = None
    status: str = "queued"  # queued | running | done | rejected | failed | cancelled
    error: str | None = None
    result: dict | None = None
    sd_steps: int = 0

    @property
    def latency_s(self):
        return None if self.done_s is None else self.done_s - self.arrival_s


@dataclass
class ServeStats:
    outcomes: dict = field(default_factory=dict)
    ticks: int = 0
    launches: int = 0
    wall_s: float = 0.0
    max_resident: int = 0
    device_busy_s: float = 0.0

    def latencies(self):
        return np.array([o.latency_s for o in self.outcomes.values() if o.status == "done"])

    def summary(self):
        lat = self.latencies()
        done = [o for o in self.outcomes.values() if o.status == "done"]
        sd = sum(o.sd_steps for o in done)
        return {
            "done": len(done),
            "rejected": sum(o.status == "rejected" for o in self.outcomes.values()),
            "failed": sum(o.status == "failed" for o in self.outcomes.values()),
            "cancelled": sum(o.status == "cancelled" for o in self.outcomes.values()),
            "p50_s": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_s": float(np.percentile(lat, 99)) if lat.size else None,
            "mean_s": float(lat.mean()) if lat.size else None,
            "sd_steps": int(sd),
            "sd_steps_per_s": sd / self.wall_s if self.wall_s > 0 else None,
            "wall_s": self.wall_s,
            "ticks": self.ticks,
            "max_resident": self.max_resident,
        }


class Server:
    """Continuous-batching scheduler.

    executor: object with footprint(req, state), admit(req, state) -> handle,
      batch(handles) -> batch, step(batch, k) (enqueue), sync(),
      collect(handles) -> [result dict] (after sync), release(handle),
      step_of(handle); optionally prepare(handles) -> batch (built while a
      tick runs) and adopt(batch) (makes a prepared batch the current one).
    budget_bytes: device bytes the resident simulations may use.
    max_resident: resident slots.
    steps_per_tick: steps per shared launch sequence between admissions.
    """

    def __init__(self, executor, budget_bytes, max_resident=4096, steps_per_tick=50,
                 clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_resident = int(max_resident)
        self.k = int(steps_per_tick)
        self.clock = clock
        self.sleep = sleep
        self._cancel = set()

    def cancel(self, rid):
        self._cancel.add(rid)

    def run(self, requests, state_of, on_tick=None):
        """Serve `requests` (each with rid, arrival_s, n_steps) whose initial
        states come from state_of(req); returns ServeStats."""
        st = ServeStats()
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival_s, r.rid)))
        for r in pending:
            st.outcomes[r.rid] = Outcome(r.rid, r.arrival_s)
        waiting = collections.deque()
        resident = {}  # rid -> (req, handle, footprint)
        used = 0
        batch = None
        batch_members = None
        t0 = self.clock()

        def cancellations():
            nonlocal used
            for rid in list(self._cancel):
                o = st.outcomes.get(rid)
                if o is not None and rid in resident:
                    _, h, fp = resident.pop(rid)
                    self.ex.release(h)
                    used -= fp
                    o.status = "cancelled"
                elif o is not None:
                    for q in (waiting, pending):
                        for r in list(q):
                            if r.rid == rid:
                                q.remove(r)
                                o.status = "cancelled"
                self._cancel.discard(rid)

        def admit_arrived():
            # arrivals join the FIFO queue; the head is admitted when a slot is
            # free and its footprint fits the budget (no overtaking)
            nonlocal used
            now = self.clock() - t0
            while pending and pending[0].arrival_s <= now:
                waiting.append(pending.popleft())
            while waiting and len(resident) < self.max_resident:
                req = waiting[0]
                o = st.outcomes[req.rid]
                try:
                    state = state_of(req)
                    fp = int(self.ex.footprint(req, state))
                except Exception as e:  # noqa: BLE001  (per-request isolation)
                    waiting.popleft()
                    o.status, o.error = "failed", f"{type(e).__name__}: {e}"
                    continue
                if fp > self.budget:
                    waiting.popleft()
                    o.status, o.error = "rejected", f"footprint {fp} B exceeds budget {self.budget} B"
                    continue
                if used + fp > self.budget:
                    break  # back-pressure: wait until a resident request finishes
                waiting.popleft()
                try:
                    h = self.ex.admit(req, state)
                except Exception as e:  # noqa: BLE001
                    o.status, o.error = "failed", f"{type(e).__name__}: {e}"
                    continue
                resident[req.rid] = (req, h, fp)
                used += fp
                o.status, o.admit_s = "running", self.clock() - t0
            st.max_resident = max(st.max_resident, len(resident))

        prepared = None  # (members, batch) built while the previous tick ran
        can_prepare = hasattr(self.ex, "prepare") and hasattr(self.ex, "adopt")
        while pending or waiting or resident:
            cancellations()
            if not resident:
                admit_arrived()
                if not resident:
                    if pending:
                        wait = pending[0].arrival_s - (self.clock() - t0)
                        if wait > 0:
                            self.sleep(min(wait, 0.01))
                    elif waiting:  # nothing resident and the head can never fit
                        raise RuntimeError("admission stalled with an empty device")
                    continue
            members = tuple(sorted(resident))
            if members != batch_members:
                if prepared is not None and prepared[0] == members:
                    batch = self.ex.adopt(prepared[1])
                else:
                    batch = self.ex.batch([resident[r][1] for r in members])
                batch_members = members
            prepared = None
            t_dev = self.clock()
            self.ex.step(batch, self.k)  # enqueue: one shared launch per step
            st.launches += self.k
            st.ticks += 1
            finished = [r for r in members
                        if self.ex.step_of(resident[r][1]) >= resident[r][0].n_steps]
            admit_arrived()  # host admission work overlaps the device tick
            if can_prepare:  # and so does building the next tick's batch
                done = set(finished)
                nxt = tuple(sorted(r for r in resident if r not in done))
                if nxt and nxt != members:
                    prepared = (nxt, self.ex.prepare([resident[r][1] for r in nxt]))
            self.ex.sync()
            st.device_busy_s += self.clock() - t_dev
            results = self.ex.collect([resident[r][1] for r in finished]) if finished else []
            t_done = self.clock() - t0
            for rid, res in zip(finished, results):
                req, h, fp = resident.pop(rid)
                o = st.outcomes[rid]
                o.status, o.done_s, o.result = "done", t_done, res
                o.sd_steps = int(res.get("sd_steps", 0)) if isinstance(res, dict) else 0
                self.ex.release(h)
                used -= fp
            if on_tick is not None:
                on_tick(st, resident, used)
        st.wall_s = self.clock() - t0
        return st


class GpuExecutor:
    """Executor over the C ABI: one sdm_sim per request, shared launches via
    sdm_batch.  Device memory comes from torch's caching allocator, which
    recycles the blocks of finished requests (the pooled arena)."""

    def __init__(self, device="cuda", stream=None, keep_state=False):
        import torch

        from . import binding as B

        self.keep_state = keep_state
        self.B = B
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.admit_stream = torch.cuda.Stream()
        self._batch = None  # the batch the ticks run
        self._next = None  # a batch prepared for the next tick
        self._ws = [None, None]  # their workspaces (the current one is _ws[_cur])
        self._cur = 0

    def footprint(self, req, state):
        B = self.B
        cfg = B.make_config(state.n_slots, state.n_cells, state.n_attr, state.dt, state.dv,
                            state.kernel, state.adaptive, state.b, req.seed)
        ws = B.sdm_workspace_bytes(cfg, state.cell_off)
        if ws == 0:
            raise ValueError("invalid configuration")
        return ws + state.n_slots * (16 + 8 * state.n_attr) + 8 * (state.n_cells + 1)

    def admit(self, req, state):
        torch = self.torch
        # state upload and validation on a side stream: it overlaps the tick
        # running on the main stream
        with torch.cuda.stream(self.admit_stream):
            st = state
            st.seed = req.seed
            sim = self.B.Sim(st, device=self.device, stream=self.admit_stream)
            self.B.sdm_set_step_limit(sim.handle, req.n_steps)
        self.admit_stream.synchronize()
        sim.n_live0 = int((state.xi > 0).sum())
        return sim

    def _make(self, sims, slot, stream):
        handles = [s.handle for s in sims]
        nbytes = self.B.sdm_batch_workspace_bytes(handles)
        if self._ws[slot] is None or self._ws[slot].numel() < nbytes:
            self._ws[slot] = self.B.workspace_tensor(int(nbytes * 1.25) + 4096, self.device)
        return self.B.sdm_batch_create(handles, self._ws[slot], stream)

    def _free(self, b):
        if b is not None:
            self.B.sdm_batch_free(b)

    def batch(self, sims):
        """A batch for the next tick, built on the tick stream (after sync)."""
        self._free(self._batch)
        self._free(self._next)
        self._batch = self._next = None
        self._batch = self._make(sims, self._cur, self.stream)
        return self._batch

    def prepare(self, sims):
        """A batch for the next tick, built while the current tick runs: its
        tables go to the other workspace (not in use by the running batch),
        uploaded on the admission stream."""
        self._free(self._next)
        self._next = None
        self._next = self._make(sims, 1 - self._cur, self.admit_stream)
        return self._next

    def adopt(self, b):
        """Make a prepared batch current (the tick that used the old one has
        been synchronised)."""
        assert b is self._next
        self._free(self._batch)
        self._batch, self._next = b, None
        self._cur = 1 - self._cur
        return b

    def step(self, batch, k):
        self.B.sdm_batch_step(batch, k, self.stream)

    def step_of(self, sim):
        return self.B.sdm_get_step(sim.handle)

    def collect(self, sims):
        torch = self.torch
        bufs = []
        for s in sims:
            C_ = s.cfg.n_cells
            m0 = torch.empty(C_, dtype=torch.int64, device=self.device)
            m12 = torch.empty((C_, 2), dtype=torch.float64, device=self.device)
            self.B.sdm_moments(s.handle, m0, m12, None, None, None, self.stream)
            bufs.append((m0, m12))
        self.stream.synchronize()
        out = []
        for s, (m0, m12) in zip(sims, bufs):
            st = self.B.sdm_stats(s.handle, self.stream)
            r = {"m0": m0.cpu().numpy(), "m1": m12[:, 0].cpu().numpy(),
                 "m2": m12[:, 1].cpu().numpy(), "sd_steps": st["live_sd_steps"],
                 "steps": self.B.sdm_get_step(s.handle)}
            if self.keep_state:
                r["xi"], r["v"], _ = s.state()
            out.append(r)
        return out

    def sync(self):
        self.stream.synchronize()

    def release(self, sim):
        sim.close()

    def close(self):
        self._free(self._batch)
        self._free(self._next)
        self._batch = self._next = None


def serve_one_at_a_time(requests, state_of, executor, clock=time.perf_counter, sleep=time.sleep):
    """Baseline: FIFO, each request alone with its own per-step launches."""
    st = ServeStats()
    reqs = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
    t0 = clock()
    for r in reqs:
        o = Outcome(r.rid, r.arrival_s)
        st.outcomes[r.rid] = o
        wait = r.arrival_s - (clock() - t0)
        if wait > 0:
            sleep(wait)
        try:
            state = state_of(r)
            h = executor.admit(r, state)
        except Exception as e:  # noqa: BLE001
            o.status, o.error = "failed", f"{type(e).__name__}: {e}"
            continue
        o.admit_s = clock() - t0
        executor.step_alone(h, r.n_steps)
        st.launches += r.n_steps
        executor.sync()
        res = executor.collect([h])[0]
        o.status, o.done_s, o.result = "done", clock() - t0, res
        o.sd_steps = int(res.get("sd_steps", 0))
        executor.release(h)
    st.wall_s = clock() - t0
    return st


def _step_alone(self, sim, n):
    self.B.sdm_coalescence_step(sim.handle, n, self.stream)


GpuExecutor.step_alone = _step_alone
