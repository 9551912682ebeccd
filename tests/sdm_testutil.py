"""Helpers shared by the GPU tests: run the same seeded state through the HIP
library (via the C ABI binding) and through the CPU oracle."""
from __future__ import annotations

import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def ocfg(orc, st, **kw):
    d = dict(n_slots=st.n_slots, n_cells=st.n_cells, n_attr=st.n_attr, dt=st.dt, dv=st.dv,
             b=st.b, kernel=st.kernel, adaptive=st.adaptive, seed=st.seed)
    d.update(kw)
    return orc.OracleConfig(**d)


class GpuRun:
    """A simulation on the GPU through the C ABI, with an optional gamma sink."""

    def __init__(self, B, st, sink=False, tuning=None, max_substeps=0):
        import torch

        self.B = B
        self.st = st
        self.sim = B.Sim(st, max_substeps=max_substeps)
        self.sink = None
        if sink:
            npairs = int((np.diff(st.cell_off) // 2).sum())
            self.sink = torch.full((max(2 * npairs, 2),), -7, dtype=torch.int64, device="cuda")
            B.sdm_debug_gamma_sink(self.sim.handle, self.sink)
        if tuning is not None:
            t = B.sdm_get_tuning(self.sim.handle)
            for k, v in tuning.items():
                setattr(t, k, v)
            B.sdm_set_tuning(self.sim.handle, t)

    def step(self, n=1):
        self.sim.step(n)

    def state(self):
        return self.sim.state()

    def log(self):
        import torch

        torch.cuda.synchronize()
        npairs = int((np.diff(self.st.cell_off) // 2).sum())
        return self.sink[: 2 * npairs].cpu().numpy().reshape(-1, 2)

    def set_state(self, xi, v, attrs):
        import torch

        self.sim.xi.copy_(torch.from_numpy(np.ascontiguousarray(xi)))
        self.sim.v.copy_(torch.from_numpy(np.ascontiguousarray(v)))
        if self.sim.attrs is not None:
            self.sim.attrs.copy_(torch.from_numpy(np.ascontiguousarray(attrs)))
        torch.cuda.synchronize()

    def close(self):
        self.sim.close()


def rel_close(a, b, rel):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.maximum(np.abs(a), np.abs(b))
    diff = np.abs(a - b)
    return bool(np.all((diff == 0) | (diff <= rel * den)))
