"""ctypes wrapper of the plain-C SDM oracle (test infrastructure only).

Every function here marshals numpy arrays into ``sdm_oracle.c`` and back; the
arithmetic lives in the C file, which cites the SDM description it follows
(Shima et al. 2009, as named by the PySDM v1 paper, sections "Introduction",
"API in brief" and "Box environment examples").
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

GOLOVIN = 0
GEOMETRIC = 1
ST_SUBSTEP_CAP = 1
ST_GAMMA_CAP = 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sdm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Plain C, IEEE fp64, no contraction of a*b+c, no fast-math.
CFLAGS = ["-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile ``sdm_oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("n_slots", C.c_int64),
        ("n_cells", C.c_int32),
        ("n_attr", C.c_int32),
        ("dt", C.c_double),
        ("dv", C.c_double),
        ("b", C.c_double),
        ("kernel", C.c_int32),
        ("adaptive", C.c_int32),
        ("max_substeps", C.c_int32),
        ("n_threads", C.c_int32),
        ("seed", C.c_uint64),
    ]


@dataclass
class OracleConfig:
    n_slots: int
    n_cells: int
    n_attr: int = 0
    dt: float = 1.0
    dv: float = 1e6
    b: float = 1500.0
    kernel: int = GOLOVIN
    adaptive: bool = False
    max_substeps: int = 1024
    n_threads: int = 1
    seed: int = 0

    def c(self) -> _Cfg:
        return _Cfg(self.n_slots, self.n_cells, self.n_attr, self.dt, self.dv, self.b,
                    self.kernel, int(bool(self.adaptive)), self.max_substeps, self.n_threads,
                    self.seed & 0xFFFFFFFFFFFFFFFF)


_lib = None


def lib():
    """Load (building first if needed) the oracle shared library."""
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        L.orc_philox4x32_10.argtypes = [P, P, P]
        L.orc_philox_fill.argtypes = [C.c_uint32] * 4 + [C.c_uint64, C.c_int64, P]
        L.orc_phi.argtypes = [C.c_uint32, C.c_uint32]
        L.orc_phi.restype = C.c_double
        L.orc_radius.argtypes = [C.c_double]
        L.orc_radius.restype = C.c_double
        L.orc_terminal_velocity.argtypes = [C.c_double]
        L.orc_terminal_velocity.restype = C.c_double
        L.orc_kernel.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double]
        L.orc_kernel.restype = C.c_double
        L.orc_scale_factor.argtypes = [C.c_int64]
        L.orc_scale_factor.restype = C.c_int64
        L.orc_pair_probability.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_int64,
                                           C.c_int64, C.c_double, C.c_double, C.c_int64]
        L.orc_pair_probability.restype = C.c_double
        L.orc_gamma.argtypes = [C.c_double, C.c_double]
        L.orc_gamma.restype = C.c_int64
        L.orc_update_pair.argtypes = [P, P, P, C.c_int32, C.c_int64]
        L.orc_cell_order.argtypes = [P, C.c_int64, C.c_uint64, C.c_int32, C.c_uint32,
                                     C.c_uint32, P]
        L.orc_cell_order.restype = C.c_int64
        L.orc_pairs_for_order.argtypes = [C.c_int32, C.c_double, C.c_double, P, P, P,
                                          C.c_int64, P]
        L.orc_step.argtypes = [C.POINTER(_Cfg), P, P, P, P, C.c_uint32, P, P, P]
        L.orc_step.restype = C.c_uint32
        L.orc_cell_adaptive_trace.argtypes = [C.POINTER(_Cfg), P, P, P, C.c_int64, C.c_int32,
                                              C.c_uint32, C.c_int32, P, P, P, P, P, P]
        L.orc_cell_adaptive_trace.restype = C.c_int32
        L.orc_moments.argtypes = [C.POINTER(_Cfg), P, P, P, P, P, P, P, P, C.c_int32, P]
        L.orc_probe_mul_add.argtypes = [C.c_double] * 3
        L.orc_probe_mul_add.restype = C.c_double
        L.orc_max_threads.restype = C.c_int32
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _need(a, dtype):
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags["C_CONTIGUOUS"]):
        raise TypeError(f"expected a C-contiguous {np.dtype(dtype).name} array")
    return a


# ----------------------------------------------------------------------------
# Scalar / small helpers (pins)
# ----------------------------------------------------------------------------

def philox4x32_10(ctr, key):
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def philox_fill(c0, c1, c2, c3, seed, n):
    out = np.zeros(4 * n, dtype=np.uint32)
    lib().orc_philox_fill(c0, c1, c2, c3, seed & 0xFFFFFFFFFFFFFFFF, n, _ptr(out))
    return out.reshape(n, 4)


def phi_from_words(hi, lo):
    return lib().orc_phi(hi, lo)


def radius(v):
    return lib().orc_radius(v)


def terminal_velocity(r):
    return lib().orc_terminal_velocity(r)


def kernel_value(kind, b, v1, v2):
    return lib().orc_kernel(kind, b, v1, v2)


def scale_factor(n):
    return lib().orc_scale_factor(n)


def pair_probability(kind, b, q, xa, xb, va, vb, scale):
    return lib().orc_pair_probability(kind, b, q, xa, xb, va, vb, scale)


def gamma_from(p, phi):
    return lib().orc_gamma(p, phi)


def update_pair(xi2, v2, attrs2, gamma):
    """Apply the update rule to one pair; arrays are modified in place."""
    xi2 = _need(xi2, np.int64)
    v2 = _need(v2, np.float64)
    n_attr = 0 if attrs2 is None else attrs2.shape[0]
    if attrs2 is not None:
        _need(attrs2, np.float64)
    lib().orc_update_pair(_ptr(xi2), _ptr(v2), _ptr(attrs2), n_attr, gamma)


def cell_order(xi_cell, seed, c, s, u=0):
    """Live cell-local slots of one cell in permuted order."""
    xi_cell = _need(np.ascontiguousarray(xi_cell, dtype=np.int64), np.int64)
    order = np.zeros(max(len(xi_cell), 1), dtype=np.int64)
    n = lib().orc_cell_order(_ptr(xi_cell), len(xi_cell), seed & 0xFFFFFFFFFFFFFFFF, c, s, u,
                             _ptr(order))
    return order[:n].copy()


def pairs_for_order(kind, b, q, xi, v, order):
    xi = np.ascontiguousarray(xi, dtype=np.int64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    order = np.ascontiguousarray(order, dtype=np.int64)
    out = np.zeros(max(len(order) // 2, 1), dtype=np.float64)
    lib().orc_pairs_for_order(kind, b, q, _ptr(xi), _ptr(v), _ptr(order), len(order), _ptr(out))
    return out[: len(order) // 2].copy()


def pair_base(cell_off):
    """Start of each cell's candidate-pair range in the pair log (int64[C+1])."""
    sizes = np.diff(np.asarray(cell_off, dtype=np.int64))
    return np.concatenate([[0], np.cumsum(sizes // 2)]).astype(np.int64)


def step(cfg: OracleConfig, xi, v, attrs, cell_off, step_index, want_log=False,
         want_substeps=False):
    """One outer step, in place.  Returns dict(status, tallies, log?, substeps?)."""
    _need(xi, np.int64)
    _need(v, np.float64)
    _need(cell_off, np.int64)
    if cfg.n_attr:
        _need(attrs, np.float64)
        assert attrs.size == cfg.n_attr * cfg.n_slots
    assert xi.size == cfg.n_slots and v.size == cfg.n_slots and cell_off.size == cfg.n_cells + 1
    log = np.zeros(2 * int(pair_base(cell_off)[-1]), dtype=np.int64) if want_log else None
    sub = np.zeros(cfg.n_cells, dtype=np.int32) if want_substeps else None
    tallies = np.zeros(3, dtype=np.int64)
    c = cfg.c()
    st = lib().orc_step(C.byref(c), _ptr(xi), _ptr(v), _ptr(attrs if cfg.n_attr else None),
                        _ptr(cell_off), step_index, _ptr(log), _ptr(sub), _ptr(tallies))
    out = {"status": int(st), "tallies": tallies}
    if want_log:
        out["log"] = log.reshape(-1, 2)
    if want_substeps:
        out["substeps"] = sub
    return out


def cell_adaptive_trace(cfg: OracleConfig, xi, v, attrs, c, step_index, cap=4096):
    """One adaptive outer step of a single cell (the whole arrays are the
    cell), in place, recording every substep.  Returns a list of dicts with
    dt_left, dt_sub, n_live, clamped and the substep's pair log (rows
    (a | b << 32, gamma)), and the status bits."""
    _need(xi, np.int64)
    _need(v, np.float64)
    n = xi.size
    assert cfg.n_slots == n and v.size == n
    if cfg.n_attr:
        _need(attrs, np.float64)
        assert attrs.size == cfg.n_attr * n
    npair = n // 2
    dl = np.zeros(cap)
    ds = np.zeros(cap)
    nl = np.zeros(cap, dtype=np.int64)
    cl = np.zeros(cap, dtype=np.int32)
    log = np.zeros(max(cap * 2 * npair, 1), dtype=np.int64)
    st = np.zeros(1, dtype=np.uint32)
    cc = cfg.c()
    k = lib().orc_cell_adaptive_trace(C.byref(cc), _ptr(xi), _ptr(v),
                                      _ptr(attrs if cfg.n_attr else None), n, c, step_index, cap,
                                      _ptr(dl), _ptr(ds), _ptr(nl), _ptr(cl), _ptr(log), _ptr(st))
    subs = []
    for i in range(k):
        subs.append({"dt_left": float(dl[i]), "dt_sub": float(ds[i]), "n_live": int(nl[i]),
                     "clamped": bool(cl[i]),
                     "log": log[i * 2 * npair:(i + 1) * 2 * npair].reshape(-1, 2).copy()})
    return subs, int(st[0])


def moments(cfg: OracleConfig, xi, v, attrs, cell_off, vol_edges=None):
    C_ = cfg.n_cells
    m0 = np.zeros(C_, dtype=np.int64)
    m12 = np.zeros((C_, 2), dtype=np.float64)
    asum = np.zeros((C_, max(cfg.n_attr, 1)), dtype=np.float64)
    nb = 0 if vol_edges is None else len(vol_edges) - 1
    spec = np.zeros((C_, max(nb, 1)), dtype=np.float64)
    edges = None if vol_edges is None else np.ascontiguousarray(vol_edges, dtype=np.float64)
    c = cfg.c()
    lib().orc_moments(C.byref(c), _ptr(xi), _ptr(v), _ptr(attrs if cfg.n_attr else None),
                      _ptr(cell_off), _ptr(m0), _ptr(m12), _ptr(asum), _ptr(edges), nb,
                      _ptr(spec))
    return {"m0": m0, "m1": m12[:, 0].copy(), "m2": m12[:, 1].copy(),
            "attr_sums": asum[:, : cfg.n_attr].copy(), "spectrum": spec[:, :nb].copy()}


def probe_mul_add(a, b, c):
    return lib().orc_probe_mul_add(a, b, c)


def max_threads():
    return lib().orc_max_threads()
