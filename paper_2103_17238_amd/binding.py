"""ctypes binding of libsdm (include/sdm.h): argument marshalling only.

Every function has the name of the C entry point it wraps and does no
arithmetic of its own: device arrays are torch tensors (their data_ptr is
passed), streams are torch streams (their hipStream_t is passed).  The
library must have been built (``__graft_entry__.build()``); importing this
module raises if ``libsdm.so`` is missing, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsdm.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"libsdm.so not built at {_LIB_PATH}; run __graft_entry__.build()")
_lib = C.CDLL(_LIB_PATH)

SDM_OK, SDM_EINVAL, SDM_ENOMEM, SDM_EDEVICE, SDM_ESTATE, SDM_EAGAIN = 0, -1, -2, -3, -4, -5
SDM_GOLOVIN, SDM_GEOMETRIC = 0, 1
SDM_FLAG_SUBSTEP_CAP, SDM_FLAG_GAMMA_CAP = 1, 2
SDM_FLAG_BUCKET_OVERFLOW, SDM_FLAG_INVALID_STATE, SDM_FLAG_COURANT = 4, 8, 16

EXPORTED = [
    "sdm_workspace_bytes", "sdm_init", "sdm_coalescence_step", "sdm_moments", "sdm_status_word",
    "sdm_reset_status", "sdm_stats", "sdm_get_step", "sdm_set_step", "sdm_set_step_limit",
    "sdm_debug_gamma_sink", "sdm_get_tuning", "sdm_set_tuning", "sdm_autotune_scratch_bytes",
    "sdm_autotune", "sdm_batch_workspace_bytes", "sdm_batch_create", "sdm_batch_step",
    "sdm_batch_free", "sdm_free", "sdm_strerror", "sdm_philox_fill", "sdm_kernel_values",
    "sdm_rebind", "sdm_displace_workspace_bytes", "sdm_displace", "sdm_displace_noalloc",
    "sdm_displace_noalloc_max_cells", "sdm_condensation_step",
]


class sdm_config(C.Structure):
    _fields_ = [
        ("n_slots", C.c_int64),
        ("n_cells", C.c_int32),
        ("n_attr", C.c_int32),
        ("dt_s", C.c_double),
        ("dv_m3", C.c_double),
        ("kernel", C.c_int32),
        ("adaptive", C.c_int32),
        ("golovin_b_per_s", C.c_double),
        ("seed", C.c_uint64),
        ("max_substeps", C.c_int32),
        ("reserved", C.c_int32),
    ]


class sdm_tuning(C.Structure):
    _fields_ = [
        ("wave_class_mask", C.c_int32),
        ("waves_per_cell", C.c_int32),
        ("big_bucket_target", C.c_int32),
        ("lpt_order", C.c_int32),
        ("mid_max_slots", C.c_int32),
        ("big_bucket_cap", C.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_P = C.c_void_p
_H = C.c_void_p  # opaque handles
_S = C.c_int  # sdm_status


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("sdm_workspace_bytes", C.c_size_t, C.POINTER(sdm_config), _P)
_sig("sdm_init", _S, C.POINTER(_H), C.POINTER(sdm_config), _P, _P, _P, _P, _P, C.c_size_t, _P)
_sig("sdm_coalescence_step", _S, _H, C.c_int32, _P)
_sig("sdm_moments", _S, _H, _P, _P, _P, _P, C.c_int32, _P, _P)
_sig("sdm_status_word", _S, _H, C.POINTER(C.c_uint32), _P)
_sig("sdm_reset_status", _S, _H, _P)
_sig("sdm_stats", _S, _H, C.POINTER(C.c_uint64), _P)
_sig("sdm_get_step", C.c_uint32, _H)
_sig("sdm_set_step", _S, _H, C.c_uint32)
_sig("sdm_set_step_limit", _S, _H, C.c_uint32)
_sig("sdm_debug_gamma_sink", _S, _H, _P, C.c_int64)
_sig("sdm_get_tuning", _S, _H, C.POINTER(sdm_tuning))
_sig("sdm_set_tuning", _S, _H, C.POINTER(sdm_tuning), _P)
_sig("sdm_autotune_scratch_bytes", C.c_size_t, _H)
_sig("sdm_autotune", _S, _H, _P, C.c_size_t, C.c_int32, C.c_char_p, C.POINTER(sdm_tuning), _P)
_sig("sdm_batch_workspace_bytes", C.c_size_t, C.POINTER(_H), C.c_int32)
_sig("sdm_batch_create", _S, C.POINTER(_H), C.POINTER(_H), C.c_int32, _P, C.c_size_t, _P)
_sig("sdm_batch_step", _S, _H, C.c_int32, _P)
_sig("sdm_batch_free", None, _H)
_sig("sdm_free", None, _H)
_sig("sdm_strerror", C.c_char_p, _S)
_sig("sdm_philox_fill", _S, _P, C.c_int64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
     C.c_uint64, _P)
_sig("sdm_kernel_values", _S, C.c_int32, C.c_double, _P, _P, C.c_int64, _P, _P)


class sdm_displace_args(C.Structure):
    _fields_ = [
        ("nx", C.c_int32),
        ("nz", C.c_int32),
        ("n_attr", C.c_int32),
        ("reserved", C.c_int32),
        ("n_slots", C.c_int64),
        ("courant_x", _P),
        ("courant_z", _P),
        ("xi", _P),
        ("v", _P),
        ("attrs", _P),
        ("pos", _P),
        ("cell_off", _P),
        ("xi_out", _P),
        ("v_out", _P),
        ("attrs_out", _P),
        ("pos_out", _P),
        ("cell_off_out", _P),
        ("status", _P),
    ]


_sig("sdm_rebind", _S, _H, _P, _P, _P, _P, _P)
_sig("sdm_displace_workspace_bytes", C.c_size_t, C.c_int32, C.c_int32)
_sig("sdm_displace", _S, C.POINTER(sdm_displace_args), _P, C.c_size_t, _P)
_sig("sdm_displace_noalloc", _S, C.POINTER(sdm_displace_args), _P)
_sig("sdm_displace_noalloc_max_cells", C.c_int64)


class sdm_cond_config(C.Structure):
    _fields_ = [
        ("dt_s", C.c_double),
        ("dry_volume_attr", C.c_int32),
        ("kappa_attr", C.c_int32),
        ("max_iter", C.c_int32),
        ("reserved", C.c_int32),
    ]


_sig("sdm_condensation_step", _S, _H, C.POINTER(sdm_cond_config), _P, _P, _P, _P)


class SdmError(RuntimeError):
    def __init__(self, call, status):
        super().__init__(f"{call} failed: {_lib.sdm_strerror(status).decode()} ({status})")
        self.status = status


def _check(call, st):
    if st != SDM_OK:
        raise SdmError(call, st)


def library_path():
    return _LIB_PATH


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_config(n_slots, n_cells, n_attr=0, dt_s=1.0, dv_m3=1e6, kernel=SDM_GOLOVIN,
                adaptive=False, golovin_b_per_s=1500.0, seed=0, max_substeps=0) -> sdm_config:
    return sdm_config(int(n_slots), int(n_cells), int(n_attr), float(dt_s), float(dv_m3),
                      int(kernel), int(bool(adaptive)), float(golovin_b_per_s),
                      int(seed) & 0xFFFFFFFFFFFFFFFF, int(max_substeps), 0)


# ---------------------------------------------------------------------------
# 1:1 wrappers
# ---------------------------------------------------------------------------

def sdm_workspace_bytes(cfg: sdm_config, host_cell_off=None) -> int:
    off = None
    if host_cell_off is not None:
        host_cell_off = np.ascontiguousarray(host_cell_off, dtype=np.int64)
        off = host_cell_off.ctypes.data_as(C.c_void_p)
    return int(_lib.sdm_workspace_bytes(C.byref(cfg), off))


def sdm_init(cfg: sdm_config, xi, v, attrs, cell_off, workspace, stream=None):
    h = _H()
    _check("sdm_init", _lib.sdm_init(C.byref(h), C.byref(cfg), _ptr(xi), _ptr(v), _ptr(attrs),
                                     _ptr(cell_off), _ptr(workspace),
                                     workspace.numel() * workspace.element_size(),
                                     _stream(stream)))
    return h


def sdm_coalescence_step(h, n_steps: int, stream=None):
    _check("sdm_coalescence_step", _lib.sdm_coalescence_step(h, int(n_steps), _stream(stream)))


def sdm_condensation_step(h, cc: sdm_cond_config, temperature, pressure, saturation,
                          stream=None):
    _check("sdm_condensation_step",
           _lib.sdm_condensation_step(h, C.byref(cc), _ptr(temperature), _ptr(pressure),
                                      _ptr(saturation), _stream(stream)))


def sdm_moments(h, m0=None, m12=None, attr_sums=None, vol_edges=None, spectrum=None,
                stream=None):
    n_bins = 0 if vol_edges is None else int(vol_edges.numel()) - 1
    _check("sdm_moments", _lib.sdm_moments(h, _ptr(m0), _ptr(m12), _ptr(attr_sums),
                                           _ptr(vol_edges), n_bins, _ptr(spectrum),
                                           _stream(stream)))


def sdm_status_word(h, stream=None) -> int:
    out = C.c_uint32(0)
    _check("sdm_status_word", _lib.sdm_status_word(h, C.byref(out), _stream(stream)))
    return int(out.value)


def sdm_reset_status(h, stream=None):
    _check("sdm_reset_status", _lib.sdm_reset_status(h, _stream(stream)))


def sdm_stats(h, stream=None):
    out = (C.c_uint64 * 4)()
    _check("sdm_stats", _lib.sdm_stats(h, out, _stream(stream)))
    return {"live_sd_steps": int(out[0]), "colliding_pairs": int(out[1]),
            "cell_substeps": int(out[2]), "cell_steps": int(out[3])}


def sdm_get_step(h) -> int:
    return int(_lib.sdm_get_step(h))


def sdm_set_step(h, step: int):
    _check("sdm_set_step", _lib.sdm_set_step(h, int(step)))


def sdm_set_step_limit(h, limit: int):
    _check("sdm_set_step_limit", _lib.sdm_set_step_limit(h, int(limit) & 0xFFFFFFFF))


def sdm_debug_gamma_sink(h, buf):
    cap = 0 if buf is None else buf.numel()
    _check("sdm_debug_gamma_sink", _lib.sdm_debug_gamma_sink(h, _ptr(buf), cap))


def sdm_get_tuning(h) -> sdm_tuning:
    t = sdm_tuning()
    _check("sdm_get_tuning", _lib.sdm_get_tuning(h, C.byref(t)))
    return t


def sdm_set_tuning(h, t: sdm_tuning, stream=None):
    _check("sdm_set_tuning", _lib.sdm_set_tuning(h, C.byref(t), _stream(stream)))


def sdm_autotune_scratch_bytes(h) -> int:
    return int(_lib.sdm_autotune_scratch_bytes(h))


def sdm_autotune(h, scratch, trial_steps=3, cache_path=None, stream=None) -> sdm_tuning:
    t = sdm_tuning()
    nbytes = 0 if scratch is None else scratch.numel() * scratch.element_size()
    path = None if cache_path is None else os.fsencode(cache_path)
    _check("sdm_autotune", _lib.sdm_autotune(h, _ptr(scratch), nbytes, int(trial_steps), path,
                                             C.byref(t), _stream(stream)))
    return t


def sdm_batch_workspace_bytes(handles) -> int:
    arr = (_H * len(handles))(*[h.value if isinstance(h, _H) else h for h in handles])
    return int(_lib.sdm_batch_workspace_bytes(arr, len(handles)))


def sdm_batch_create(handles, workspace, stream=None):
    arr = (_H * len(handles))(*[h.value if isinstance(h, _H) else h for h in handles])
    b = _H()
    _check("sdm_batch_create", _lib.sdm_batch_create(
        C.byref(b), arr, len(handles), _ptr(workspace),
        workspace.numel() * workspace.element_size(), _stream(stream)))
    return b


def sdm_batch_step(b, n_steps: int, stream=None):
    _check("sdm_batch_step", _lib.sdm_batch_step(b, int(n_steps), _stream(stream)))


def sdm_batch_free(b):
    _lib.sdm_batch_free(b)


def sdm_free(h):
    _lib.sdm_free(h)


def sdm_rebind(h, xi, v, attrs, cell_off, stream=None):
    _check("sdm_rebind", _lib.sdm_rebind(h, _ptr(xi), _ptr(v), _ptr(attrs), _ptr(cell_off),
                                         _stream(stream)))


def sdm_displace_workspace_bytes(nx: int, nz: int) -> int:
    return int(_lib.sdm_displace_workspace_bytes(int(nx), int(nz)))


def sdm_displace(nx, nz, courant_x, courant_z, xi, v, attrs, pos, cell_off, xi_out, v_out,
                 attrs_out, pos_out, cell_off_out, status, workspace, stream=None):
    a = sdm_displace_args(int(nx), int(nz), int(attrs.shape[0]) if attrs is not None else 0, 0,
                          int(xi.numel()), _ptr(courant_x), _ptr(courant_z), _ptr(xi), _ptr(v),
                          _ptr(attrs), _ptr(pos), _ptr(cell_off), _ptr(xi_out), _ptr(v_out),
                          _ptr(attrs_out), _ptr(pos_out), _ptr(cell_off_out), _ptr(status))
    _check("sdm_displace", _lib.sdm_displace(C.byref(a), _ptr(workspace),
                                             workspace.numel() * workspace.element_size(),
                                             _stream(stream)))


def sdm_displace_noalloc(nx, nz, courant_x, courant_z, xi, v, attrs, pos, cell_off, xi_out,
                         v_out, attrs_out, pos_out, cell_off_out, status, stream=None):
    a = sdm_displace_args(int(nx), int(nz), int(attrs.shape[0]) if attrs is not None else 0, 0,
                          int(xi.numel()), _ptr(courant_x), _ptr(courant_z), _ptr(xi), _ptr(v),
                          _ptr(attrs), _ptr(pos), _ptr(cell_off), _ptr(xi_out), _ptr(v_out),
                          _ptr(attrs_out), _ptr(pos_out), _ptr(cell_off_out), _ptr(status))
    _check("sdm_displace_noalloc", _lib.sdm_displace_noalloc(C.byref(a), _stream(stream)))


def sdm_displace_noalloc_max_cells() -> int:
    return int(_lib.sdm_displace_noalloc_max_cells())


def sdm_strerror(st: int) -> str:
    return _lib.sdm_strerror(st).decode()


def sdm_philox_fill(out, n, c0, c1, c2, c3, seed, stream=None):
    _check("sdm_philox_fill", _lib.sdm_philox_fill(_ptr(out), int(n), c0, c1, c2, c3,
                                                   int(seed) & 0xFFFFFFFFFFFFFFFF,
                                                   _stream(stream)))


def sdm_kernel_values(kernel, golovin_b, v1, v2, out, stream=None):
    _check("sdm_kernel_values", _lib.sdm_kernel_values(int(kernel), float(golovin_b), _ptr(v1),
                                                       _ptr(v2), int(v1.numel()), _ptr(out),
                                                       _stream(stream)))


# ---------------------------------------------------------------------------
# Convenience holder: device tensors + handle (still marshalling only)
# ---------------------------------------------------------------------------

def workspace_tensor(nbytes, device="cuda"):
    import torch

    # 256-byte alignment comes from torch's caching allocator (512-byte blocks)
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Sim:
    """One simulation: owns its device tensors and workspace, borrows nothing."""

    def __init__(self, state, device="cuda", stream=None, max_substeps=0, any_layout=False):
        import torch

        self.device = device
        self.cfg = make_config(state.n_slots, state.n_cells, state.n_attr, state.dt, state.dv,
                               state.kernel, state.adaptive, state.b, state.seed, max_substeps)
        self.xi = torch.from_numpy(state.xi).to(device)
        self.v = torch.from_numpy(state.v).to(device)
        self.attrs = (torch.from_numpy(np.ascontiguousarray(state.attrs)).to(device)
                      if state.n_attr else None)
        self.cell_off = torch.from_numpy(state.cell_off).to(device)
        # any_layout: workspace for every cell layout (sdm_rebind after displacement)
        self.ws = workspace_tensor(
            sdm_workspace_bytes(self.cfg, None if any_layout else state.cell_off), device)
        self.handle = sdm_init(self.cfg, self.xi, self.v, self.attrs, self.cell_off, self.ws,
                               stream)

    def step(self, n=1, stream=None):
        sdm_coalescence_step(self.handle, n, stream)

    def state(self):
        import torch

        torch.cuda.synchronize()
        at = self.attrs.cpu().numpy() if self.attrs is not None else np.zeros((0, self.cfg.n_slots))
        return self.xi.cpu().numpy(), self.v.cpu().numpy(), at

    def moments(self, vol_edges=None, stream=None):
        import torch

        C_ = self.cfg.n_cells
        A = self.cfg.n_attr
        m0 = torch.empty(C_, dtype=torch.int64, device=self.device)
        m12 = torch.empty((C_, 2), dtype=torch.float64, device=self.device)
        asum = torch.empty((C_, max(A, 1)), dtype=torch.float64, device=self.device)
        e = spec = None
        if vol_edges is not None:
            e = torch.as_tensor(np.asarray(vol_edges, dtype=np.float64), device=self.device)
            spec = torch.empty((C_, e.numel() - 1), dtype=torch.float64, device=self.device)
        sdm_moments(self.handle, m0, m12, asum if A else None, e, spec, stream)
        torch.cuda.synchronize()
        out = {"m0": m0.cpu().numpy(), "m1": m12[:, 0].cpu().numpy(),
               "m2": m12[:, 1].cpu().numpy(), "attr_sums": asum[:, :A].cpu().numpy()}
        if spec is not None:
            out["spectrum"] = spec.cpu().numpy()
        return out

    def close(self):
        if self.handle is not None:
            sdm_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Kinematic2D:
    """Displacement of a Sim's droplets in a prescribed 2D flow (nx x nz cells,
    c = ix * nz + iz): holds the face Courant numbers, the droplet positions
    and a second set of state buffers; each step displaces and re-segments
    into the other buffers and re-points the Sim at them (sdm_rebind).  The
    Sim must have been made with any_layout=True."""

    def __init__(self, sim: Sim, nx, nz, courant_x, courant_z, pos, stream=None):
        import torch

        dev = sim.device
        self.sim, self.nx, self.nz = sim, int(nx), int(nz)
        self.cx = torch.as_tensor(np.ascontiguousarray(courant_x, dtype=np.float64), device=dev)
        self.cz = torch.as_tensor(np.ascontiguousarray(courant_z, dtype=np.float64), device=dev)
        self.pos = torch.as_tensor(np.ascontiguousarray(pos, dtype=np.float64), device=dev)
        self.other = (torch.empty_like(sim.xi), torch.empty_like(sim.v),
                      torch.empty_like(sim.attrs) if sim.attrs is not None else None,
                      torch.empty_like(self.pos), torch.empty_like(sim.cell_off))
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        nb = sdm_displace_workspace_bytes(nx, nz)
        if nb == 0:
            raise ValueError("displacement needs nx, nz >= 1")
        self.ws = workspace_tensor(nb, dev)

    def displace(self, stream=None):
        """One displacement + re-segmentation (enqueue only); swaps buffers."""
        s = self.sim
        xo, vo, ao, po, oo = self.other
        sdm_displace(self.nx, self.nz, self.cx, self.cz, s.xi, s.v, s.attrs, self.pos, s.cell_off,
                     xo, vo, ao, po, oo, self.status, self.ws, stream)
        self.other = (s.xi, s.v, s.attrs, self.pos, s.cell_off)
        s.xi, s.v, s.attrs, self.pos, s.cell_off = xo, vo, ao, po, oo

    def rebind(self, stream=None):
        """Re-plan the Sim's coalescence launches for the current layout."""
        s = self.sim
        sdm_rebind(s.handle, s.xi, s.v, s.attrs, s.cell_off, stream)

    def step(self, stream=None):
        self.displace(stream)
        self.rebind(stream)

    def flags(self):
        import torch

        torch.cuda.synchronize()
        return int(self.status.item()) & 0xFFFFFFFF
