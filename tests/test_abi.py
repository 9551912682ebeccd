"""The C ABI library loads on the CPU and exports every entry point that
include/sdm.h declares (no compute calls without a GPU)."""
import ctypes
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "sdm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sdm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_core_calls():
    names = declared()
    for n in ("sdm_init", "sdm_coalescence_step", "sdm_moments", "sdm_batch_step", "sdm_free"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2103_17238_amd import binding

    lib = ctypes.CDLL(binding.library_path())
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.check_output(["nm", "-D", "--defined-only", binding.library_path()], text=True)
    exported = {ln.split()[-1] for ln in out.splitlines() if ln.split()}
    assert set(declared()) <= exported
    assert set(binding.EXPORTED) == set(declared())


def test_host_side_sizes_and_errors():
    from paper_2103_17238_amd import binding as B

    cfg = B.make_config(1000, 4)
    bound = B.sdm_workspace_bytes(cfg)
    exact = B.sdm_workspace_bytes(cfg, [0, 100, 600, 700, 1000])
    assert 0 < exact <= bound
    assert B.sdm_workspace_bytes(B.make_config(10, 0)) == 0  # no cells
    assert B.sdm_workspace_bytes(B.make_config(10, 2, dt_s=-1.0)) == 0
    assert B.sdm_workspace_bytes(cfg, [0, 100, 50, 700, 1000]) == 0  # offsets not monotone
    assert B.sdm_strerror(B.SDM_ENOMEM) == "workspace too small"


def test_workspace_bound_covers_big_cells():
    """The layout-free workspace bound covers the exact size of layouts with
    big cells of many sizes (one and several chunks, many buckets), and a cell
    above 8 388 608 slots is an invalid layout."""
    import numpy as np

    from paper_2103_17238_amd import binding as B

    n = 8388608
    one = B.sdm_workspace_bytes(B.make_config(n, 1), [0, n])
    assert 0 < one <= B.sdm_workspace_bytes(B.make_config(n, 1))
    assert B.sdm_workspace_bytes(B.make_config(n + 1, 1), [0, n + 1]) == 0
    assert B.sdm_workspace_bytes(B.make_config(n + 1, 2), [0, 1, n + 1]) > 0
    for sizes in ([513, 600, 20000], [262144, 262145], [1 << 20, 3], [5000] * 7, [100] * 50):
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
        for adaptive in (False, True):
            cfg = B.make_config(int(off[-1]), len(sizes), n_attr=2, adaptive=adaptive)
            exact = B.sdm_workspace_bytes(cfg, off)
            assert 0 < exact <= B.sdm_workspace_bytes(cfg), (sizes, adaptive)


def test_displace_argument_checks():
    """Argument errors of sdm_displace are caught on the host before any HIP
    call (fake device addresses are never dereferenced)."""
    import ctypes as C

    from paper_2103_17238_amd import binding as B

    assert B.sdm_displace_workspace_bytes(0, 5) == 0
    assert B.sdm_displace_workspace_bytes(1, 1) > 0
    lib = C.CDLL(B.library_path())
    f = lib.sdm_displace
    f.restype = C.c_int
    f.argtypes = [C.POINTER(B.sdm_displace_args), C.c_void_p, C.c_size_t, C.c_void_p]

    def args(nx=4, nz=4, n=100, A=1, **kw):
        base = 1 << 40
        a = B.sdm_displace_args(nx, nz, A, 0, n)
        names = ["courant_x", "courant_z", "xi", "v", "attrs", "pos", "cell_off", "xi_out",
                 "v_out", "attrs_out", "pos_out", "cell_off_out", "status"]
        for k, nm in enumerate(names):
            setattr(a, nm, base + (k << 24))
        for k, val in kw.items():
            setattr(a, k, val)
        return a

    ws = 1 << 45
    good = args()
    assert f(C.byref(args(nx=0)), ws, 1 << 30, None) == B.SDM_EINVAL
    assert f(C.byref(args(A=17)), ws, 1 << 30, None) == B.SDM_EINVAL
    assert f(C.byref(args(reserved=1)), ws, 1 << 30, None) == B.SDM_EINVAL
    assert f(C.byref(args(xi=None)), ws, 1 << 30, None) == B.SDM_EINVAL
    assert f(C.byref(args(xi_out=good.xi + 8)), ws, 1 << 30, None) == B.SDM_EINVAL  # overlap
    assert f(C.byref(good), ws + 8, 1 << 30, None) == B.SDM_EINVAL  # misaligned workspace
    assert f(C.byref(good), ws, 16, None) == B.SDM_ENOMEM
