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
