"""The CPU oracle built under AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, OpenMP over cells on two threads), run through tests/sanitize_driver.c
on uneven cells (empty, one-SD and full cells, dead slots, ties, splits,
multiple collisions, adaptive substeps, attributes, moments and a spectrum):
no sanitizer report, and every output bit-identical to the regular build's.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2103_17238_amd import inputs as I

from sdm_testutil import ocfg

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("san") / "sanitize_driver")
    cmd = ["gcc", "-std=c11", "-D_GNU_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", out, os.path.join(HERE, "sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "sdm_oracle.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("no sanitizer runtime: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return out


def _write_input(path, st, cfg, n_steps, edges):
    with open(path, "wb") as f:
        hdr = [cfg.n_slots, cfg.n_cells, cfg.n_attr, cfg.kernel, int(cfg.adaptive),
               cfg.max_substeps, cfg.n_threads, n_steps, len(edges) - 1]
        f.write(np.array(hdr, dtype=np.int64).tobytes())
        f.write(np.array([cfg.seed], dtype=np.uint64).tobytes())
        f.write(np.array([cfg.dt, cfg.dv, cfg.b], dtype=np.float64).tobytes())
        f.write(st.xi.astype(np.int64).tobytes())
        f.write(st.v.astype(np.float64).tobytes())
        f.write(np.ascontiguousarray(st.attrs, dtype=np.float64).tobytes())
        f.write(st.cell_off.astype(np.int64).tobytes())
        f.write(np.asarray(edges, dtype=np.float64).tobytes())


class _Reader:
    def __init__(self, path):
        self.b = open(path, "rb").read()
        self.at = 0

    def take(self, dtype, n):
        dt = np.dtype(dtype)
        a = np.frombuffer(self.b, dtype=dt, count=n, offset=self.at)
        self.at += dt.itemsize * n
        return a


CASES = {
    # geometric kernel, adaptive substeps (p boosted so that several are
    # needed), three attributes
    "geometric-adaptive": dict(kernel=I.GEOMETRIC, adaptive=True, n_attr=3, p_boost=1.0,
                               dv=1e2),
    # Golovin with p > 1 (multiple collisions per pair) and ties / splits
    "golovin-plain": dict(kernel=I.GOLOVIN, adaptive=False, n_attr=2, p_boost=3e4, dv=1e6),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_sanitized_oracle_matches_regular_build(orc, driver, tmp_path, case):
    kw = CASES[case]
    st = I.random_cells(24, 300, n_attr=kw["n_attr"], kernel=kw["kernel"], rng_seed=11,
                        dv=kw["dv"], p_boost=kw["p_boost"])
    st.adaptive = kw["adaptive"]
    cfg = ocfg(orc, st, n_threads=2, max_substeps=64)
    n_steps = 4
    edges = np.geomspace(1e-18, 1e-9, 17)
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write_input(inp, st, cfg, n_steps, edges)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=23",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=24",
               OMP_NUM_THREADS="2")
    r = subprocess.run([driver, inp, outp], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-3000:]

    # the regular build on the same inputs
    o = st.copy()
    npairs = int(orc.pair_base(o.cell_off)[-1])
    rd = _Reader(outp)
    collided = 0
    for s in range(n_steps):
        ref = orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s, want_log=True, want_substeps=True)
        assert int(rd.take(np.uint32, 1)[0]) == ref["status"], s
        tal = rd.take(np.int64, 3)
        assert np.array_equal(tal, ref["tallies"]), s
        assert np.array_equal(rd.take(np.int32, st.n_cells), ref["substeps"]), s
        assert np.array_equal(rd.take(np.int64, 2 * npairs), ref["log"].reshape(-1)), s
        collided += int(tal[2])
    assert np.array_equal(rd.take(np.int64, st.n_slots), o.xi)
    assert np.array_equal(rd.take(np.float64, st.n_slots).view(np.uint64), o.v.view(np.uint64))
    A = st.n_attr
    assert np.array_equal(rd.take(np.float64, A * st.n_slots).view(np.uint64),
                          np.ascontiguousarray(o.attrs).reshape(-1).view(np.uint64))
    m = orc.moments(cfg, o.xi, o.v, o.attrs, o.cell_off, edges)
    assert np.array_equal(rd.take(np.int64, st.n_cells), m["m0"])
    m12 = rd.take(np.float64, 2 * st.n_cells).reshape(-1, 2)
    assert np.array_equal(m12[:, 0], m["m1"]) and np.array_equal(m12[:, 1], m["m2"])
    assert np.array_equal(rd.take(np.float64, st.n_cells * A).reshape(st.n_cells, A),
                          m["attr_sums"])
    assert np.array_equal(rd.take(np.float64, st.n_cells * 16).reshape(st.n_cells, 16),
                          m["spectrum"])
    assert rd.at == len(rd.b)
    # the case did exercise collisions (and, adaptive, several substeps)
    assert collided > 0
    if kw["adaptive"]:
        assert ref["substeps"].max() > 1
