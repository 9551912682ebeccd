"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars: int64 multiplicities bit-exact; volumes and attributes within 1e-12
relative under the Golovin kernel (bit-exact is expected: same operations in
the same order); under the geometric kernel, where the device and host cube
roots may differ in the last bit, a teacher-forced comparison (the oracle
restarts from the GPU's pre-step state every step) must find at most 1e-6 of
the pair-steps with a different gamma.
"""
import numpy as np
import pytest

from oracle import closed_form as cf
from paper_2103_17238_amd import inputs as I

from sdm_testutil import GpuRun, ocfg, rel_close, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_17238_amd import binding

    return binding


def test_philox_parity(B, orc):
    import torch

    for (c0, c1, c2, c3, seed, n) in [(0, 0, 0, 0, 0, 1 << 20), (0xFFFF0000, 7, 3599, 3, 42, 1 << 20),
                                      (5, 65535, 199, 1, 0xDEADBEEFCAFEF00D, 1 << 21)]:
        say(f"philox c=({c0},{c1},{c2},{c3}) seed={seed} n={n}")
        out = torch.empty(4 * n, dtype=torch.int32, device="cuda")
        B.sdm_philox_fill(out, n, c0, c1, c2, c3, seed)
        torch.cuda.synchronize()
        gpu = out.cpu().numpy().view(np.uint32).reshape(n, 4)
        ref = orc.philox_fill(c0, c1, c2, c3, seed, n)
        assert np.array_equal(gpu, ref)


def test_kernel_values(B, orc):
    import torch

    rng = np.random.default_rng(3)
    n = 20000
    v1 = cf.volume_of_radius(10 ** rng.uniform(-6.5, -2.5, size=n))
    v2 = cf.volume_of_radius(10 ** rng.uniform(-6.5, -2.5, size=n))
    for kind in (0, 1):
        say(f"kernel values kind={kind}")
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        B.sdm_kernel_values(kind, 1500.0, torch.from_numpy(v1).cuda(), torch.from_numpy(v2).cuda(),
                            out)
        torch.cuda.synchronize()
        g = out.cpu().numpy()
        ref = np.array([orc.kernel_value(kind, 1500.0, a, b) for a, b in zip(v1, v2)])
        if kind == 0:
            assert np.array_equal(g, ref)
        else:
            # cube roots may differ in the last bit between the device and host
            # libraries; |u1 - u2| can cancel, so errors are measured against
            # the uncancelled magnitude pi (r1 + r2)^2 (u1 + u2)
            r1 = np.array([orc.radius(a) for a in v1])
            r2 = np.array([orc.radius(b) for b in v2])
            u1 = np.array([orc.terminal_velocity(r) for r in r1])
            u2 = np.array([orc.terminal_velocity(r) for r in r2])
            scale = np.pi * (r1 + r2) ** 2 * (u1 + u2)
            err = np.abs(g - ref) / scale
            say(f"  geometric: exact {(g == ref).mean():.6f}, max err/scale {err.max():.3e}")
            assert err.max() < 1e-14


def _compare_run(B, orc, st, steps, sink=True, tuning=None, every=1, label=""):
    """Free run of GPU and oracle from the same state; bit-exact (Golovin)."""
    g = GpuRun(B, st, sink=sink, tuning=tuning)
    o = st.copy()
    cfg = ocfg(orc, o)
    for s in range(steps):
        g.step(1)
        out = orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s, want_log=sink)
        if (s + 1) % every == 0 or s == steps - 1:
            xi, v, at = g.state()
            assert np.array_equal(xi, o.xi), f"{label} xi differs at step {s}"
            assert rel_close(v, o.v, 1e-12), f"{label} v differs at step {s}"
            assert rel_close(at, o.attrs, 1e-12), f"{label} attrs differ at step {s}"
            if sink:
                assert np.array_equal(g.log(), out["log"]), f"{label} pair log differs at step {s}"
    xi, v, at = g.state()
    exact = np.array_equal(v, o.v) and np.array_equal(at, o.attrs)
    g.close()
    return exact


def test_golovin_box_small_all_steps(B, orc):
    """The 2^13-SD Golovin box, all 3600 steps, compared after every step."""
    st = I.golovin_box(2 ** 13)
    say("golovin box 2^13, 3600 steps")
    assert _compare_run(B, orc, st, 3600, sink=False, label="golovin-2^13")


@pytest.mark.parametrize("max_sd,seed,n_attr,boost", [
    (70, 1, 0, 1.0), (300, 2, 2, 1.0), (512, 3, 1, 1e4), (1500, 4, 3, 1.0), (3000, 5, 0, 3e3),
])
def test_golovin_random_cells(B, orc, max_sd, seed, n_attr, boost):
    """Uneven cells (0, 1, ragged, up to and past the one-wave limit), dead
    slots, ties, equal splits and gamma > 1."""
    st = I.random_cells(40, max_sd, n_attr=n_attr, rng_seed=seed, p_boost=boost)
    say(f"golovin random cells max_sd={max_sd} seed={seed} A={n_attr} boost={boost}")
    assert _compare_run(B, orc, st, 25, label=f"rc{max_sd}")


def test_golovin_tunings_same_result(B, orc):
    st = I.random_cells(64, 900, n_attr=1, rng_seed=9, p_boost=100.0)
    for tu in [dict(wave_class_mask=0x10, waves_per_cell=1, big_bucket_target=32),
               dict(wave_class_mask=0x1F, waves_per_cell=8, big_bucket_target=1024),
               dict(wave_class_mask=0x1A, waves_per_cell=2, big_bucket_target=128),
               dict(wave_class_mask=0x14, waves_per_cell=4, big_bucket_target=64, mid_max_slots=0),
               dict(wave_class_mask=0x18, waves_per_cell=2, mid_max_slots=2048),
               dict(wave_class_mask=0x1C, waves_per_cell=1)]:
        say(f"tuning {tu}")
        assert _compare_run(B, orc, st, 6, tuning=tu, label=str(tu))


def test_bucket_overflow_path_exact(B, orc):
    """A 2^16-SD cell with 1024-SD buckets: many buckets exceed the LDS stage
    and take the slow exact path."""
    st = I.golovin_box(2 ** 16)
    say("bucket overflow path 2^16")
    g = GpuRun(B, st, sink=True, tuning=dict(big_bucket_target=1024))
    o = st.copy()
    cfg = ocfg(orc, o)
    for s in range(3):
        g.step(1)
        out = orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s, want_log=True)
        xi, v, _ = g.state()
        assert np.array_equal(xi, o.xi) and np.array_equal(v, o.v)
        assert np.array_equal(g.log(), out["log"])
    assert B.sdm_status_word(g.sim.handle) & B.SDM_FLAG_BUCKET_OVERFLOW
    g.close()


@pytest.mark.parametrize("target,cap", [(64, 48), (32, 8)])
def test_big_cell_small_sort_cap_exact(B, orc, target, cap):
    """An LDS sort stage shorter than the expected bucket size: most buckets
    are ranked in global memory (the slow exact path, flagged), the others in
    LDS; pairs and state still equal the oracle's."""
    st = I.golovin_box(2 ** 15, seed=3)
    say(f"big-cell slow path target={target} cap={cap}")
    g = GpuRun(B, st, sink=True, tuning=dict(big_bucket_target=target, big_bucket_cap=cap,
                                             mid_max_slots=0))
    o = st.copy()
    cfg = ocfg(orc, o)
    for s in range(3):
        g.step(1)
        out = orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s, want_log=True)
        xi, v, _ = g.state()
        assert np.array_equal(xi, o.xi) and np.array_equal(v, o.v)
        assert np.array_equal(g.log(), out["log"])
    assert B.sdm_status_word(g.sim.handle) & B.SDM_FLAG_BUCKET_OVERFLOW
    g.close()


@pytest.mark.parametrize("adaptive", [False, True])
def test_sparse_big_cells_empty_buckets(B, orc, adaptive):
    """Big cells of up to 20000 slots with 98 % dead slots and 32-SD buckets:
    most buckets are empty, so the partner of a bucket's last entry sits
    several buckets on; with attributes, bit-exact against the oracle."""
    st = I.random_cells(12, 20000, n_attr=1, dead_fraction=0.98, rng_seed=41, p_boost=3e3)
    st.adaptive = adaptive
    say(f"sparse big cells adaptive={adaptive}")
    assert _compare_run(B, orc, st, 6, tuning=dict(mid_max_slots=0, big_bucket_target=32),
                        label=f"sparse-{adaptive}")


def test_big_cell_several_key_groups(B, orc):
    """A 2^19-SD cell: each key block takes several Philox groups per thread
    (counted, then recomputed and placed); bit-exact with the pair log."""
    st = I.golovin_box(2 ** 19, seed=5)
    say("golovin box 2^19")
    assert _compare_run(B, orc, st, 3, label="golovin-2^19")


def test_big_cell_maximum_size(B, orc):
    """A cell of the largest size a layout may have (8 388 608 SDs): 256 key
    blocks of 32 768 slots, 16 384 buckets of about 512 entries (none past
    the LDS stage); two steps bit-exact with the pair log, status clean, and
    the cell's moments (one workgroup over all its slots) against the
    oracle's: the int64 count exact, the sums within 2 ceil(log2 n) ulps."""
    n = 8388608
    st = I.golovin_box(n, seed=7)
    say("golovin box 2^23 (largest cell)")
    assert _compare_run(B, orc, st, 2, label="golovin-2^23")
    g = B.Sim(st)
    g.step(1)
    assert B.sdm_status_word(g.handle) == 0
    gm = g.moments()
    xi, v, at = g.state()
    g.close()
    om = orc.moments(ocfg(orc, st), xi, v, at, st.cell_off)
    assert np.array_equal(gm["m0"], om["m0"])
    bound = 2 * np.ceil(np.log2(n)) * 2.0 ** -53
    for k in ("m1", "m2"):
        assert rel_close(gm[k], om[k], bound), k


def test_big_golovin_box(B, orc):
    """One 2^17-SD cell (the big-cell path) for 20 steps, bit-exact."""
    st = I.golovin_box(2 ** 17)
    say("golovin box 2^17")
    assert _compare_run(B, orc, st, 20, every=5, label="golovin-2^17")


def _teacher_forced(B, orc, st, steps, label, max_frac=1e-6):
    g = GpuRun(B, st, sink=True)
    cfg = ocfg(orc, st)
    mism = tot = 0
    for s in range(steps):
        xi0, v0, a0 = g.state()
        o_xi, o_v, o_a = xi0.copy(), v0.copy(), np.ascontiguousarray(a0.copy())
        g.step(1)
        out = orc.step(cfg, o_xi, o_v, o_a, st.cell_off, s, want_log=True)
        glog = g.log()
        used = out["log"][:, 0] >= 0
        assert np.array_equal(glog[:, 0], out["log"][:, 0]), f"{label}: pairs differ at {s}"
        mism += int((glog[used, 1] != out["log"][used, 1]).sum())
        tot += int(used.sum())
    g.close()
    say(f"  {label}: gamma mismatches {mism} of {tot}")
    assert tot > 0
    assert mism <= max(max_frac * tot, 0), (mism, tot)
    return mism, tot


def test_geometric_teacher_forced_cells(B, orc):
    st = I.random_cells(48, 700, n_attr=2, kernel=I.GEOMETRIC, rng_seed=21, p_boost=1.0)
    _teacher_forced(B, orc, st, 30, "geometric random cells")


def test_geometric_grid_small(B, orc):
    st = I.grid(16, 16, 128, max_sd=200, n_attr=3, kernel=I.GEOMETRIC)
    _teacher_forced(B, orc, st, 20, "geometric 16x16 grid")


def test_geometric_big_box(B, orc):
    st = I.geometric_box(2 ** 17)
    _teacher_forced(B, orc, st, 4, "geometric box 2^17")


def test_geometric_spectrum_within_one_percent(B, orc):
    """Free runs of the geometric box (2^13 SDs, 1200 steps): the mass-density
    spectrum of GPU and oracle agree within 1 % (relative L1 over bins)."""
    st = I.geometric_box(2 ** 13)
    say("geometric box 2^13 spectrum, 1200 steps")
    g = GpuRun(B, st, sink=False)
    o = st.copy()
    cfg = ocfg(orc, o)
    for s in range(1200):
        orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s)
    g.step(1200)
    er = cf.radius_edges(1e-6, 5e-3, 48)
    ev = cf.volume_of_radius(er)
    gm = g.sim.moments(ev)
    om = orc.moments(cfg, o.xi, o.v, o.attrs, o.cell_off, ev)
    gs, os_ = gm["spectrum"].sum(0), om["spectrum"].sum(0)
    l1 = np.abs(gs - os_).sum() / os_.sum()
    xi, _, _ = g.state()
    say(f"  spectrum L1 {l1:.3e}; identical xi: {np.array_equal(xi, o.xi)}")
    assert l1 <= 0.01
    g.close()


def _golden_spectrum(path):
    out = {"bins": []}
    for line in open(path):
        if line.startswith("#"):
            continue
        k = line.split()
        if k[0] == "bin":
            out["bins"].append(float(k[2]))
        else:
            out[k[0]] = float(k[1]) if k[0] in ("m1", "m2") else int(k[1])
    out["bins"] = np.array(out["bins"])
    return out


def test_geometric_box_2p17_spectrum_3600_steps(B):
    """The geometric box at its stated size (2^17 SDs in one cell, the
    big-cell path), free-run for all 3600 steps: the mass spectrum at
    t = 3600 s is within 1 % (relative L1 over 48 bins) of the oracle's,
    which tests/golden/make_geometric_box_spectrum.py stored by running the
    oracle on the same input; the droplet count is compared too."""
    import os

    gold = _golden_spectrum(os.path.join(os.path.dirname(__file__), "golden",
                                         "geometric_box_2p17_3600s.txt"))
    st = I.geometric_box(2 ** 17)
    say("geometric box 2^17, 3600 steps (free run)")
    g = GpuRun(B, st, sink=False)
    g.step(3600)
    ev = cf.volume_of_radius(cf.radius_edges(1e-6, 5e-3, 48))
    gm = g.sim.moments(ev)
    xi, _, _ = g.state()
    gs = gm["spectrum"][0]
    l1 = np.abs(gs - gold["bins"]).sum() / gold["bins"].sum()
    say(f"  spectrum L1 {l1:.3e}; M0 {int(gm['m0'][0])} vs {gold['m0']}; "
        f"live {int((xi > 0).sum())} vs {gold['live']}")
    assert l1 <= 0.01
    assert abs(int(gm["m0"][0]) - gold["m0"]) <= 0.01 * gold["m0"]
    assert B.sdm_get_step(g.sim.handle) == 3600
    g.close()


def test_adaptive_golovin_bit_exact(B, orc):
    st = I.random_cells(30, 400, n_attr=2, rng_seed=31, p_boost=3e3)
    st.adaptive = True
    say("adaptive golovin random cells")
    assert _compare_run(B, orc, st, 8, label="adaptive-golovin")


@pytest.mark.parametrize("boost,uniform", [(300.0, False), (3e4, False), (0.0, True)])
def test_adaptive_attributes_many_collisions(B, orc, boost, uniform):
    """Attributes under adaptive substepping, bit-exact: cells of up to 500
    SDs with 3 attributes, from a few collisions per step to every pair of a
    cell colliding (and splitting) in each of many substeps."""
    st = I.random_cells(24, 500, n_attr=3, rng_seed=37, p_boost=max(boost, 1.0))
    if uniform:
        live = st.xi > 0
        st.xi[live] = 1000
        st.v[:] = float(np.mean(st.v))
        # every pair gets the same p: 5 in a 50-SD cell, 50 in a 500-SD cell
        st.b = 5.0 * st.dv / (1000 * 2 * st.v[0] * 49 * st.dt)
    st.adaptive = True
    say(f"adaptive attributes boost={boost} uniform={uniform}")
    assert _compare_run(B, orc, st, 4, label=f"adaptive-attrs-{boost}-{uniform}")


@pytest.mark.parametrize("mid_max", [16384, -1])
def test_plain_mid_and_big_routes(B, orc, mid_max):
    """Plain Golovin cells of up to 16384 slots: every mid-size class
    (mid_max_slots = 16384), or the automatic route (the default: with at
    most 32 such cells, those above 4096 slots on the big-cell path);
    bit-exact against the oracle, pair logs equal."""
    st = I.random_cells(24, 16384, n_attr=1, rng_seed=41, p_boost=1e3)
    tu = dict(mid_max_slots=mid_max)
    g = B.Sim(st)
    assert B.sdm_get_tuning(g.handle).mid_max_slots == -1
    g.close()
    say(f"plain mid-size and big routes, mid_max_slots={mid_max}")
    assert _compare_run(B, orc, st, 6, sink=True, tuning=tu, label=f"mid{mid_max}")


def test_adaptive_mid_cells_bit_exact(B, orc):
    """Adaptive substeps in the mid-size kernel (cells of 513..16384 slots)."""
    st = I.random_cells(12, 3000, n_attr=2, rng_seed=33, p_boost=1e3)
    st.adaptive = True
    say("adaptive golovin mid-size cells")
    assert _compare_run(B, orc, st, 6, label="adaptive-mid")


def test_adaptive_geometric_drizzle(B, orc):
    """The drizzle grid in adaptive mode: teacher-forced per step; substeps
    occur, gamma stays <= 1 and the status word is clean."""
    st = I.grid(16, 16, 256, n_attr=6, kernel=I.GEOMETRIC, drizzle=True, adaptive=True)
    g = GpuRun(B, st, sink=True)
    cfg = ocfg(orc, st)
    bad_cells = pair_substeps = 0
    for s in range(4):
        xi0, v0, a0 = g.state()
        o_xi, o_v, o_a = xi0.copy(), v0.copy(), np.ascontiguousarray(a0.copy())
        live = np.diff(np.concatenate([[0], np.cumsum(o_xi > 0)])[st.cell_off])
        g.step(1)
        out = orc.step(cfg, o_xi, o_v, o_a, st.cell_off, s, want_log=True, want_substeps=True)
        xi, v, at = g.state()
        assert g.log()[:, 1].max() <= 1
        for c in range(st.n_cells):
            sl = slice(st.cell_off[c], st.cell_off[c + 1])
            if not (np.array_equal(xi[sl], o_xi[sl]) and rel_close(v[sl], o_v[sl], 1e-12)
                    and rel_close(at[:, sl], o_a[:, sl], 1e-12)):
                bad_cells += 1
        pair_substeps += int((out["substeps"].astype(np.int64) * (live // 2)).sum())
        assert out["substeps"].max() > 1
    stats = B.sdm_stats(g.sim.handle)
    allowed = int(1e-6 * pair_substeps)
    say(f"  adaptive: differing cell-steps {bad_cells} of {pair_substeps} pair-substeps "
        f"(allowed {allowed}); stats {stats}")
    assert stats["cell_substeps"] > stats["cell_steps"]
    assert B.sdm_status_word(g.sim.handle) == 0
    # a differing cell-step means at least one differing gamma among its pairs
    assert bad_cells <= allowed
    g.close()


@pytest.mark.parametrize("case", ["box", "cells-big-path", "cells-overflow"])
def test_adaptive_big_cells_bit_exact(B, orc, case):
    """Adaptive substepping on the big-cell path (cells above the mid-size
    limit, or every cell above 512 slots with mid_max_slots = 0): the Golovin
    kernel with b raised so that cells take several substeps; state and the
    last substep's pairs and gammas equal the oracle's at every step."""
    if case == "box":
        st = I.golovin_box(2 ** 15, seed=7)
        st.b *= 3000.0
        tuning = None
    else:
        st = I.random_cells(16, 3000, n_attr=2, rng_seed=35, p_boost=1e3)
        tuning = dict(mid_max_slots=0)
        if case == "cells-overflow":
            tuning.update(big_bucket_target=64, big_bucket_cap=40)
    st.adaptive = True
    say(f"adaptive big cells: {case}")
    g = GpuRun(B, st, sink=True, tuning=tuning)
    o = st.copy()
    cfg = ocfg(orc, o)
    subs = 0
    for s in range(4):
        g.step(1)
        out = orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s, want_log=True, want_substeps=True)
        subs = max(subs, int(out["substeps"].max()))
        xi, v, at = g.state()
        assert np.array_equal(xi, o.xi), s
        assert np.array_equal(v, o.v) and np.array_equal(at, o.attrs), s
        assert np.array_equal(g.log(), out["log"]), s
    stats = B.sdm_stats(g.sim.handle)
    say(f"  most substeps in a step {subs}; stats {stats}")
    assert subs > 1 and stats["cell_substeps"] > stats["cell_steps"]
    g.close()


def test_adaptive_big_geometric_teacher_forced(B, orc):
    """The 2^17 geometric box in adaptive mode at dt = 30 s (so that it
    substeps): teacher-forced per step, differing steps within 1e-6 of the
    pair-substeps (last-bit cube-root differences)."""
    st = I.geometric_box(2 ** 17)
    st.adaptive = True
    st.dt = 30.0
    g = GpuRun(B, st, sink=True)
    cfg = ocfg(orc, st)
    bad = pair_substeps = 0
    for s in range(3):
        xi0, v0, a0 = g.state()
        o_xi, o_v, o_a = xi0.copy(), v0.copy(), np.ascontiguousarray(a0.copy())
        live = int((o_xi > 0).sum())
        g.step(1)
        out = orc.step(cfg, o_xi, o_v, o_a, st.cell_off, s, want_substeps=True)
        xi, v, _ = g.state()
        pair_substeps += int(out["substeps"][0]) * (live // 2)
        if not (np.array_equal(xi, o_xi) and rel_close(v, o_v, 1e-12)):
            bad += 1
        say(f"  step {s}: substeps {int(out['substeps'][0])}")
    allowed = int(1e-6 * pair_substeps)
    say(f"  differing steps {bad} of {pair_substeps} pair-substeps (allowed {allowed})")
    assert bad <= allowed
    assert B.sdm_stats(g.sim.handle)["cell_substeps"] > 3
    g.close()


def test_adaptive_big_substep_cap(B, orc):
    st = I.golovin_box(2 ** 15, seed=2)
    st.b *= 3000.0
    st.adaptive = True
    g = GpuRun(B, st, sink=False, max_substeps=1)
    o = st.copy()
    cfg = ocfg(orc, o, max_substeps=1)
    g.step(1)
    out = orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, 0)
    assert out["status"] & orc.ST_SUBSTEP_CAP
    assert B.sdm_status_word(g.sim.handle) & B.SDM_FLAG_SUBSTEP_CAP
    xi, v, _ = g.state()
    assert np.array_equal(xi, o.xi) and np.array_equal(v, o.v)
    g.close()


def test_substep_cap_flag(B, orc):
    st = I.grid(4, 4, 64, kernel=I.GEOMETRIC, drizzle=True, adaptive=True)
    g = GpuRun(B, st, sink=False, max_substeps=1)
    o = st.copy()
    cfg = ocfg(orc, o, max_substeps=1)
    g.step(1)
    out = orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, 0)
    assert out["status"] & orc.ST_SUBSTEP_CAP
    assert B.sdm_status_word(g.sim.handle) & B.SDM_FLAG_SUBSTEP_CAP
    g.close()


def test_gamma_cap_flag(B, orc):
    st = I.random_cells(4, 40, rng_seed=7, p_boost=1e40)
    say("gamma cap")
    assert _compare_run(B, orc, st, 2, label="gamma-cap")
    g = GpuRun(B, st)
    g.step(1)
    assert B.sdm_status_word(g.sim.handle) & B.SDM_FLAG_GAMMA_CAP
    g.close()


@pytest.mark.parametrize("case", ["wide", "narrow-1024-bins"])
def test_moments_parity(B, orc, case):
    """Moments and spectrum against the oracle: cells of up to 2000 slots (four
    waves per cell) with 40 bins covering every SD, and cells of up to 300
    slots (one wave per cell) with 1024 narrow bins that leave SDs outside."""
    if case == "wide":
        st = I.random_cells(50, 2000, n_attr=3, rng_seed=41)
        ev = cf.volume_of_radius(cf.radius_edges(1e-6, 5e-3, 40))
    else:
        st = I.random_cells(300, 300, n_attr=2, rng_seed=43)
        ev = cf.volume_of_radius(cf.radius_edges(8e-6, 14e-6, 1025))
    g = GpuRun(B, st, sink=False)
    g.step(5)
    xi, v, at = g.state()
    gm = g.sim.moments(ev)
    om = orc.moments(ocfg(orc, st), xi, v, np.ascontiguousarray(at), st.cell_off, ev)
    assert np.array_equal(gm["m0"], om["m0"])
    nmax = int(np.diff(st.cell_off).max())
    bound = 2 * np.ceil(np.log2(max(nmax, 2))) * 2.0 ** -53
    for k in ("m1", "m2", "attr_sums", "spectrum"):
        assert rel_close(gm[k], om[k], bound), k
    g.close()


def test_resume_equals_continuous(B, orc):
    import torch

    st = I.random_cells(20, 600, n_attr=1, rng_seed=51, p_boost=50.0)
    a = GpuRun(B, st)
    a.step(40)
    xa, va, aa = a.state()
    b = GpuRun(B, st)
    b.step(20)
    xb, vb, ab = b.state()
    b.close()
    c = GpuRun(B, st)
    c.set_state(xb, vb, ab)
    B.sdm_set_step(c.sim.handle, 20)
    c.step(20)
    xc, vc, ac = c.state()
    assert np.array_equal(xa, xc) and np.array_equal(va, vc) and np.array_equal(aa, ac)
    assert B.sdm_get_step(c.sim.handle) == 40
    a.close()
    c.close()
    torch.cuda.synchronize()


def test_repeat_runs_identical(B):
    st = I.grid(32, 32, 200, max_sd=500, n_attr=2, kernel=I.GEOMETRIC)
    outs = []
    for _ in range(2):
        g = GpuRun(B, st)
        g.step(10)
        outs.append(g.state())
        g.close()
    for x, y in zip(outs[0], outs[1]):
        assert np.array_equal(x, y)


def test_step_limit(B, orc):
    st = I.random_cells(10, 200, rng_seed=61, p_boost=100.0)
    g = GpuRun(B, st)
    B.sdm_set_step_limit(g.sim.handle, 3)
    g.step(10)
    assert B.sdm_get_step(g.sim.handle) == 3
    o = st.copy()
    cfg = ocfg(orc, o)
    for s in range(3):
        orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s)
    xi, v, _ = g.state()
    assert np.array_equal(xi, o.xi) and np.array_equal(v, o.v)
    g.close()


def test_batch_equals_separate(B, orc):
    """Shared launches over several simulations of different kernels, sizes,
    seeds and modes give each one exactly its solo result.  The batch has
    cells in the small and large workgroup-per-cell classes, mid-size cells
    and one big cell, so every group of launches runs, on both streams."""
    import torch

    states = [I.random_cells(12, 300, n_attr=2, rng_seed=71, p_boost=30.0),
              I.golovin_box(2 ** 12, seed=5),
              I.geometric_box(2 ** 11, seed=9),
              I.grid(8, 8, 128, max_sd=200, n_attr=3, kernel=I.GEOMETRIC, seed=3),
              I.golovin_box(2 ** 15, seed=13)]
    states[3].adaptive = True
    solo = []
    for st in states:
        g = GpuRun(B, st)
        g.step(7)
        solo.append(g.state())
        g.close()
    runs = [GpuRun(B, st) for st in states]
    handles = [r.sim.handle for r in runs]
    ws = B.workspace_tensor(B.sdm_batch_workspace_bytes(handles))
    b = B.sdm_batch_create(handles, ws)
    B.sdm_batch_step(b, 3)
    B.sdm_batch_step(b, 4)
    torch.cuda.synchronize()
    for r, ref in zip(runs, solo):
        assert B.sdm_get_step(r.sim.handle) == 7
        for x, y in zip(r.state(), ref):
            assert np.array_equal(x, y)
    B.sdm_batch_free(b)
    for r in runs:
        r.close()


@pytest.mark.parametrize("case", ["plain-golovin", "plain-geometric", "adaptive", "limit"])
def test_fused_steps_equal_single_steps(B, orc, case):
    """A multi-step call fuses up to 8 steps per launch with each cell kept
    in LDS; the result, the pair log of the last step and the statistics
    equal those of the same steps taken one call at a time (and, for the
    Golovin case, the oracle's)."""
    if case == "plain-golovin":
        st = I.random_cells(40, 500, n_attr=2, rng_seed=81, p_boost=30.0)
    elif case == "plain-geometric":
        st = I.grid(8, 8, 200, max_sd=380, n_attr=3, kernel=I.GEOMETRIC, seed=4)
    else:
        st = I.grid(8, 8, 200, max_sd=380, n_attr=3, kernel=I.GEOMETRIC, drizzle=True,
                    adaptive=True, seed=6)
    steps = 19  # fused launches of 8, 8 and 3 steps
    one = GpuRun(B, st, sink=True)
    many = GpuRun(B, st, sink=True)
    if case == "limit":  # the limit falls inside the second fused launch
        B.sdm_set_step_limit(one.sim.handle, 11)
        B.sdm_set_step_limit(many.sim.handle, 11)
    say(f"fused steps: {case}")
    for _ in range(steps):
        one.step(1)
    many.step(steps)
    for x, y in zip(one.state(), many.state()):
        assert np.array_equal(x, y)
    assert np.array_equal(one.log(), many.log())
    assert B.sdm_stats(one.sim.handle) == B.sdm_stats(many.sim.handle)
    assert B.sdm_get_step(one.sim.handle) == B.sdm_get_step(many.sim.handle)
    if case == "plain-golovin":
        o = st.copy()
        cfg = ocfg(orc, o)
        for s_ in range(steps):
            orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s_)
        xi, v, at = many.state()
        assert np.array_equal(xi, o.xi) and np.array_equal(v, o.v) and np.array_equal(at, o.attrs)
    one.sim.close()
    many.sim.close()


def test_invalid_inputs(B):
    import torch

    st = I.random_cells(5, 50, rng_seed=81)
    bad = st.copy()
    bad.xi[3] = -1
    with pytest.raises(B.SdmError) as e:
        B.Sim(bad)
    assert e.value.status == B.SDM_EINVAL
    bad = st.copy()
    live = np.nonzero(bad.xi > 0)[0][0]
    bad.v[live] = 0.0
    with pytest.raises(B.SdmError):
        B.Sim(bad)
    bad = st.copy()
    bad.cell_off[2] = bad.cell_off[3] + 1
    with pytest.raises(B.SdmError):
        B.Sim(bad)
    cfg = B.make_config(st.n_slots, st.n_cells)
    small = torch.empty(256, dtype=torch.uint8, device="cuda")
    xi = torch.from_numpy(st.xi).cuda()
    v = torch.from_numpy(st.v).cuda()
    off = torch.from_numpy(st.cell_off).cuda()
    with pytest.raises(B.SdmError) as e:
        B.sdm_init(cfg, xi, v, None, off, small)
    assert e.value.status == B.SDM_ENOMEM
    sim = B.Sim(st)  # more spectrum bins than sdm_moments takes
    edges = torch.linspace(1e-18, 1e-12, 1026, dtype=torch.float64, device="cuda")
    spec = torch.empty((st.n_cells, 1025), dtype=torch.float64, device="cuda")
    with pytest.raises(B.SdmError) as e:
        B.sdm_moments(sim.handle, vol_edges=edges, spectrum=spec)
    assert e.value.status == B.SDM_EINVAL
    sim.close()


def test_empty_and_tiny(B, orc):
    for st in [I.random_cells(3, 1, rng_seed=1), I.random_cells(6, 2, rng_seed=2)]:
        assert _compare_run(B, orc, st, 3, label="tiny")
    st = I.State(np.zeros(0, dtype=np.int64), np.zeros(0), np.zeros((0, 0)),
                 np.zeros(5, dtype=np.int64))
    g = B.Sim(st)
    g.step(3)
    assert B.sdm_get_step(g.handle) == 3
    g.close()


def test_autotune_keeps_results_and_caches(B, orc, tmp_path, monkeypatch):
    """The autotuner times shapes on a scratch copy: the handle's state and
    counter are untouched, results after tuning still match the oracle, and
    a second handle with the same key reuses the cached choice, named by the
    call or, with no path passed, by SDM_TUNE_CACHE."""
    st = I.random_cells(64, 900, n_attr=1, rng_seed=91, p_boost=30.0)
    g = GpuRun(B, st)
    scratch = B.workspace_tensor(B.sdm_autotune_scratch_bytes(g.sim.handle))
    cache = str(tmp_path / "tune.jsonl")
    say("autotune random cells")
    t1 = B.sdm_autotune(g.sim.handle, scratch, trial_steps=2, cache_path=cache).as_dict()
    say(f"  chosen {t1}")
    xi, v, _ = g.state()
    assert np.array_equal(xi, st.xi) and np.array_equal(v, st.v)
    assert B.sdm_get_step(g.sim.handle) == 0
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == 1 and '"key"' in lines[0]
    o = st.copy()
    cfg = ocfg(orc, o)
    for s in range(4):
        g.step(1)
        orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s)
    xi, v, at = g.state()
    assert np.array_equal(xi, o.xi) and np.array_equal(v, o.v) and np.array_equal(at, o.attrs)
    g.close()
    g2 = GpuRun(B, st)
    t2 = B.sdm_autotune(g2.sim.handle, None, trial_steps=2, cache_path=cache).as_dict()
    assert t2 == t1
    assert len(open(cache).read().strip().splitlines()) == 1
    g2.close()
    monkeypatch.setenv("SDM_TUNE_CACHE", cache)
    g3 = GpuRun(B, st)
    t3 = B.sdm_autotune(g3.sim.handle, None, trial_steps=2).as_dict()  # no scratch: a cache hit
    assert t3 == t1
    assert len(open(cache).read().strip().splitlines()) == 1
    g3.close()


def test_large_batch_many_members(B, orc):
    """512 simulations in one batch (one cell each, 2..600 SDs: every
    workgroup-per-cell class and the smallest mid-size class), plain and
    adaptive, each with its own seed, a third of them with a step limit
    inside the run: every member equals its own oracle run bit for bit and
    its step counter stops at its limit."""
    import torch

    rng = np.random.default_rng(5)
    states, limits = [], []
    for i in range(512):
        st = I.golovin_box(int(rng.integers(2, 601)), seed=1000 + i)
        st.adaptive = bool(i % 2)
        states.append(st)
        limits.append(int(rng.integers(1, 6)) if i % 3 == 0 else None)
    say("batch of 512 simulations")
    runs = [GpuRun(B, st) for st in states]
    for r, lim in zip(runs, limits):
        if lim is not None:
            B.sdm_set_step_limit(r.sim.handle, lim)
    handles = [r.sim.handle for r in runs]
    ws = B.workspace_tensor(B.sdm_batch_workspace_bytes(handles))
    b = B.sdm_batch_create(handles, ws)
    B.sdm_batch_step(b, 2)
    B.sdm_batch_step(b, 4)
    torch.cuda.synchronize()
    for r, st, lim in zip(runs, states, limits):
        steps = 6 if lim is None else min(6, lim)
        o = st.copy()
        cfg = ocfg(orc, o)
        for s in range(steps):
            orc.step(cfg, o.xi, o.v, o.attrs, o.cell_off, s)
        xi, v, _ = r.state()
        assert B.sdm_get_step(r.sim.handle) == steps
        assert np.array_equal(xi, o.xi) and np.array_equal(v, o.v), (st.n_slots, st.adaptive)
    B.sdm_batch_free(b)
    for r in runs:
        r.close()


def _sub_state(st, cells):
    """Only the given cells keep their slots (cell indices unchanged)."""
    counts = np.diff(st.cell_off)
    keep = np.zeros(st.n_cells, dtype=bool)
    keep[cells] = True
    off = np.zeros(st.n_cells + 1, dtype=np.int64)
    np.cumsum(np.where(keep, counts, 0), out=off[1:])
    idx = np.concatenate([np.arange(st.cell_off[c], st.cell_off[c + 1]) for c in sorted(cells)])
    return idx, off


@pytest.fixture(scope="module")
def grid256():
    return I.grid_256x256()


def _gather(g, idx_t):
    """The GPU state of the sampled slots (device gather, then one copy)."""
    import torch

    torch.cuda.synchronize()
    xi = g.sim.xi.index_select(0, idx_t).cpu().numpy()
    v = g.sim.v.index_select(0, idx_t).cpu().numpy()
    at = g.sim.attrs.index_select(1, idx_t).cpu().numpy()
    return xi, v, np.ascontiguousarray(at)


@pytest.mark.parametrize("mask,kernel", [(0x10, I.GEOMETRIC), (0x1C, I.GEOMETRIC),
                                         (0x1C, I.GOLOVIN)])
def test_full_grid256_teacher_forced(B, orc, grid256, mask, kernel):
    """The benchmark's workload at full size (256 x 256 cells, 16.8 M SDs,
    adaptive, 6 attributes) in the benchmark's launch shapes (one class, or
    the 256/384/512-slot classes on two streams), six single-step calls, so
    that both dispatch-order lists of the adaptive cells are read.  Before
    every step the oracle takes the GPU's state of 2000 sampled cells and
    advances them one step; each sampled cell must then equal the GPU's.  A
    cell differs only if some gamma of one of its substeps differed, so the
    count of differing cell-steps bounds the gamma mismatches from below and
    must stay within 1e-6 of the pair-substeps (geometric kernel, where a
    last-bit cube-root difference could flip a gamma); with the Golovin kernel
    (b raised tenfold so that drizzle cells substep) it must be zero."""
    import torch

    st = grid256.copy()
    st.kernel = kernel
    if kernel == I.GOLOVIN:
        st.b = 1.5e4
    say(f"full 256x256 grid: {st.n_slots} slots, kernel {kernel}, class mask {mask:#x}")
    g = GpuRun(B, st, tuning=dict(wave_class_mask=mask, waves_per_cell=1))
    rng = np.random.default_rng(5)
    counts = np.diff(st.cell_off)
    cells = set(rng.choice(st.n_cells, size=2000, replace=False).tolist())
    cells |= {int(np.argmax(counts)), int(np.argmin(counts)), 0, st.n_cells - 1}
    cells = sorted(cells)
    idx, off = _sub_state(st, cells)
    idx_t = torch.from_numpy(idx).cuda()
    cfg = orc.OracleConfig(n_slots=len(idx), n_cells=st.n_cells, n_attr=st.n_attr, dt=st.dt,
                           dv=st.dv, b=st.b, kernel=st.kernel, adaptive=True, seed=st.seed)
    bad = pair_substeps = multi = 0
    for s in range(6):
        o_xi, o_v, o_a = _gather(g, idx_t)
        live = np.diff(np.concatenate([[0], np.cumsum(o_xi > 0)])[off])
        g.step(1)
        xi, v, at = _gather(g, idx_t)
        out = orc.step(cfg, o_xi, o_v, o_a, off, s, want_substeps=True)
        sub = out["substeps"]
        for c in cells:
            os_ = slice(off[c], off[c + 1])
            same = (np.array_equal(xi[os_], o_xi[os_]) and rel_close(v[os_], o_v[os_], 1e-12)
                    and rel_close(at[:, os_], o_a[:, os_], 1e-12))
            bad += 0 if same else 1
            pair_substeps += int(sub[c]) * int(live[c] // 2)
            multi += int(sub[c] > 1)
    allowed = 0 if kernel == I.GOLOVIN else int(1e-6 * pair_substeps)
    say(f"  {len(cells)} cells x 6 steps: {multi} cell-steps with substeps, "
        f"{pair_substeps} pair-substeps, differing cell-steps {bad} (allowed {allowed})")
    assert multi > 0
    assert bad <= allowed
    assert B.sdm_status_word(g.sim.handle) == 0
    g.close()


def test_full_grid64_teacher_forced(B, orc):
    """The 64 x 64 grid at full size (min(Poisson(128), 200) SDs, 3 attributes)."""
    st = I.grid_64x64()
    _teacher_forced(B, orc, st, 5, "geometric 64x64 grid (full size)")
