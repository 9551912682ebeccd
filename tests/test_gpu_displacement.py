"""GPU parity of displacement + re-segmentation (sdm_displace through the C
ABI) against the CPU oracle: every output bit-exact (the same fp64 operations
in the same order decide the new cells, and the slot order is an integer
result), plus the coupling with the coalescence step through sdm_rebind."""
import numpy as np
import pytest

from oracle import displacement as D
from paper_2103_17238_amd import inputs as I

from sdm_testutil import ocfg, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2103_17238_amd import binding

    return binding


def _cells(nx, nz, counts, n_attr, seed):
    rng = np.random.default_rng(seed)
    off = np.zeros(nx * nz + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    xi = rng.integers(0, 10 ** 9, size=n).astype(np.int64)
    v = rng.random(n)
    attrs = rng.random((n_attr, n))
    return xi, v, attrs, off


def _run(B, nx, nz, cx, cz, xi, v, attrs, pos, off):
    """One sdm_displace call on device copies; returns host outputs + flags."""
    import torch

    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    n = xi.size
    A = attrs.shape[0]
    ins = [d(xi), d(v), d(attrs) if A else None, d(pos), d(off)]
    outs = [torch.full((n,), -5, dtype=torch.int64, device="cuda"),
            torch.full((n,), -5.0, dtype=torch.float64, device="cuda"),
            torch.full((A, n), -5.0, dtype=torch.float64, device="cuda") if A else None,
            torch.full((2, n), -5.0, dtype=torch.float64, device="cuda"),
            torch.full((nx * nz + 1,), -5, dtype=torch.int64, device="cuda")]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = B.workspace_tensor(B.sdm_displace_workspace_bytes(nx, nz))
    B.sdm_displace(nx, nz, d(cx), d(cz), *ins, *outs, status, ws)
    torch.cuda.synchronize()
    h = [o.cpu().numpy() if o is not None else np.zeros((0, n)) for o in outs]
    return h, int(status.item()) & 0xFFFFFFFF


def _check(B, nx, nz, cx, cz, xi, v, attrs, pos, off, want_flags=0):
    got, fl = _run(B, nx, nz, cx, cz, xi, v, attrs, pos, off)
    ref = D.displace_resegment(nx, nz, cx, cz, xi, v, attrs, pos, off)
    assert fl == want_flags
    for g, r, nm in zip(got, ref[:5], ("xi", "v", "attrs", "pos", "cell_off")):
        assert np.array_equal(g, r), nm
    assert ref[5] == (D.ST_COURANT if want_flags else 0)
    return got


@pytest.mark.parametrize("nx,nz,max_sd,A,seed", [(5, 7, 70, 3, 0), (3, 3, 200, 0, 1),
                                                 (17, 4, 300, 6, 2), (40, 33, 9, 1, 3),
                                                 (9, 5, 600, 11, 4), (6, 6, 40, 16, 5)])
def test_random_flow_parity(B, nx, nz, max_sd, A, seed):
    """Random face Courant numbers in (-0.9, 0.9): every direction and the
    periodic wrap; uneven cells (empty ones, several 64-slot chunks)."""
    say(f"displace random nx={nx} nz={nz} max_sd={max_sd} A={A}")
    rng = np.random.default_rng(seed)
    counts = rng.integers(0, max_sd + 1, size=nx * nz)
    counts[0] = 0
    counts[-1] = max_sd
    xi, v, attrs, off = _cells(nx, nz, counts, A, seed)
    pos = I.positions(xi.size, seed=seed + 10)
    cx, cz = I.random_courant(nx, nz, 0.9, seed=seed + 20)
    got = _check(B, nx, nz, cx, cz, xi, v, attrs, pos, off)
    assert np.diff(got[4]).min() >= 0


@pytest.mark.parametrize("nx,nz", [(1, 7), (2, 5), (4, 1), (2, 2), (1, 1), (1, 40)])
def test_narrow_axes_parity(B, nx, nz):
    """Axes of one or two cells (a 1D column is nx = 1): random flows that
    move droplets both ways along every axis."""
    say(f"displace narrow nx={nx} nz={nz}")
    rng = np.random.default_rng(nx * 100 + nz)
    counts = rng.integers(0, 150, size=nx * nz)
    xi, v, attrs, off = _cells(nx, nz, counts, 2, nx + nz)
    pos = I.positions(xi.size, seed=nx + 3 * nz)
    cx, cz = I.random_courant(nx, nz, 0.9, seed=nx + 5 * nz)
    _check(B, nx, nz, cx, cz, xi, v, attrs, pos, off)


def test_zero_flow_and_empty(B):
    nx, nz = 4, 5
    say("displace zero flow")
    xi, v, attrs, off = _cells(nx, nz, np.arange(nx * nz) % 5, 2, 4)
    pos = I.positions(xi.size, seed=5)
    cx, cz = I.uniform_courant(nx, nz, 0.0, 0.0)
    got = _check(B, nx, nz, cx, cz, xi, v, attrs, pos, off)
    assert np.array_equal(got[0], xi) and np.array_equal(got[4], off)
    say("displace no droplets")
    xi, v, attrs, off = _cells(nx, nz, np.zeros(nx * nz, dtype=int), 0, 4)
    _check(B, nx, nz, cx, cz, xi, v, attrs, np.zeros((2, 0)), off)


def test_face_rounding_cases(B):
    """Droplets on and next to faces, fractions that round to 1."""
    nx, nz = 3, 4
    say("displace face rounding")
    counts = np.full(nx * nz, 6)
    xi, v, attrs, off = _cells(nx, nz, counts, 1, 6)
    n = xi.size
    w = np.array([0.0, 2.0 ** -60, 0.5, 1.0 - 2.0 ** -53, 0.25, 0.75])
    pos = np.stack([np.tile(w, n // 6), np.tile(w[::-1], n // 6)])
    cx, cz = I.uniform_courant(nx, nz, -2.0 ** -59, 2.0 ** -54)
    _check(B, nx, nz, cx, cz, xi, v, attrs, pos, off)
    cx, cz = I.uniform_courant(nx, nz, 0.5, -0.75)
    _check(B, nx, nz, cx, cz, xi, v, attrs, pos, off)


def test_courant_violation_flag(B):
    nx, nz = 5, 3
    say("displace Courant violation")
    xi, v, attrs, off = _cells(nx, nz, np.full(nx * nz, 10), 2, 7)
    pos = I.positions(xi.size, seed=8)
    cx, cz = I.uniform_courant(nx, nz, 1.5, 0.2)
    _check(B, nx, nz, cx, cz, xi, v, attrs, pos, off, want_flags=B.SDM_FLAG_COURANT)


def test_invalid_offsets_leave_outputs(B):
    nx, nz = 3, 3
    say("displace invalid offsets")
    xi, v, attrs, off = _cells(nx, nz, np.full(nx * nz, 4), 0, 9)
    bad = off.copy()
    bad[4] = bad[5] + 1  # decreasing
    pos = I.positions(xi.size, seed=9)
    cx, cz = I.uniform_courant(nx, nz, 0.1, 0.1)
    got, fl = _run(B, nx, nz, cx, cz, xi, v, attrs, pos, bad)
    assert fl & B.SDM_FLAG_INVALID_STATE
    assert np.all(got[0] == -5) and np.all(got[4] == -5)


def test_grid256_single_eddy_parity(B):
    """The 256 x 256 grid (16.8 M slots, 6 attributes) in the single-eddy
    flow, two steps, whole arrays compared."""
    import torch

    st = I.grid_256x256()
    nx = nz = 256
    cx, cz = I.single_eddy_courant(nx, nz)
    pos = I.positions(st.n_slots)
    say("displace grid256 single eddy, 2 steps")
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    cur = [d(st.xi), d(st.v), d(st.attrs), d(pos), d(st.cell_off)]
    nxt = [torch.empty_like(t) for t in cur]
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = B.workspace_tensor(B.sdm_displace_workspace_bytes(nx, nz))
    dcx, dcz = d(cx), d(cz)
    ref = (st.xi, st.v, st.attrs, pos, st.cell_off)
    for k in range(2):
        B.sdm_displace(nx, nz, dcx, dcz, *cur, *nxt, status, ws)
        cur, nxt = nxt, cur
        ref = D.displace_resegment(nx, nz, cx, cz, *ref[:5])
        assert ref[5] == 0
        torch.cuda.synchronize()
        for g, r, nm in zip(cur, ref[:5], ("xi", "v", "attrs", "pos", "cell_off")):
            assert np.array_equal(g.cpu().numpy(), r), (k, nm)
    assert int(status.item()) == 0
    moved = np.abs(np.diff(ref[4]) - np.diff(st.cell_off)).sum()
    assert moved > 0


@pytest.mark.parametrize("adaptive", [False, True])
def test_coupled_with_coalescence(B, orc, adaptive):
    """Displacement, re-plan (sdm_rebind) and a coalescence step, three
    times, against the oracle's displacement and step (Golovin kernel: the
    coalescence is bit-exact too)."""
    nx, nz = 12, 9
    say(f"coupled displacement + coalescence adaptive={adaptive}")
    st = I.grid(nx, nz, 60, n_attr=2, kernel=I.GOLOVIN, adaptive=adaptive)
    if adaptive:
        st.b *= 40.0
    cx, cz = I.random_courant(nx, nz, 0.8, seed=11)
    pos = I.positions(st.n_slots, seed=12)
    sim = B.Sim(st, any_layout=True)
    kin = B.Kinematic2D(sim, nx, nz, cx, cz, pos)
    cfg = ocfg(orc, st)
    xi, v, at, off, p = st.xi.copy(), st.v.copy(), st.attrs.copy(), st.cell_off.copy(), pos
    for k in range(3):
        kin.step()
        sim.step(1)
        xi, v, at, p, off, fl = D.displace_resegment(nx, nz, cx, cz, xi, v, at, p, off)
        xi, v, at = xi.copy(), v.copy(), np.ascontiguousarray(at)
        orc.step(cfg, xi, v, at, off, k)
        gx, gv, ga = sim.state()
        assert np.array_equal(gx, xi), k
        assert np.array_equal(gv, v), k
        assert np.array_equal(ga, at), k
        assert np.array_equal(sim.cell_off.cpu().numpy(), off), k
        assert np.array_equal(kin.pos.cpu().numpy(), p), k
    assert kin.flags() == 0
    st2 = B.sdm_stats(sim.handle)
    assert st2["colliding_pairs"] > 0
    # moments follow the current layout
    gm = sim.moments()
    om = orc.moments(cfg, xi, v, at, off)
    assert np.array_equal(gm["m0"], om["m0"])
    assert np.allclose(gm["m1"], om["m1"], rtol=1e-12, atol=0)
    sim.close()


@pytest.mark.parametrize("mask,empty", [(0x10, False), (0x01, False), (0x1F, True)])
def test_rebind_paths(B, orc, mask, empty):
    """The re-plan after displacement: 0x10 (every cell in the 512-slot
    class) always takes the device-side refresh; 0x01 (64-slot class first)
    makes cells outgrow their class, and empty cells that receive droplets
    have no task: both fall back to the host re-plan.  A host re-plan
    (sdm_set_tuning) and the gamma sink after device-side rebinds must see
    the current layout.  Everything against the oracle, bit for bit."""
    import torch

    nx, nz = 10, 8
    say(f"rebind paths mask={mask:#x} empty={empty}")
    if empty:
        st = I.random_cells(nx * nz, 90, n_attr=1, rng_seed=21)
    else:
        st = I.grid(nx, nz, 60, n_attr=1, kernel=I.GOLOVIN, seed=3)
    cx, cz = I.random_courant(nx, nz, 0.85, seed=31)
    pos = I.positions(st.n_slots, seed=32)
    sim = B.Sim(st, any_layout=True)
    t = B.sdm_get_tuning(sim.handle)
    t.wave_class_mask = mask
    B.sdm_set_tuning(sim.handle, t)
    kin = B.Kinematic2D(sim, nx, nz, cx, cz, pos)
    cfg = ocfg(orc, st)
    xi, v, at, off, p = st.xi.copy(), st.v.copy(), st.attrs.copy(), st.cell_off.copy(), pos
    for k in range(4):
        kin.step()
        xi, v, at, p, off, fl = D.displace_resegment(nx, nz, cx, cz, xi, v, at, p, off)
        xi, v, at = xi.copy(), v.copy(), np.ascontiguousarray(at)
        if k == 2:  # a host re-plan on the current layout
            t.waves_per_cell = 2
            B.sdm_set_tuning(sim.handle, t)
        want_log = k == 3
        if want_log:
            npairs = int((np.diff(off) // 2).sum())
            sink = torch.full((2 * npairs,), -7, dtype=torch.int64, device="cuda")
            B.sdm_debug_gamma_sink(sim.handle, sink)
        sim.step(1)
        out = orc.step(cfg, xi, v, at, off, k, want_log=want_log)
        gx, gv, ga = sim.state()
        assert np.array_equal(gx, xi) and np.array_equal(gv, v) and np.array_equal(ga, at), k
        if want_log:
            torch.cuda.synchronize()
            assert np.array_equal(sink.cpu().numpy().reshape(-1, 2), out["log"])
    assert kin.flags() == 0
    sim.close()


def test_batch_refuses_after_rebind(B):
    """A batch made before a member's rebind refuses to step (its tables
    point at the old buffers); a batch made afterwards steps."""
    import torch

    nx, nz = 5, 4
    st = I.grid(nx, nz, 30, kernel=I.GOLOVIN)
    sims = [B.Sim(st, any_layout=True), B.Sim(st, any_layout=True)]
    handles = [s.handle for s in sims]
    ws = B.workspace_tensor(B.sdm_batch_workspace_bytes(handles))
    batch = B.sdm_batch_create(handles, ws)
    B.sdm_batch_step(batch, 1)
    cx, cz = I.random_courant(nx, nz, 0.8, seed=41)
    kin = B.Kinematic2D(sims[0], nx, nz, cx, cz, I.positions(st.n_slots, seed=42))
    kin.step()
    with pytest.raises(B.SdmError):
        B.sdm_batch_step(batch, 1)
    B.sdm_batch_free(batch)
    ws2 = B.workspace_tensor(B.sdm_batch_workspace_bytes(handles))
    batch2 = B.sdm_batch_create(handles, ws2)
    B.sdm_batch_step(batch2, 1)
    torch.cuda.synchronize()
    B.sdm_batch_free(batch2)
    for s in sims:
        s.close()


def test_rebind_rejects_bad_layout(B):
    import torch

    st = I.grid(4, 4, 20, kernel=I.GOLOVIN)
    sim = B.Sim(st, any_layout=True)
    bad = st.cell_off.copy()
    bad[-1] += 1
    with pytest.raises(B.SdmError):
        B.sdm_rebind(sim.handle, sim.xi, sim.v, sim.attrs, torch.from_numpy(bad).cuda())
    sim.step(1)  # the handle still works on its old layout
    torch.cuda.synchronize()
    sim.close()
