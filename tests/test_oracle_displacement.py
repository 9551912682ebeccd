"""Pins of the displacement / re-segmentation oracle against facts fixed
independently of its code: a hand-worked example in dyadic numbers (exact in
fp64), the identity of a zero flow, the closed form of a uniform flow, a
brute-force re-segmentation, conservation, the Courant flag and the
divergence-free input flow."""
import numpy as np
import pytest

from oracle import displacement as D
from paper_2103_17238_amd import inputs as I


def _state(counts, n_attr=0, seed=0):
    rng = np.random.default_rng(seed)
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    xi = rng.integers(0, 1000, size=n).astype(np.int64)
    v = rng.random(n) + np.arange(n)  # unique: identifies a droplet
    attrs = rng.random((n_attr, n))
    return xi, v, attrs, off


def test_hand_worked_example():
    """3 x 3 cells, six droplets, Courant numbers and positions chosen so that
    every product and sum is exact; expected values worked out by hand from
    d = (1 - w) c_low + w c_high, w' = w + d, shift floor(w'), periodic."""
    nx = nz = 3
    cx = np.zeros((4, 3))
    cz = np.zeros((3, 4))
    cx[0, 0], cx[1, 0], cx[2, 0], cx[3, 0] = 0.25, 0.5, 0.5, 0.25
    cx[2, 2], cx[3, 2], cx[0, 2] = 0.5, 0.5, 0.5
    cz[0, 0], cz[0, 3] = -0.5, -0.5
    cz[2, 0] = 0.25
    cz[2, 2], cz[2, 3] = 0.25, 0.25
    cz[1, 2] = -2.0 ** -59
    # slots: cell 0: A, C; cell 4: D; cell 5: G; cell 6: F; cell 8: B
    off = np.array([0, 2, 2, 2, 2, 3, 4, 5, 5, 6], dtype=np.int64)
    pos = np.array([[0.75, 0.25, 0.5, 0.5, 0.75, 0.5],
                    [0.5, 0.25, 0.5, 2.0 ** -60, 0.5, 0.875]])
    names = np.array(list("ACDGFB"))
    # A: x 0.75 + (0.25*0.25 + 0.75*0.5) = 1.1875 -> cell x 1, 0.1875;
    #    z 0.5 + (0.5*-0.5 + 0.5*0) = 0.25 -> cell (1, 0) = 3
    # C: x 0.25 + 0.3125 = 0.5625; z 0.25 - 0.375 = -0.125 -> 0.875, z 2 -> cell 2
    # D: no x flow; z 0.5 + 0.5 * -2^-59 rounds to 0.5 -> stays in cell 4
    # G: x 0.5 + 0.5*0.5 = 0.75; z 2^-60 - 2^-59 = -2^-60, fraction
    #    1 - 2^-60 rounds to 1 -> 0 in the same cell 5
    # F: x 0.75 + (0.25*0.5 + 0.75*0.25) = 1.0625 -> x wraps to 0, 0.0625;
    #    z 0.5 + 0.5*0.25 = 0.625 -> cell (0, 0) = 0
    # B: x 0.5 + 0.5 = 1.0 -> x wraps to 0, 0.0; z 0.875 + 0.25 = 1.125 ->
    #    z wraps to 0, 0.125 -> cell 0
    new_pos, new_cell, flags = D.displace(nx, nz, cx, cz, pos, off)
    assert flags == 0
    assert dict(zip(names, new_cell.tolist())) == {"A": 3, "C": 2, "D": 4, "G": 5, "F": 0, "B": 0}
    want = {"A": (0.1875, 0.25), "C": (0.5625, 0.875), "D": (0.5, 0.5), "G": (0.75, 0.0),
            "F": (0.0625, 0.625), "B": (0.0, 0.125)}
    for k, nm in enumerate(names):
        assert (new_pos[0, k], new_pos[1, k]) == want[nm], nm
    xi = np.arange(6, dtype=np.int64)
    out = D.displace_resegment(nx, nz, cx, cz, xi, xi * 1.0, np.zeros((0, 6)), pos, off)
    # new cell 0 holds F (old cell 6) before B (old cell 8), then C, A, D, G
    assert "".join(names[out[0]]) == "FBCADG"
    assert out[4].tolist() == [0, 2, 2, 3, 4, 5, 6, 6, 6, 6]


def test_zero_flow_is_identity():
    nx, nz = 5, 4
    xi, v, attrs, off = _state(np.random.default_rng(1).integers(0, 9, size=nx * nz), 2)
    pos = I.positions(xi.size, seed=7)
    cx, cz = I.uniform_courant(nx, nz, 0.0, 0.0)
    x2, v2, a2, p2, o2, fl = D.displace_resegment(nx, nz, cx, cz, xi, v, attrs, pos, off)
    assert fl == 0
    assert np.array_equal(x2, xi) and np.array_equal(v2, v) and np.array_equal(a2, attrs)
    assert np.array_equal(p2, pos) and np.array_equal(o2, off)


@pytest.mark.parametrize("ux,uz", [(0.3, -0.45), (-0.9, 0.7), (0.05, 0.0)])
def test_uniform_flow_closed_form(ux, uz):
    """Uniform Courant numbers: every droplet moves by exactly (ux, uz) cells
    (up to rounding) in the periodic domain."""
    nx, nz = 6, 5
    counts = np.random.default_rng(2).integers(0, 7, size=nx * nz)
    xi, v, attrs, off = _state(counts)
    rng = np.random.default_rng(3)
    pos = rng.uniform(0.01, 0.99, size=(2, xi.size))
    # keep away from faces so that rounding cannot decide the cell
    for w, u in ((pos[0], ux), (pos[1], uz)):
        f = (w + u) % 1.0
        near = (f < 1e-6) | (f > 1 - 1e-6)
        w[near] += 0.003
    cx, cz = I.uniform_courant(nx, nz, ux, uz)
    new_pos, new_cell, fl = D.displace(nx, nz, cx, cz, pos, off)
    assert fl == 0
    c = np.repeat(np.arange(nx * nz), counts)
    ax = (c // nz + pos[0] + ux) % nx
    az = (c % nz + pos[1] + uz) % nz
    assert np.array_equal(new_cell, np.floor(ax).astype(int) * nz + np.floor(az).astype(int))
    assert np.allclose(new_pos[0], ax - np.floor(ax), atol=1e-12, rtol=0)
    assert np.allclose(new_pos[1], az - np.floor(az), atol=1e-12, rtol=0)


def test_resegment_matches_brute_force():
    """Stable order by new cell, against a loop that visits new cells in
    order and collects the old slots that land there."""
    rng = np.random.default_rng(4)
    n, C = 300, 23
    new_cell = rng.integers(0, C, size=n)
    order, off = D.resegment(new_cell, C)
    brute, boff = [], [0]
    for c in range(C):
        for j in range(n):
            if new_cell[j] == c:
                brute.append(j)
        boff.append(len(brute))
    assert order.tolist() == brute
    assert off.tolist() == boff


def test_conservation_and_layout():
    nx, nz = 7, 9
    counts = np.random.default_rng(5).integers(0, 40, size=nx * nz)
    counts[3] = 0
    xi, v, attrs, off = _state(counts, 3, seed=5)
    pos = I.positions(xi.size, seed=8)
    cx, cz = I.random_courant(nx, nz, amp=0.9, seed=9)
    x2, v2, a2, p2, o2, fl = D.displace_resegment(nx, nz, cx, cz, xi, v, attrs, pos, off)
    assert fl == 0
    assert o2[0] == 0 and o2[-1] == xi.size and np.all(np.diff(o2) >= 0)
    perm = np.argsort(v)  # v identifies droplets
    perm2 = np.argsort(v2)
    assert np.array_equal(v[perm], v2[perm2])
    assert np.array_equal(xi[perm], x2[perm2])
    assert np.array_equal(attrs[:, perm], a2[:, perm2])
    assert xi.sum() == x2.sum()
    assert np.all((p2 >= 0.0) & (p2 < 1.0))
    # droplets moved at most one cell per axis (periodic distance)
    c_old = np.repeat(np.arange(nx * nz), counts)[perm]
    c_new = np.repeat(np.arange(nx * nz), np.diff(o2))[perm2]
    dx = (c_new // nz - c_old // nz) % nx
    dz = (c_new % nz - c_old % nz) % nz
    assert np.all(np.isin(dx, [0, 1, nx - 1])) and np.all(np.isin(dz, [0, 1, nz - 1]))
    assert len(np.unique(c_new - c_old)) > 5  # several directions exercised


def test_courant_flag():
    nx, nz = 4, 4
    xi, v, attrs, off = _state(np.full(nx * nz, 3))
    pos = np.full((2, xi.size), 0.5)
    cx, cz = I.uniform_courant(nx, nz, 0.999, -0.999)
    assert D.displace(nx, nz, cx, cz, pos, off)[2] == 0
    cx, cz = I.uniform_courant(nx, nz, 1.0, 0.0)
    assert D.displace(nx, nz, cx, cz, pos, off)[2] == D.ST_COURANT
    cx, cz = I.uniform_courant(nx, nz, 0.0, -1.5)
    new_pos, new_cell, fl = D.displace(nx, nz, cx, cz, pos, off)
    assert fl == D.ST_COURANT
    c = np.repeat(np.arange(nx * nz), 3)
    assert np.all((new_cell // nz - c // nz) % nx == 0)  # clamped to one cell


def test_single_eddy_input_is_divergence_free():
    cx, cz = I.single_eddy_courant(32, 24)
    div = (cx[1:, :] - cx[:-1, :]) + (cz[:, 1:] - cz[:, :-1])
    assert np.abs(div).max() < 1e-15
    assert np.all(cz[:, 0] == 0.0) and np.all(cz[:, -1] == 0.0)
    assert np.array_equal(cx[0], cx[-1])


def test_position_out_of_range_flags():
    nx, nz = 3, 3
    xi, v, attrs, off = _state(np.full(nx * nz, 2))
    pos = np.full((2, xi.size), 0.5)
    pos[1, 4] = 1.0
    cx, cz = I.uniform_courant(nx, nz, 0.0, 0.0)
    assert D.displace(nx, nz, cx, cz, pos, off)[2] == D.ST_COURANT


@pytest.mark.parametrize("nx,nz", [(1, 7), (2, 5), (4, 1), (2, 2), (1, 1)])
def test_narrow_axes(nx, nz):
    """Axes of one or two cells: every droplet lands in the cell the periodic
    domain puts it in (closed form of a uniform flow), and the slot order is
    the stable order by new cell (brute force)."""
    counts = np.random.default_rng(nx * 10 + nz).integers(0, 30, size=nx * nz)
    xi, v, attrs, off = _state(counts, 1, seed=7)
    rng = np.random.default_rng(8)
    pos = rng.uniform(0.02, 0.98, size=(2, xi.size))
    ux, uz = 0.6, -0.7
    for w, u in ((pos[0], ux), (pos[1], uz)):
        f = (w + u) % 1.0
        w[(f < 1e-6) | (f > 1 - 1e-6)] += 0.003
    cx, cz = I.uniform_courant(nx, nz, ux, uz)
    new_pos, new_cell, fl = D.displace(nx, nz, cx, cz, pos, off)
    assert fl == 0
    c = np.repeat(np.arange(nx * nz), counts)
    ax = (c // nz + pos[0] + ux) % nx
    az = (c % nz + pos[1] + uz) % nz
    assert np.array_equal(new_cell, np.floor(ax).astype(int) * nz + np.floor(az).astype(int))
    assert np.allclose(new_pos[0], ax - np.floor(ax), atol=1e-12, rtol=0)
    order, o2 = D.resegment(new_cell, nx * nz)
    brute = [j for cc in range(nx * nz) for j in range(xi.size) if new_cell[j] == cc]
    assert order.tolist() == brute
