"""Pins of the oracle's per-pair arithmetic (CPU only).

Each test checks the oracle against something fixed outside it: a closed form
(the scale factor), brute force over all orders of tiny cells (the expected
number of collisions per step must equal the unscaled pair sum of the
Smoluchowski-consistent rate, Shima et al. 2009), worked examples of the
collision-count and update rules, hand-computed kernel values, exact integer
and correctly rounded sums for the moments, and an FP-contraction probe.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import closed_form as cf

GOL, GEO = 0, 1


def test_scale_factor_closed_form(orc):
    for n in range(2, 200):
        expect = Fraction(n * (n - 1) // 2, n // 2)
        assert expect.denominator == 1
        assert orc.scale_factor(n) == expect.numerator
    assert [orc.scale_factor(n) for n in range(2, 8)] == [1, 3, 3, 5, 5, 7]


@pytest.mark.parametrize("kind", [GOL, GEO])
@pytest.mark.parametrize("n", [2, 3, 4, 5, 6, 7])
def test_brute_force_all_orders(orc, kind, n):
    """Averaged over all n! orders, the sum of scaled pair probabilities equals
    the sum over all C(n,2) pairs of max(xi) K dt/dV."""
    rng = np.random.default_rng(100 + n + 10 * kind)
    xi = rng.integers(1, 10 ** 9, size=n).astype(np.int64)
    v = cf.volume_of_radius(10e-6 * 2.0 ** rng.normal(0, 1, size=n))
    b, q = 1500.0, 1.0 / 1e6
    total = 0.0
    count = 0
    for perm in itertools.permutations(range(n)):
        total += math.fsum(orc.pairs_for_order(kind, b, q, xi, v, np.array(perm)))
        count += 1
    mean = total / count
    direct = math.fsum(max(xi[j], xi[k]) * orc.kernel_value(kind, b, v[j], v[k]) * q
                       for j in range(n) for k in range(j + 1, n))
    assert mean == pytest.approx(direct, rel=1e-12)


def test_pair_probability_uses_larger_multiplicity(orc):
    k = orc.kernel_value(GOL, 1500.0, 1e-15, 3e-15)
    p = orc.pair_probability(GOL, 1500.0, 1e-6, 7, 900, 1e-15, 3e-15, 5)
    assert p == ((900.0 * k) * 5.0) * 1e-6
    assert orc.pair_probability(GOL, 1500.0, 1e-6, 900, 7, 1e-15, 3e-15, 5) == p


@pytest.mark.parametrize("p,phi,gamma", [
    (2.25, 0.2, 3), (2.25, 0.25, 2), (2.25, 0.3, 2), (1.0, 0.0, 1), (0.0, 0.0, 0),
    (0.0, 0.999, 0), (0.5, 0.4999999, 1), (0.5, 0.5, 0), (7.0, 0.0, 7),
    (1e-300, 0.0, 1), (3.0e18, 0.5, 3 * 10 ** 18), (1e30, 0.1, 2 ** 62),
])
def test_gamma_rule(orc, p, phi, gamma):
    assert orc.gamma_from(p, phi) == gamma


# (xi_a, xi_b, v_a, v_b, gamma) -> (xi_a, xi_b, v_a, v_b)
WORKED = [
    ((5, 2, 1.0, 10.0, 2), (1, 2, 1.0, 12.0)),   # j*=a, g=2, remainder 1
    ((4, 2, 1.0, 10.0, 3), (1, 1, 12.0, 12.0)),  # g capped at xi_j/xi_k=2, split
    ((3, 3, 1.0, 2.0, 1), (1, 2, 3.0, 3.0)),     # tie -> first member is j*, split
    ((1, 1, 1.0, 2.0, 5), (0, 1, 3.0, 3.0)),     # split of xi_k=1 kills the first
    ((2, 7, 3.0, 1.0, 1), (2, 5, 4.0, 1.0)),     # j*=b
    ((2, 7, 3.0, 1.0, 0), (2, 7, 3.0, 1.0)),     # gamma=0: nothing
    ((10, 3, 1.0, 2.0, 1), (7, 3, 1.0, 3.0)),
    ((9, 3, 1.0, 2.0, 100), (1, 2, 5.0, 5.0)),   # g=3 uses xi_j up: split h=1
]


@pytest.mark.parametrize("inp,out", WORKED)
def test_update_worked_examples(orc, inp, out):
    xa, xb, va, vb, g = inp
    xi = np.array([xa, xb], dtype=np.int64)
    v = np.array([va, vb], dtype=np.float64)
    attrs = np.array([[va * 3, vb * 3], [1.0, 2.0]], dtype=np.float64)
    s_xv = xa * va + xb * vb
    orc.update_pair(xi, v, attrs, g)
    assert (xi.tolist(), v.tolist()) == ([out[0], out[1]], [out[2], out[3]])
    assert xi[0] * v[0] + xi[1] * v[1] == s_xv  # sum of xi v conserved
    assert xi[0] * attrs[0, 0] + xi[1] * attrs[0, 1] == 3 * s_xv  # attributes follow v
    assert (xi >= 0).all()


def test_update_large_gamma_attrs_follow(orc):
    xi = np.array([10 ** 12, 10 ** 6], dtype=np.int64)
    v = np.array([2.0 ** -50, 2.0 ** -40], dtype=np.float64)
    attrs = np.array([[2.0 ** -60, 2.0 ** -61]], dtype=np.float64)
    orc.update_pair(xi, v, attrs, 17)
    assert xi.tolist() == [10 ** 12 - 17 * 10 ** 6, 10 ** 6]
    assert v[1] == 2.0 ** -40 + 17 * 2.0 ** -50 and v[0] == 2.0 ** -50
    assert attrs[0, 1] == 2.0 ** -61 + 17 * 2.0 ** -60


R = cf.volume_of_radius


@pytest.mark.parametrize("kind,r1,r2,expect,rel", [
    (GOL, 30.531e-6, 30.531e-6, 3.576292e-10, 2e-7),
    (GEO, 10e-6, 20e-6, 1.009394e-10, 2e-6),
    (GEO, 30e-6, 50e-6, 3.828219e-9, 2e-6),
    (GEO, 100e-6, 1000e-6, 2.112085e-5, 2e-6),
    (GEO, 10e-6, 12e-6, 7.961500e-12, 2e-6),
    (GEO, 20e-6, 20e-6, 0.0, 0.0),
])
def test_kernel_hand_values(orc, kind, r1, r2, expect, rel):
    k = orc.kernel_value(kind, 1500.0, float(R(r1)), float(R(r2)))
    assert k == pytest.approx(expect, rel=rel, abs=0.0)
    assert orc.kernel_value(kind, 1500.0, float(R(r2)), float(R(r1))) == k  # symmetric


def test_terminal_velocity_regimes(orc):
    # Rogers & Yau (1989): 1.19e6 cm^-1 s^-1 r^2, 8e3 s^-1 r, 2.01e3 cm^0.5 s^-1 r^0.5
    assert orc.terminal_velocity(10e-6) == pytest.approx(1.19e8 * 1e-10, rel=1e-15)
    assert orc.terminal_velocity(300e-6) == pytest.approx(8e3 * 300e-6, rel=1e-15)
    assert orc.terminal_velocity(1.5e-3) == pytest.approx(2.01e3 * math.sqrt(0.15) * 1e-2,
                                                         rel=1e-14)
    # continuous: regimes meet at k2/k1 and (k3/k2)^2
    for r in (8e3 / 1.19e8, (201.0 / 8e3) ** 2):
        lo, hi = orc.terminal_velocity(r * (1 - 1e-9)), orc.terminal_velocity(r * (1 + 1e-9))
        assert abs(hi - lo) < 1e-8
    r_grid = np.logspace(-6, -2.3, 400)
    u = [orc.terminal_velocity(r) for r in r_grid]
    assert all(b >= a for a, b in zip(u, u[1:]))


def test_radius_inverts_volume(orc):
    for r in (1e-6, 30.531e-6, 1e-3):
        assert orc.radius(float(R(r))) == pytest.approx(r, rel=4e-16 * 4)


def test_moments_exact_and_rounded(orc):
    rng = np.random.default_rng(5)
    cell_off = np.array([0, 0, 1, 50, 300], dtype=np.int64)
    n = int(cell_off[-1])
    xi = rng.integers(0, 2 ** 50, size=n).astype(np.int64)
    xi[rng.random(n) < 0.2] = 0
    v = cf.volume_of_radius(10e-6 * 3.0 ** rng.normal(0, 1, size=n))
    attrs = rng.random((2, n))
    edges_r = cf.radius_edges()
    edges_v = cf.volume_of_radius(edges_r)
    cfg = orc.OracleConfig(n_slots=n, n_cells=4, n_attr=2)
    m = orc.moments(cfg, xi, v, attrs, cell_off, edges_v)
    for c in range(4):
        sl = slice(cell_off[c], cell_off[c + 1])
        live = xi[sl] > 0
        xs, vs, As = xi[sl][live], v[sl][live], attrs[:, sl][:, live]
        assert m["m0"][c] == sum(int(x) for x in xs)
        w1 = [float(x) * y for x, y in zip(xs, vs)]
        assert m["m1"][c] == pytest.approx(math.fsum(w1), rel=2 ** -52, abs=0)
        assert m["m2"][c] == pytest.approx(math.fsum(a * y for a, y in zip(w1, vs)),
                                           rel=2 ** -52, abs=0)
        for qq in range(2):
            assert m["attr_sums"][c, qq] == pytest.approx(
                math.fsum(float(x) * a for x, a in zip(xs, As[qq])), rel=2 ** -52, abs=0)
        for k in range(len(edges_v) - 1):
            inb = (vs >= edges_v[k]) & (vs < edges_v[k + 1])
            assert m["spectrum"][c, k] == pytest.approx(
                math.fsum(float(x) * y for x, y in zip(xs[inb], vs[inb])), rel=2 ** -52, abs=0)


def test_no_fp_contraction(orc):
    a, b, c = 1.0 + 2.0 ** -30, 1.0 - 2.0 ** -30, -1.0
    # exact a*b = 1 - 2^-60 rounds to 1.0; fused would give -2^-60
    assert orc.probe_mul_add(a, b, c) == 0.0
