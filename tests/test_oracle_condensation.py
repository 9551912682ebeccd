"""Pins of the condensation oracle (CPU): tabulated values and textbook
magnitudes for the thermodynamic terms, closed forms and limits of the
equilibrium curve and of the growth step, an independent root finder and an
independent ODE integrator for the implicit step."""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from oracle import condensation as cd


def test_saturation_pressure_against_tables():
    """Saturation vapour pressure over water (standard tables: 1228 Pa at
    10 C, 2339 Pa at 20 C, 4246 Pa at 30 C) within 0.3 %."""
    for t_c, e in [(10.0, 1228.0), (20.0, 2339.0), (30.0, 4246.0)]:
        assert abs(cd.saturation_pressure(273.15 + t_c) / e - 1.0) < 3e-3


def test_diffusivity_magnitude():
    """Vapour diffusivity in air: about 0.24-0.25 cm^2/s at 20 C and 1 atm,
    inversely proportional to pressure."""
    d = cd.diffusivity(293.15, 101325.0)
    assert 2.35e-5 < d < 2.55e-5
    assert cd.diffusivity(293.15, 50662.5) == pytest.approx(2 * d, rel=1e-14)


def test_growth_parameter_magnitude():
    """1 / (F_k + F_d), the growth parameter of r dr/dt = G (S - S_eq), is of
    order 100 um^2/s for cloud conditions (Rogers & Yau 1989), larger when
    warmer and at lower pressure."""
    for T in (273.15, 283.15, 293.15):
        for p in (80e3, 100e3):
            fk, fd = cd.growth_terms(T, p)
            assert fk > 0 and fd > 0
            assert 0.3e-10 < 1.0 / (fk + fd) < 2.0e-10
    g = lambda T, p: 1.0 / sum(cd.growth_terms(T, p))
    assert g(293.15, 100e3) > g(273.15, 100e3)
    assert g(283.15, 80e3) > g(283.15, 100e3)


def test_growth_law_is_the_linearised_heat_and_vapour_balance():
    """F_k + F_d against the exact balance it linearises: a flat water
    surface at temperature T_s loses latent heat L F by conduction,
    K (T_s - T) = L F, while vapour diffuses to it, F = D (rho_v - rho_vs(T_s)),
    with rho_vs(T_s) = e_s(T_s) / (R_v T_s) and e_s following Clausius-
    Clapeyron from the oracle's e_s(T).  Solved for T_s by bisection at
    S - 1 = 1e-6, the flux per unit (S - 1) equals rho_w / (F_k + F_d) to
    1e-5 (a dropped term, such as the -1 in F_k, shifts it by several %)."""
    for T in (273.15, 283.15, 293.15):
        for p in (70e3, 100e3):
            es = cd.saturation_pressure(T)
            D = cd.diffusivity(T, p)
            S = 1.0 + 1e-6
            rho_v = S * es / (cd.R_V * T)

            def rho_vs(ts):
                return es * np.exp(cd.LV / cd.R_V * (1.0 / T - 1.0 / ts)) / (cd.R_V * ts)

            lo, hi = T - 1.0, T + 1.0
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                h = cd.LV * D * (rho_v - rho_vs(mid)) - cd.K_AIR * (mid - T)
                lo, hi = (mid, hi) if h > 0 else (lo, mid)
            flux = D * (rho_v - rho_vs(0.5 * (lo + hi)))
            fk, fd = cd.growth_terms(T, p)
            assert flux / (S - 1.0) == pytest.approx(cd.RHO_W / (fk + fd), rel=1e-5), (T, p)


def test_kelvin_coefficient_magnitude():
    """A = 2 sigma / (rho_w R_v T): about 3.3e-7 / T m (Rogers & Yau quote
    3.3e-5 / T cm with a slightly larger surface tension), within 8 %."""
    for T in (273.15, 293.15):
        assert abs(cd.kelvin_a(T) / (3.3e-7 / T) - 1.0) < 0.08


def test_equilibrium_curve_limits():
    """Pure water: S_eq = exp(A / r), close to 1 + A / r for r >> A.  With
    solute, far above the dry radius, S_eq = 1 + A / r - kappa r_d^3 / r^3 to
    second order; at the dry radius S_eq = 0."""
    a = cd.kelvin_a(283.15)
    for r in (1e-7, 1e-6, 1e-5):
        s = cd.s_eq(r * r, 0.0, 0.0, a)
        assert abs(s - (1.0 + a / r)) <= 2 * (a / r) ** 2
    rd, kappa = 5e-8, 0.6
    rd3 = rd ** 3
    for r in (10 * rd, 30 * rd, 100 * rd):
        s = cd.s_eq(r * r, rd3, kappa, a)
        approx = 1.0 + a / r - kappa * rd3 / r ** 3
        err2 = (a / r) ** 2 + (kappa * rd3 / r ** 3) ** 2 + (a / r) * (kappa * rd3 / r ** 3)
        assert abs(s - approx) <= 2 * err2
    assert cd.s_eq(rd * rd, rd3, kappa, a) == 0.0
    assert cd.s_eq(0.9 * rd * rd, rd3, kappa, a) == 0.0


def test_critical_supersaturation():
    """The maximum of S_eq - 1 over r against Petters & Kreidenweis's
    approximation sqrt(4 A^3 / (27 kappa r_d^3)) (within 10 % for dry radii
    where the critical radius is far above the dry one)."""
    a = cd.kelvin_a(283.15)
    for rd, kappa in [(2e-8, 0.6), (5e-8, 0.6), (5e-8, 0.1), (1e-7, 1.2)]:
        r = np.geomspace(1.01 * rd, 1e-4, 200001)
        sc = (cd.s_eq(r * r, rd ** 3, kappa, a) - 1.0).max()
        approx = np.sqrt(4 * a ** 3 / (27 * kappa * rd ** 3))
        assert abs(sc / approx - 1.0) < 0.1, (rd, kappa, sc, approx)


def test_derivative_against_differences():
    """d S_eq / dx against central differences of S_eq."""
    a = cd.kelvin_a(283.15)
    rd, kappa = 5e-8, 0.6
    for r in (6e-8, 2e-7, 1e-6, 1e-5):
        x = r * r
        h = x * 1e-6
        fd = (cd.s_eq(x + h, rd ** 3, kappa, a) - cd.s_eq(x - h, rd ** 3, kappa, a)) / (2 * h)
        assert cd.s_eq_dx(x, rd ** 3, kappa, a) == pytest.approx(fd, rel=1e-5)


def test_pure_diffusion_closed_form():
    """No curvature and no solute: S_eq = 1, so x1 = x0 + c (S - 1) exactly
    (growth and evaporation)."""
    x0 = np.array([1e-10, 4e-10, 2.5e-9])
    c = 2.0 * 0.5 / sum(cd.growth_terms(283.15, 90e3))
    for S in (1.01, 1.0005, 0.995):
        x1 = cd.solve_x(x0, np.zeros(3), 0.0, 0.0, 0.0, c, S)
        assert np.allclose(x1, x0 + c * (S - 1.0), rtol=1e-14, atol=0)


def _bisect(f, lo, hi, n=200):
    for _ in range(n):
        mid = 0.5 * (lo + hi)
        neg = f(mid) < 0
        lo = np.where(neg, mid, lo)
        hi = np.where(neg, hi, mid)
    return 0.5 * (lo + hi)


def test_solver_against_bisection():
    """Where the implicit equation has a single root (subsaturated air, and
    supersaturated air around droplets far above their critical radius) the
    bracketed Newton root equals a 200-step bisection of the same equation."""
    rng = np.random.default_rng(3)
    T = 283.15
    a = cd.kelvin_a(T)
    c = 2.0 * 1.0 / sum(cd.growth_terms(T, 90e3))
    for case in ("subsaturated", "droplets"):
        n = 400
        if case == "subsaturated":
            rd = 10 ** rng.uniform(-8.3, -6.7, n)
            r0 = rd * 10 ** rng.uniform(0.01, 2.5, n)
            S = rng.uniform(0.8, 0.999, n)
        else:
            rd = 10 ** rng.uniform(-8.3, -7.5, n)
            r0 = 10 ** rng.uniform(-5.3, -4.3, n)
            S = rng.uniform(1.0, 1.01, n)
        kappa = rng.uniform(0.05, 1.2, n)
        rd3 = rd ** 3
        x0 = r0 * r0
        xd = np.cbrt(rd3) ** 2
        x1 = cd.solve_x(x0, xd, rd3, kappa, a, c, S)
        ref = _bisect(lambda x: x - x0 - c * (S - cd.s_eq(x, rd3, kappa, a)), xd.copy(),
                      np.maximum(xd, x0 + c * S))
        assert np.allclose(x1, ref, rtol=1e-12, atol=0), case


def test_haze_particle_stays_at_equilibrium():
    """A haze particle at its Koehler equilibrium for S below the critical
    saturation (the root of S_eq = S below the critical radius, found by
    bisection) does not move in a step of 1, 10 or 100 s."""
    T = 283.15
    a = cd.kelvin_a(T)
    G = 1.0 / sum(cd.growth_terms(T, 90e3))
    for rd, kappa, S in [(2e-8, 0.6, 1.002), (5e-8, 0.3, 0.95), (1e-8, 1.0, 1.004)]:
        rd3 = rd ** 3
        r = np.geomspace(1.001 * rd, 1e-5, 100001)
        rc = r[np.argmax(cd.s_eq(r * r, rd3, kappa, a))]
        xe = _bisect(lambda x: cd.s_eq(x, rd3, kappa, a) - S, np.array([(1.001 * rd) ** 2]),
                     np.array([rc * rc]))
        for dt in (1.0, 10.0, 100.0):
            x1 = cd.solve_x(xe, np.array([np.cbrt(rd3) ** 2]), rd3, kappa, a, 2 * dt * G, S)
            assert x1[0] == pytest.approx(xe[0], rel=1e-9), (rd, kappa, S, dt)


def test_small_steps_follow_the_ode():
    """Many small implicit steps converge to the growth ODE
    r dr/dt = (S - S_eq(r)) / (F_k + F_d) integrated independently (RK45,
    tight tolerances): within 1e-4 after 2 s in 2000 steps."""
    T, p, S = 283.15, 90e3, 1.003
    a = cd.kelvin_a(T)
    G = 1.0 / sum(cd.growth_terms(T, p))
    rd, kappa = 3e-8, 0.6
    rd3 = rd ** 3
    r_init = 2e-6

    def rhs(t, y):
        r = y[0]
        return [G * (S - cd.s_eq(r * r, rd3, kappa, a)) / r]

    sol = solve_ivp(rhs, (0.0, 2.0), [r_init], rtol=1e-11, atol=1e-16)
    x = np.array([r_init ** 2])
    dt = 2.0 / 2000
    c = 2.0 * dt * G
    for _ in range(2000):
        x = cd.solve_x(x, np.array([rd * rd]), rd3, kappa, a, c, S)
    assert abs(np.sqrt(x[0]) / sol.y[0, -1] - 1.0) < 1e-4


def test_step_keeps_multiplicity_dry_volume_and_dead_slots():
    """A step changes only live wet volumes, never below the dry volume; each
    live droplet moves towards equilibrium: it grows where S exceeds its
    S_eq and shrinks where S is below it."""
    rng = np.random.default_rng(5)
    n = 300
    off = np.array([0, 100, 200, 300], dtype=np.int64)
    xi = rng.integers(1, 1000, n).astype(np.int64)
    xi[::7] = 0
    vd = cd.FOUR_PI_3 * (10 ** rng.uniform(-8, -7, n)) ** 3
    v = vd * 10 ** rng.uniform(0.5, 4, n)
    attrs = np.stack([vd, 0.5 * vd])
    v0 = v.copy()
    a0 = attrs.copy()
    S = np.array([1.01, 0.5, 0.98])
    cd.step(xi, v, attrs, off, [283.15] * 3, [90e3] * 3, S, 5.0, 0, 1)
    assert np.array_equal(attrs, a0)
    dead = xi == 0
    assert np.array_equal(v[dead], v0[dead])
    live = ~dead
    assert np.all(v[live] >= vd[live])
    x0 = np.cbrt(v0 / cd.FOUR_PI_3) ** 2
    se = cd.s_eq(x0, vd / cd.FOUR_PI_3, 0.5, cd.kelvin_a(283.15))
    drive = np.repeat(S, 100) - se
    grow = live & (drive > 1e-9)
    shrink = live & (drive < -1e-9)
    assert grow.sum() > 20 and shrink.sum() > 100
    assert np.all(v[grow] > v0[grow]) and np.all(v[shrink] < v0[shrink])
