"""CPU oracle for diffusional growth (condensation / evaporation) of super-droplets.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the smoke
check and the CPU-baseline leg of the benchmark may call it; the product path
never does.  Plain numpy, IEEE fp64, written from the physics below, not from
any listing.

The PySDM v1 paper lists condensational growth among its dynamics (sections
"Introduction" and "API in brief") and drives it with ambient thermodynamics
in its parcel examples, where supersaturation activates aerosol into cloud
droplets and the modes differ in hygroscopicity (section "Adiabatic parcel
examples"), but fixes none of the physics.  Readings taken here (each a
textbook formula, named where it is used):

  - a super-droplet carries its wet volume v (the coalescence volume) and two
    extensive attributes: its dry volume v_d and kappa * v_d, with kappa the
    hygroscopicity parameter (Petters & Kreidenweis 2007); both are summed on
    coalescence like every extensive attribute, so the merged droplet's kappa
    is the dry-volume-weighted mean;
  - the ambient state is given per cell and held fixed over the step:
    temperature T [K], pressure p [Pa] and saturation ratio S (vapour
    pressure over saturation pressure; no feedback of the condensed water on
    the vapour within the step: that belongs to ambient thermodynamics);
  - equilibrium saturation ratio over a droplet of radius r with dry radius
    r_d (kappa-Koehler, Petters & Kreidenweis 2007):
        S_eq(r) = (r^3 - r_d^3) / (r^3 - r_d^3 (1 - kappa)) * exp(A / r),
    A = 2 sigma / (rho_w R_v T), and S_eq = 0 at or below the dry radius;
  - growth by vapour diffusion and heat conduction (Maxwell-Mason form,
    Rogers & Yau 1989, ch. 7):  r dr/dt = (S - S_eq(r)) / (F_k + F_d), with
        F_k = (L / (R_v T) - 1) L rho_w / (K T),
        F_d = rho_w R_v T / (D e_s(T)),
    D = 2.11e-5 (T / 273.15)^1.94 (101325 / p) m^2/s (Pruppacher & Klett
    1997), e_s(T) = 611.2 exp(17.67 (T - 273.15) / (T - 29.65)) Pa (Bolton
    1980), and constants sigma = 0.072 N/m, rho_w = 1000 kg/m^3,
    R_v = 461.5 J/(kg K), L = 2.5e6 J/kg, K = 2.4e-2 W/(m K);
  - time integration: one implicit Euler step in x = r^2 over dt,
        g(x) = x - x0 - c (S - S_eq(sqrt x)) = 0,  c = 2 dt / (F_k + F_d);
    g(x_d) < 0 at the dry size x_d = r_d^2 and g(x0 + c S) >= 0 (S_eq >= 0),
    so a root lies in [x_d, max(x_d, x0 + c S)]; it is found by Newton's
    method kept inside that bracket (a step that leaves the bracket, or a
    non-positive slope, is replaced by the bracket's midpoint; the bracket
    shrinks to the current point by the sign of g), from x0 clamped into the
    bracket, until the step is at most 1e-14 of x or after max_iter
    iterations;
  - the new wet volume is (4 pi / 3) r^3 with r = sqrt(x); multiplicities,
    dry volumes and kappa are unchanged; dead super-droplets (xi = 0) are
    left untouched; a wet volume below the dry volume is taken as the dry
    volume.

g has a single root for subsaturated air and for droplets well above
their critical radius; for haze particles and just-activated droplets at
time steps of about a second it can have three (the haze equilibrium, the
unstable equilibrium beyond the critical radius, and a root far beyond it).
The step's result is the root the bracketed Newton iteration reaches from
x0, the haze equilibrium for a particle sitting at it; a device whose
transcendental functions round differently in the last bit can, in rare
marginal cases, follow another path.
"""
from __future__ import annotations

import numpy as np

SIGMA = 0.072      # N/m, surface tension of water
RHO_W = 1000.0     # kg/m^3
R_V = 461.5        # J/(kg K)
LV = 2.5e6         # J/kg, latent heat of vaporisation
K_AIR = 2.4e-2     # W/(m K), thermal conductivity of air
D0 = 2.11e-5       # m^2/s, vapour diffusivity at 273.15 K and 101325 Pa
FOUR_PI_3 = 4.0 * np.pi / 3.0
TOL = 1e-14


def saturation_pressure(T):
    """e_s(T) [Pa] over plane water (Bolton 1980)."""
    T = np.asarray(T, dtype=np.float64)
    return 611.2 * np.exp(17.67 * (T - 273.15) / (T - 29.65))


def diffusivity(T, p):
    """D(T, p) [m^2/s] of water vapour in air (Pruppacher & Klett 1997)."""
    T = np.asarray(T, dtype=np.float64)
    return D0 * (T / 273.15) ** 1.94 * (101325.0 / np.asarray(p, dtype=np.float64))


def growth_terms(T, p):
    """(F_k, F_d) [s/m^2] of the Maxwell-Mason growth law (Rogers & Yau 1989)."""
    T = np.asarray(T, dtype=np.float64)
    fk = (LV / (R_V * T) - 1.0) * LV * RHO_W / (K_AIR * T)
    fd = RHO_W * R_V * T / (diffusivity(T, p) * saturation_pressure(T))
    return fk, fd


def kelvin_a(T):
    """A = 2 sigma / (rho_w R_v T) [m], the curvature coefficient."""
    return 2.0 * SIGMA / (RHO_W * R_V * np.asarray(T, dtype=np.float64))


def s_eq(x, rd3, kappa, a):
    """Equilibrium saturation ratio at x = r^2 (kappa-Koehler); 0 at or
    below the dry size."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(x)
    r3 = x * r
    above = r3 > rd3
    with np.errstate(divide="ignore", invalid="ignore"):
        f = (r3 - rd3) / (r3 - rd3 * (1.0 - kappa)) * np.exp(a / r)
    return np.where(above, f, 0.0)


def s_eq_dx(x, rd3, kappa, a):
    """d S_eq / dx at x = r^2 (0 at or below the dry size)."""
    x = np.asarray(x, dtype=np.float64)
    r = np.sqrt(x)
    r3 = x * r
    above = r3 > rd3
    with np.errstate(divide="ignore", invalid="ignore"):
        den = r3 - rd3 * (1.0 - kappa)
        f1 = (r3 - rd3) / den
        f2 = np.exp(a / r)
        d = f2 * ((rd3 * kappa) * (1.5 * r) / (den * den) - f1 * a / (2.0 * r3))
    return np.where(above, d, 0.0)


def solve_x(x0, xd, rd3, kappa, a, c, S, max_iter=32):
    """Root of g(x) = x - x0 - c (S - S_eq(x)) in [xd, max(xd, x0 + c S)] by
    bracketed Newton (element-wise over arrays)."""
    x0 = np.maximum(np.asarray(x0, dtype=np.float64), xd)
    lo = np.array(xd, dtype=np.float64, copy=True)
    hi = np.maximum(xd, x0 + c * S)
    x = np.minimum(np.maximum(x0, lo), hi)
    active = np.ones_like(x, dtype=bool)
    for _ in range(max_iter):
        if not active.any():
            break
        g = x - x0 - c * (S - s_eq(x, rd3, kappa, a))
        gp = 1.0 + c * s_eq_dx(x, rd3, kappa, a)
        zero = active & (g == 0.0)
        active &= ~zero
        lo = np.where(active & (g < 0.0), x, lo)
        hi = np.where(active & (g > 0.0), x, hi)
        with np.errstate(divide="ignore", invalid="ignore"):
            xn = x - g / gp
        bad = ~(gp > 0.0) | ~(xn >= lo) | ~(xn <= hi)
        xn = np.where(bad, 0.5 * (lo + hi), xn)
        done = np.abs(xn - x) <= TOL * xn
        x = np.where(active, xn, x)
        active &= ~done
    return x


def step(xi, v, attrs, cell_off, T, p, S, dt, dry_attr, kappa_attr, max_iter=32):
    """One condensation step in place on v; T, p, S per cell.  attrs[dry_attr]
    is the dry volume, attrs[kappa_attr] kappa times the dry volume."""
    C = len(cell_off) - 1
    cell = np.repeat(np.arange(C), np.diff(cell_off))
    T = np.asarray(T, dtype=np.float64)[cell]
    p = np.asarray(p, dtype=np.float64)[cell]
    Sc = np.asarray(S, dtype=np.float64)[cell]
    fk, fd = growth_terms(T, p)
    c = 2.0 * dt / (fk + fd)
    a = kelvin_a(T)
    vd = attrs[dry_attr]
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = np.where(vd > 0.0, attrs[kappa_attr] / vd, 0.0)
    rd3 = vd / FOUR_PI_3
    rd = np.cbrt(rd3)
    xd = rd * rd
    r0 = np.cbrt(np.maximum(v, vd) / FOUR_PI_3)
    live = xi > 0
    x1 = solve_x(r0 * r0, xd, rd3, kappa, a, c, Sc, max_iter)
    r1 = np.sqrt(x1)
    v1 = FOUR_PI_3 * (x1 * r1)
    v[live] = v1[live]
    return v
