"""Analytic solution of the Smoluchowski equation for the Golovin kernel.

TEST INFRASTRUCTURE ONLY (pins the oracle; see the package docstring).

The PySDM v1 paper (section "Box environment examples") compares its SDM box
run with the Golovin additive kernel K = b (v1 + v2) against the analytic
solution of the Smoluchowski equation.  For an exponential initial spectrum
n(v, 0) = (N0 / v0) exp(-v / v0) that solution (Golovin 1963; Scott 1968) is

    tau    = 1 - exp(-b N0 v0 t),       x = v / v0,
    n(v,t) = (N0 / v0) (1 - tau) / (x sqrt(tau)) exp(-(1 + tau) x) I1(2 x sqrt(tau)),

with moments M0 = N0 exp(-b M1 t), M1 = N0 v0 (constant), M2 = 2 N0 v0^2
exp(2 b M1 t).  exp(-(1+tau) x) I1(2 x sqrt(tau)) is evaluated as
ive(1, z) exp(-x (1 - sqrt(tau))^2) with z = 2 x sqrt(tau), which stays finite
where I1 alone overflows.

The mass-density spectrum dm/dlnr is rho_w v dN/dlnr = 3 rho_w v^2 n(v); a
bin's value is its average over ln r, (1 / dlnr) * integral of rho_w v n(v) dv.
"""
from __future__ import annotations

import numpy as np
from scipy import integrate, special

RHO_W = 1000.0  # kg m^-3, density of liquid water


def radius_edges(r_min=10e-6, r_max=5e-3, num=32):
    """Log-spaced radius bin edges [m] (the paper's 32 edges, 10 um to 5 mm)."""
    return np.logspace(np.log10(r_min), np.log10(r_max), num=num)


def volume_of_radius(r):
    return (4.0 * np.pi / 3.0) * np.asarray(r, dtype=np.float64) ** 3


def golovin_tau(t, b, n0, v0):
    return 1.0 - np.exp(-b * n0 * v0 * t)


def golovin_n(v, t, b, n0, v0):
    """Number density per unit volume and per unit droplet volume [m^-3 m^-3]."""
    v = np.asarray(v, dtype=np.float64)
    x = v / v0
    if t == 0:
        return (n0 / v0) * np.exp(-x)
    tau = golovin_tau(t, b, n0, v0)
    st = np.sqrt(tau)
    z = 2.0 * x * st
    return (n0 / v0) * (1.0 - tau) / (x * st) * special.ive(1, z) * np.exp(-x * (1.0 - st) ** 2)


def golovin_moments(t, b, n0, v0):
    m1 = n0 * v0
    return {
        "m0": n0 * np.exp(-b * m1 * t),
        "m1": m1,
        "m2": 2.0 * n0 * v0 * v0 * np.exp(2.0 * b * m1 * t),
    }


def golovin_dm_dlnr_bins(r_edges, t, b, n0, v0, rho_w=RHO_W):
    """Bin-averaged dm/dlnr [kg m^-3 per unit ln r] on the given radius edges."""
    r_edges = np.asarray(r_edges, dtype=np.float64)
    out = np.zeros(len(r_edges) - 1)
    for k in range(len(r_edges) - 1):
        xa = volume_of_radius(r_edges[k]) / v0
        xb = volume_of_radius(r_edges[k + 1]) / v0
        # integral of rho_w v n(v) dv = rho_w n0 v0 * integral of x * (v0 n(x v0) / n0) dx
        f = lambda x: x * golovin_n(x * v0, t, b, n0, v0) * v0 / n0  # noqa: E731
        val, _ = integrate.quad(f, xa, xb, limit=200, epsabs=0.0, epsrel=1e-10)
        out[k] = rho_w * n0 * v0 * val / np.log(r_edges[k + 1] / r_edges[k])
    return out


def sdm_dm_dlnr(spectrum_sum_xi_v, r_edges, dv, rho_w=RHO_W):
    """Convert per-bin sums of xi*v [m^3] into dm/dlnr [kg m^-3 per unit ln r]."""
    r_edges = np.asarray(r_edges, dtype=np.float64)
    return rho_w * np.asarray(spectrum_sum_xi_v) / dv / np.log(r_edges[1:] / r_edges[:-1])
