"""Seeded synthetic inputs for SDM box and grid workloads.

Initialisation only: this module draws or samples multiplicities, volumes,
extensive attributes and cell layouts with numpy, and holds none of the
coalescence arithmetic.  Both the HIP path's tests/benchmark and the CPU
oracle take their inputs from here, so neither depends on the other.

Workloads follow the PySDM v1 paper's box set-up (section "API in brief": an
exponential spectrum sampled so that every super-droplet starts with the same
multiplicity, dt = 1 s, dV = 1e6 m^3, Golovin b = 1.5e3 1/s) and the
geometric-kernel box of section "Box environment examples", widened to grids of
independent cells and to a stream of box requests.

Readings (where the paper gives no value):
  - deterministic sampling takes quantile midpoints (i + 1/2) / n;
  - the mean volume v0 is that of a 30.531 um radius sphere and N0 dV is an
    exact integer (2^23 m^-3 x 1e6 m^3);
  - N dV is split into integers xi_i = floor(N dV / n) + [i < N dV mod n] so
    that the total is exact;
  - grid cells draw their SD count from numpy.random.default_rng(0), extra
    attributes from default_rng(1) and the drizzle cells of the large grid
    from default_rng(2).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy import special

GOLOVIN = 0
GEOMETRIC = 1


def sphere_volume(r):
    return (4.0 * np.pi / 3.0) * np.asarray(r, dtype=np.float64) ** 3


def split_count(total: int, n: int) -> np.ndarray:
    """Integers xi_i >= 0 with sum exactly `total`: floor(total/n) + [i < total mod n]."""
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    base, rem = divmod(int(total), n)
    xi = np.full(n, base, dtype=np.int64)
    xi[:rem] += 1
    return xi


def exponential_volumes(n: int, v0: float) -> np.ndarray:
    """Quantile midpoints of an exponential volume spectrum with mean v0."""
    u = (np.arange(n, dtype=np.float64) + 0.5) / n
    return -v0 * np.log1p(-u)


def lognormal_volumes(n: int, r_median: float, sigma_g: float) -> np.ndarray:
    """Quantile midpoints of a lognormal radius spectrum, as volumes."""
    u = (np.arange(n, dtype=np.float64) + 0.5) / n
    r = r_median * sigma_g ** special.ndtri(u)
    return sphere_volume(r)


@dataclass
class State:
    """SoA state of one simulation (host arrays)."""

    xi: np.ndarray  # int64[n_slots]
    v: np.ndarray  # float64[n_slots]
    attrs: np.ndarray  # float64[n_attr, n_slots]
    cell_off: np.ndarray  # int64[n_cells + 1]
    dt: float = 1.0
    dv: float = 1e6
    kernel: int = GOLOVIN
    b: float = 1500.0
    adaptive: bool = False
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def n_slots(self):
        return int(self.xi.size)

    @property
    def n_cells(self):
        return int(self.cell_off.size - 1)

    @property
    def n_attr(self):
        return int(self.attrs.shape[0])

    def copy(self):
        return State(self.xi.copy(), self.v.copy(), self.attrs.copy(), self.cell_off.copy(),
                     self.dt, self.dv, self.kernel, self.b, self.adaptive, self.seed,
                     dict(self.meta))


# ---------------------------------------------------------------------------
# Box workloads
# ---------------------------------------------------------------------------

V0_GOLOVIN = float(sphere_volume(30.531e-6))  # 1.19209728e-13 m^3
N0_GOLOVIN = 2 ** 23  # m^-3


def golovin_box(n_sd: int = 2 ** 13, dv: float = 1e6, n0: int = N0_GOLOVIN,
                v0: float = V0_GOLOVIN, b: float = 1500.0, seed: int = 0,
                replicas: int = 1) -> State:
    """Exponential spectrum, equal multiplicities, Golovin kernel (one cell per replica)."""
    xi1 = split_count(n0 * int(dv), n_sd) if float(dv).is_integer() else split_count(
        round(n0 * dv), n_sd)
    v1 = exponential_volumes(n_sd, v0)
    xi = np.tile(xi1, replicas)
    v = np.tile(v1, replicas)
    cell_off = np.arange(replicas + 1, dtype=np.int64) * n_sd
    return State(xi, v, np.zeros((0, xi.size)), cell_off, dt=1.0, dv=dv, kernel=GOLOVIN, b=b,
                 seed=seed, meta={"workload": "golovin_box", "n_sd": n_sd, "replicas": replicas})


def lognormal_cell(n_sd: int, n_conc: float = 1e8, dv: float = 1e6, r_median: float = 10e-6,
                   sigma_g: float = 1.4):
    xi = split_count(round(n_conc * dv), n_sd)
    v = lognormal_volumes(n_sd, r_median, sigma_g)
    return xi, v


def geometric_box(n_sd: int = 2 ** 17, dv: float = 1e6, n_conc: float = 1e8, seed: int = 0,
                  replicas: int = 1) -> State:
    """Lognormal radii (median 10 um, sigma_g 1.4), geometric sweep-out kernel."""
    xi1, v1 = lognormal_cell(n_sd, n_conc, dv)
    xi = np.tile(xi1, replicas)
    v = np.tile(v1, replicas)
    cell_off = np.arange(replicas + 1, dtype=np.int64) * n_sd
    return State(xi, v, np.zeros((0, xi.size)), cell_off, dt=1.0, dv=dv, kernel=GEOMETRIC,
                 b=0.0, seed=seed,
                 meta={"workload": "geometric_box", "n_sd": n_sd, "replicas": replicas})


# ---------------------------------------------------------------------------
# Grid workloads: many independent cells of uneven SD counts
# ---------------------------------------------------------------------------

def _attr_values(rng, n_attr, n):
    # positive, lognormal, independent of volume: dry volume then solute moles
    scales = [1e-19, 1e-16, 1e-16, 1e-17, 1e-17, 1e-18, 1e-18, 1e-18]
    out = np.empty((n_attr, n), dtype=np.float64)
    for q in range(n_attr):
        out[q] = scales[q % len(scales)] * np.exp(rng.normal(0.0, 0.5, size=n))
    return out


def grid(nx: int, ny: int, mean_sd: float, max_sd: int | None = None, n_attr: int = 0,
         dv: float = 2e6, n_conc: float = 1e8, kernel: int = GEOMETRIC, drizzle: bool = False,
         adaptive: bool = False, seed: int = 0) -> State:
    """nx*ny cells; SD counts Poisson(mean_sd) (optionally capped); lognormal cloud mode.

    drizzle=True replaces the last 4 SDs of a quarter of the cells (chosen with
    default_rng(2)) by drizzle drops (lognormal radius, median 100 um,
    sigma_g 1.2) with multiplicity floor(xi_cloud / 1000).
    """
    n_cells = nx * ny
    counts = np.random.default_rng(0).poisson(mean_sd, size=n_cells).astype(np.int64)
    if max_sd is not None:
        counts = np.minimum(counts, max_sd)
    cell_off = np.zeros(n_cells + 1, dtype=np.int64)
    np.cumsum(counts, out=cell_off[1:])
    n = int(cell_off[-1])
    xi = np.zeros(n, dtype=np.int64)
    v = np.zeros(n, dtype=np.float64)
    total = round(n_conc * dv)
    # cells with the same SD count share their deterministic sample
    cache = {}
    for c in range(n_cells):
        k = int(counts[c])
        if k == 0:
            continue
        if k not in cache:
            cache[k] = (split_count(total, k), lognormal_volumes(k, 10e-6, 1.4))
        o = cell_off[c]
        xi[o:o + k], v[o:o + k] = cache[k]
    attrs = _attr_values(np.random.default_rng(1), n_attr, n) if n_attr else np.zeros((0, n))
    if drizzle:
        rng = np.random.default_rng(2)
        pick = rng.random(n_cells) < 0.25
        for c in np.nonzero(pick)[0]:
            k = int(counts[c])
            if k < 4:
                continue
            o = cell_off[c] + k - 4
            r = 100e-6 * 1.2 ** rng.normal(0.0, 1.0, size=4)
            v[o:o + 4] = sphere_volume(r)
            xi[o:o + 4] = np.maximum(xi[o:o + 4] // 1000, 1)
    return State(xi, v, attrs, cell_off, dt=1.0, dv=dv, kernel=kernel, b=1500.0,
                 adaptive=adaptive, seed=seed,
                 meta={"workload": "grid", "nx": nx, "ny": ny, "mean_sd": mean_sd,
                       "n_attr": n_attr, "drizzle": drizzle})


def grid_64x64(seed: int = 0) -> State:
    """64x64 cells of 2e6 m^3, SD count min(Poisson(128), 200), 3 extra attributes."""
    return grid(64, 64, 128, max_sd=200, n_attr=3, dv=2e6, kernel=GEOMETRIC, seed=seed)


def grid_256x256(seed: int = 0) -> State:
    """256x256 cells of 2e6 m^3, SD count Poisson(256), 6 extra attributes, drizzle, adaptive."""
    return grid(256, 256, 256, n_attr=6, dv=2e6, kernel=GEOMETRIC, drizzle=True, adaptive=True,
                seed=seed)


# ---------------------------------------------------------------------------
# Condensation workloads: the first two extensive attributes are the dry
# volume and kappa x dry volume; the ambient state is given per cell
# ---------------------------------------------------------------------------

def _aerosol(rng, n, wet_v, haze_fraction=1 / 3):
    """Dry volumes (lognormal dry radius, median 40 nm, sigma_g 1.6), kappa
    (two modes, 0.6 and 0.1, half each) and wet volumes: a haze fraction at
    1.1-3 times the dry radius, the rest keep wet_v (at least the dry volume)."""
    rd = 40e-9 * 1.6 ** rng.normal(0.0, 1.0, size=n)
    vd = sphere_volume(rd)
    kappa = np.where(rng.random(n) < 0.5, 0.6, 0.1)
    haze = rng.random(n) < haze_fraction
    v = np.where(haze, sphere_volume(rd * rng.uniform(1.1, 3.0, size=n)), np.maximum(wet_v, vd))
    return v, np.stack([vd, kappa * vd])


def ambient(n_cells: int, seed: int = 6, s_lo: float = 0.995, s_hi: float = 1.005):
    """Per-cell temperature U(275, 295) K, pressure U(70, 100) kPa and
    saturation ratio U(s_lo, s_hi) (default_rng(seed))."""
    rng = np.random.default_rng(seed)
    return {"T": rng.uniform(275.0, 295.0, n_cells), "p": rng.uniform(70e3, 100e3, n_cells),
            "S": rng.uniform(s_lo, s_hi, n_cells)}


def aerosol_cells(n_cells: int, max_sd: int, n_attr: int = 2, rng_seed: int = 0,
                  dead_fraction: float = 0.1) -> State:
    """Uneven cells (empty and one-SD cells included, sizes up to max_sd) of
    aerosol and cloud droplets for condensation: attributes 0 and 1 are the
    dry volume and kappa x dry volume, further ones lognormal."""
    rng = np.random.default_rng(rng_seed)
    counts = rng.integers(0, max_sd + 1, size=n_cells)
    if n_cells >= 3:
        counts[0], counts[1], counts[2] = 0, 1, max_sd
    cell_off = np.zeros(n_cells + 1, dtype=np.int64)
    np.cumsum(counts, out=cell_off[1:])
    n = int(cell_off[-1])
    xi = rng.integers(1, 10 ** 9, size=n, dtype=np.int64)
    xi[rng.random(n) < dead_fraction] = 0
    wet = sphere_volume(10e-6 * 1.6 ** rng.normal(0.0, 1.0, size=n))
    v, a2 = _aerosol(rng, n, wet)
    attrs = np.concatenate([a2, _attr_values(rng, n_attr - 2, n)]) if n_attr > 2 else a2
    return State(xi, v, attrs, cell_off, dt=1.0, dv=1e6, kernel=GEOMETRIC, b=1500.0,
                 seed=rng_seed, meta={"workload": "aerosol_cells"})


def condensation_grid(nx: int = 256, ny: int = 256, seed: int = 0) -> State:
    """The 256 x 256 grid layout (Poisson(256) SDs per cell, cloud mode of
    median radius 10 um) with an aerosol population (default_rng(7)): dry
    volume and kappa x dry volume as attributes 0 and 1, a third of the SDs
    haze particles, and 4 further lognormal attributes (6 in all)."""
    st = grid(nx, ny, 256, n_attr=0, dv=2e6, kernel=GEOMETRIC, seed=seed)
    rng = np.random.default_rng(7)
    v, a2 = _aerosol(rng, st.n_slots, st.v)
    st.v = v
    st.attrs = np.concatenate([a2, _attr_values(np.random.default_rng(1), 4, st.n_slots)])
    st.meta = {"workload": "condensation_grid", "nx": nx, "ny": ny}
    return st


# ---------------------------------------------------------------------------
# Serving workload: a stream of box requests
# ---------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    arrival_s: float
    n_sd: int
    kernel: int
    n_steps: int
    seed: int


def serving_requests(n_requests: int = 4096, rate_per_s: float = 200.0, log2_min: float = 10,
                     log2_max: float = 16, n_steps: int = 600, rng_seed: int = 3):
    """Poisson arrivals, n_sd = round(2^U(log2_min, log2_max)), kernel 50/50 Golovin/geometric."""
    rng = np.random.default_rng(rng_seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    n_sd = np.round(2.0 ** rng.uniform(log2_min, log2_max, size=n_requests)).astype(np.int64)
    kern = (rng.random(n_requests) < 0.5).astype(np.int64)
    return [Request(i, float(t[i]), int(n_sd[i]), int(kern[i]), n_steps, i)
            for i in range(n_requests)]


def request_state(req: Request) -> State:
    """Initial box state of a request: Golovin requests get the exponential
    box, geometric ones the lognormal box, at the request's SD count."""
    if req.kernel == GOLOVIN:
        st = golovin_box(req.n_sd, seed=req.seed)
    else:
        st = geometric_box(req.n_sd, seed=req.seed)
    return st


# ---------------------------------------------------------------------------
# Small cases for pins and parity
# ---------------------------------------------------------------------------

def dyadic_golovin_box(n_sd: int = 2 ** 10, exponent: int = -60, seed: int = 0,
                       replicas: int = 1) -> State:
    """The Golovin box with every volume rounded to k * 2^exponent, 1 <= k < 2^24,
    so that sums of xi * v are exact integer multiples of 2^exponent while the
    volumes stay small enough for the update's fma to be exact."""
    st = golovin_box(n_sd, seed=seed, replicas=replicas)
    k = np.clip(np.round(np.ldexp(st.v, -exponent)), 1, 2 ** 24 - 1)
    st.v = np.ldexp(k, exponent)
    st.meta.update({"workload": "dyadic_golovin_box", "exponent": exponent})
    return st


def random_cells(n_cells: int, max_sd: int, n_attr: int = 0, kernel: int = GOLOVIN,
                 dead_fraction: float = 0.1, xi_max: int = 10 ** 9, rng_seed: int = 0,
                 dv: float = 1e6, p_boost: float = 1.0) -> State:
    """Uneven random cells (including empty and one-SD cells) with some dead
    slots; p_boost scales Golovin's b so that p > 1 occurs."""
    rng = np.random.default_rng(rng_seed)
    counts = rng.integers(0, max_sd + 1, size=n_cells)
    if n_cells >= 3:
        counts[0] = 0
        counts[1] = 1
        counts[2] = max_sd
    cell_off = np.zeros(n_cells + 1, dtype=np.int64)
    np.cumsum(counts, out=cell_off[1:])
    n = int(cell_off[-1])
    xi = rng.integers(1, xi_max, size=n, dtype=np.int64)
    # a few equal multiplicities so that ties and splits are exercised
    eq = rng.random(n) < 0.2
    xi[eq] = xi_max // 2
    xi[rng.random(n) < dead_fraction] = 0
    r = 10e-6 * 1.6 ** rng.normal(0.0, 1.0, size=n)
    v = sphere_volume(r)
    attrs = _attr_values(np.random.default_rng(rng_seed + 1), n_attr, n) if n_attr else \
        np.zeros((0, n))
    return State(xi, v, attrs, cell_off, dt=1.0, dv=dv, kernel=kernel, b=1500.0 * p_boost,
                 seed=rng_seed, meta={"workload": "random_cells"})


# ---------------------------------------------------------------------------
# Kinematic 2D set-up for displacement: droplet positions and a prescribed
# single-eddy flow given as face Courant numbers (inputs only: the
# displacement arithmetic is not here)
# ---------------------------------------------------------------------------

def positions(n: int, seed: int = 4) -> np.ndarray:
    """Positions of n droplets inside their cells: (2, n) fractions in [0, 1),
    uniform, from numpy.random.default_rng(seed)."""
    return np.random.default_rng(seed).random((2, n))


def single_eddy_courant(nx: int, nz: int, dt: float = 1.0, dx: float = 20.0, dz: float = 20.0,
                        w_max: float = 0.6):
    """Face Courant numbers of a non-divergent single-eddy flow over an
    nx x nz periodic-in-x domain (updraft in one half, downdraft in the other,
    no flow through the bottom and top), from the stream function
    psi(x, z) = -(w_max X / (2 pi)) sin(pi z / Z) cos(2 pi x / X) sampled at
    the cell corners; u = -dpsi/dz, w = dpsi/dx as corner differences, so the
    discrete divergence of every cell is zero up to rounding.
    Returns (cx (nx + 1, nz), cz (nx, nz + 1)).  Defaults: 20 m cells,
    w_max 0.6 m/s, dt 1 s (the drizzling stratocumulus set-up the paper's
    kinematic 2D example follows)."""
    X, Z = nx * dx, nz * dz
    x = np.arange(nx + 1)[:, None] * dx
    z = np.arange(nz + 1)[None, :] * dz
    psi = -(w_max * X / (2 * np.pi)) * np.sin(np.pi * z / Z) * np.cos(2 * np.pi * x / X)
    psi[:, 0] = 0.0
    psi[:, nz] = 0.0
    psi[nx, :] = psi[0, :]
    cx = -(psi[:, 1:] - psi[:, :-1]) * dt / (dx * dz)
    cz = (psi[1:, :] - psi[:-1, :]) * dt / (dx * dz)
    return np.ascontiguousarray(cx), np.ascontiguousarray(cz)


def uniform_courant(nx: int, nz: int, cx: float, cz: float):
    """Face Courant numbers of a uniform flow."""
    return np.full((nx + 1, nz), float(cx)), np.full((nx, nz + 1), float(cz))


def random_courant(nx: int, nz: int, amp: float = 0.9, seed: int = 5):
    """Face Courant numbers drawn uniformly from (-amp, amp) (not a physical
    flow: exercises every shift direction and the periodic wrap)."""
    rng = np.random.default_rng(seed)
    cx = rng.uniform(-amp, amp, size=(nx + 1, nz))
    cz = rng.uniform(-amp, amp, size=(nx, nz + 1))
    cx[nx, :] = cx[0, :]
    cz[:, nz] = cz[:, 0]
    return cx, cz
