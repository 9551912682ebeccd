"""Writes tests/golden/geometric_box_2p17_3600s.txt with the oracle only.

The geometric box (2^17 super-droplets in one 1e6 m^3 cell, lognormal radii
of median 10 um and geometric spread 1.4 sampled at quantile midpoints,
N = 1e8 m^-3, geometric sweep-out kernel with E = 1, dt = 1 s, Philox seed 0)
is advanced 3600 steps by the CPU oracle; the file holds the mass spectrum
sum(xi v) per radius bin (48 log-spaced bins from 1 um to 5 mm) and the
total moments at t = 3600 s.  The GPU test free-runs the same box and
compares spectra within 1 % (relative L1 over bins).
Run: python tests/golden/make_geometric_box_spectrum.py   (about two minutes)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from oracle import closed_form as cf  # noqa: E402
from paper_2103_17238_amd import inputs as I  # noqa: E402

STEPS = 3600
N_SD = 2 ** 17
EDGES_R = (1e-6, 5e-3, 48)


def main():
    st = I.geometric_box(N_SD)
    cfg = oracle.OracleConfig(n_slots=st.n_slots, n_cells=st.n_cells, n_attr=st.n_attr,
                              dt=st.dt, dv=st.dv, b=st.b, kernel=st.kernel, seed=st.seed)
    t0 = time.time()
    for s in range(STEPS):
        oracle.step(cfg, st.xi, st.v, st.attrs, st.cell_off, s)
    ev = cf.volume_of_radius(cf.radius_edges(*EDGES_R))
    m = oracle.moments(cfg, st.xi, st.v, st.attrs, st.cell_off, ev)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "geometric_box_2p17_3600s.txt")
    with open(out, "w") as f:
        f.write("# geometric box 2^17 SDs, 3600 steps, seed 0: oracle state at t = 3600 s\n")
        f.write("# written by tests/golden/make_geometric_box_spectrum.py (oracle only)\n")
        f.write(f"# radius edges: {EDGES_R[2]} log-spaced bins from {EDGES_R[0]} m to "
                f"{EDGES_R[1]} m\n")
        f.write(f"m0 {int(m['m0'][0])}\n")
        f.write(f"m1 {m['m1'][0]:.17e}\n")
        f.write(f"m2 {m['m2'][0]:.17e}\n")
        f.write(f"live {int((st.xi > 0).sum())}\n")
        for k, x in enumerate(m["spectrum"][0]):
            f.write(f"bin {k} {x:.17e}\n")
    print(f"wrote {out} in {time.time() - t0:.1f} s")


if __name__ == "__main__":
    main()
