"""Writes tests/golden/golovin_dm_dlnr_bins.txt from the oracle's closed form only.

Bin-averaged dm/dlnr [g m^-3 per unit ln r] of the analytic Golovin solution
on the paper's 31 radius bins (section 'API in brief'), for v0 = volume of a
30.531 um sphere, N0 = 2^23 m^-3, b = 1500 1/s, rho_w = 1000 kg m^-3.
Run: python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
from oracle import closed_form as cf  # noqa: E402

V0 = float(cf.volume_of_radius(30.531e-6))
N0 = 2 ** 23
B = 1500.0


def main():
    edges = cf.radius_edges()
    rows = []
    for t in (0, 1200, 2400, 3600):
        rows.append(cf.golovin_dm_dlnr_bins(edges, t, B, N0, V0) * 1e3)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golovin_dm_dlnr_bins.txt")
    with open(out, "w") as f:
        f.write("# bin r_lo_um r_hi_um dm/dlnr[g m^-3] at t = 0 1200 2400 3600 s\n")
        f.write("# written by tests/golden/make_golden.py from oracle/closed_form.py\n")
        for k in range(len(edges) - 1):
            f.write(f"{k} {edges[k] * 1e6:.6f} {edges[k + 1] * 1e6:.6f} "
                    + " ".join(f"{rows[i][k]:.9e}" for i in range(4)) + "\n")


if __name__ == "__main__":
    main()
