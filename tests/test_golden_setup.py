"""The paper's printed box set-up (tests/golden/golovin_box_setup.json, from
the PySDM v1 paper's section 'API in brief') against the input generator and
the closed-form helpers."""
import json
import os

import numpy as np
import pytest

from oracle import closed_form as cf
from paper_2103_17238_amd import inputs as I

G = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_setup_matches_paper():
    p = json.load(open(os.path.join(G, "golovin_box_setup.json")))
    st = I.golovin_box(p["n_sd"])
    assert st.n_slots == 2 ** 17
    assert st.dt == p["dt_s"] and st.dv == p["dv_m3"] and st.b == p["golovin_b_per_s"]
    # the paper rounds N0 dV and the mean volume to three digits
    assert st.xi.sum() == pytest.approx(p["exponential_norm_factor"], rel=2e-3)
    assert (st.xi == st.xi[0]).all()  # equal initial multiplicity
    assert I.V0_GOLOVIN * 1e18 == pytest.approx(p["exponential_scale_um3"], rel=2e-3)
    assert st.v.mean() == pytest.approx(I.V0_GOLOVIN, rel=2e-3)  # deterministic sample mean
    e = p["radius_bin_edges"]
    edges = cf.radius_edges()
    assert len(edges) == e["num"]
    assert edges[0] * 1e6 == pytest.approx(e["min_um"]) and edges[-1] * 1e6 == pytest.approx(
        e["max_um"])
    assert np.allclose(np.diff(np.log(edges)), np.log(edges[1] / edges[0]))


def test_closed_form_bins_regression():
    rows = np.loadtxt(os.path.join(G, "golovin_dm_dlnr_bins.txt"))
    edges = cf.radius_edges()
    for i, t in enumerate((0, 1200, 2400, 3600)):
        now = cf.golovin_dm_dlnr_bins(edges, t, 1500.0, I.N0_GOLOVIN, I.V0_GOLOVIN) * 1e3
        assert np.allclose(now, rows[:, 3 + i], rtol=1e-8, atol=1e-300)
    # mass inside [10 um, 5 mm] tends to the liquid water content 1 g m^-3
    dl = np.log(edges[1:] / edges[:-1])
    assert (rows[:, 6] * dl).sum() == pytest.approx(1.0000037, rel=1e-4)
    assert (rows[:, 3] * dl).sum() == pytest.approx(0.99940, rel=1e-4)
