"""Host-side helpers of bench.py (no GPU): which cell classes a launch shape
populates, and the committed HBM-traffic summary it reads."""
import json
import os

import numpy as np

import bench
from paper_2103_17238_amd import inputs as I


def test_launched_classes():
    st = I.grid(4, 4, 100, max_sd=500, seed=1)
    n = np.diff(st.cell_off)
    caps = bench.launched_classes(st, 0x1F)
    # every populated cell goes to the smallest enabled class that fits
    want = sorted({min(c for c in bench.CLASS_CAPS if c >= x) for x in n if 0 < x <= 512})
    assert caps == want
    assert bench.launched_classes(st, 0x00) == [512]  # the 512-slot class is always on
    assert set(bench.launched_classes(st, 0x18)) <= {384, 512}


def test_traffic_summary_is_consistent():
    path = os.path.join(bench.PROFILES, "k_cells_grid256_pmc.json")
    d = json.load(open(path))
    for key in ("kernel_source_sha", "shapes"):
        assert key in d
    for key, shape in d["shapes"].items():
        # the scale factors come from a 1 GiB copy: expected KiB / counted KiB
        cp = shape["copy_probe"]
        assert abs(shape["fetch_scale"] - cp["bytes"] / 1024 / cp["fetch_kib_raw"]) < 1e-9
        assert abs(shape["write_scale"] - cp["bytes"] / 1024 / cp["write_kib_raw"]) < 1e-9
        mask, waves = key.split("/")
        # per step: the sum over the step's kernels of (KiB per dispatch x dispatches per step)
        f = sum(k["fetch_kib_per_dispatch_raw"] * k["per_step"] for k in shape["kernels"])
        w = sum(k["write_kib_per_dispatch_raw"] * k["per_step"] for k in shape["kernels"])
        assert abs(shape["fetch_kib_per_step"] - f * shape["fetch_scale"]) < 1
        assert abs(shape["write_kib_per_step"] - w * shape["write_scale"]) < 1
        tuning = {"wave_class_mask": int(mask, 16), "waves_per_cell": int(waves)}
        got = bench.traffic_from_profiles("k_cells", "grid256", 0, tuning)
        if d["kernel_source_sha"] == bench.kernel_source_sha():
            assert got == (shape["fetch_kib_per_step"] + shape["write_kib_per_step"]) * 1024.0
        else:
            assert got is None
    assert bench.traffic_from_profiles("k_cells", "grid256", 0, {"wave_class_mask": 0x1F,
                                                                 "waves_per_cell": 8}) is None


def test_displacement_traffic_summary_is_consistent():
    d = json.load(open(os.path.join(bench.PROFILES, "k_disp_grid256_single_eddy_pmc.json")))
    cp = d["copy_probe"]
    assert abs(d["fetch_scale"] - cp["bytes"] / 1024 / cp["fetch_kib_raw"]) < 1e-9
    assert abs(d["write_scale"] - cp["bytes"] / 1024 / cp["write_kib_raw"]) < 1e-9
    f = sum(k["fetch_kib_per_dispatch_raw"] * k["per_step"] for k in d["kernels"])
    w = sum(k["write_kib_per_dispatch_raw"] * k["per_step"] for k in d["kernels"])
    assert abs(d["fetch_kib_per_step"] - f * d["fetch_scale"]) < 1
    assert abs(d["write_kib_per_step"] - w * d["write_scale"]) < 1
    got = bench.displace_traffic_from_profiles()
    if d["displace_source_sha"] == bench.displace_source_sha():
        assert got == (d["fetch_kib_per_step"] + d["write_kib_per_step"]) * 1024.0
    else:
        assert got is None
