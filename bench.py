#!/usr/bin/env python3
"""SDM collision-coalescence benchmark on one MI355X.

Default workload: the large batched grid -- 256 x 256 cells of 2e6 m^3, SD
count Poisson(256) per cell (about 16.8 M super-droplets), geometric
sweep-out kernel, 6 extra fp64 extensive attributes, int64 multiplicities,
per-cell adaptive substepping keeping gamma <= 1, a drizzle mode in a quarter
of the cells.  Its state (1.07 GB) exceeds the GPU's last-level cache, so it
is the one on which the HBM-roofline fraction means something.  One step is
one outer coalescence step of every cell: one launch per populated cell-size
class (the classes up to 256 slots and the mid-size cells on a second
stream, concurrently).

Inputs are synthetic and seeded (paper_2103_17238_amd.inputs), resident in HBM
before timing starts.  The throughput unit is the super-droplet-step (one live
SD through one outer step).  Algorithmic bytes per step: 16 per live SD
(read xi and v), 8 per dead slot (read xi), (32 + 32 A) per colliding pair,
8 per cell (offsets).

The step timed for `value` is one call per step (one launch per class).
Separate figures in the same line: `batching` (a sample of cells as one
simulation against the same cells as separate simulations) and `fusion` (the
same steps in one call, which the library runs up to 8 steps per launch with
each cell kept in LDS).

Prints ONE JSON line.  --gpus above 1 is refused: the benchmark measures one
GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "super-droplet-steps/s (coalescence) + % HBM roofline; served p50/p99 latency"
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
# steps per serving tick: paired runs on 2048 requests of the serving trace
# gave p50 13.6-15.8 ms, p99 27-31 ms at 50 against 14.1-18.2 and 32-42 ms at 25
SERVE_TICK = 50


def note(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def make_state(name):
    from paper_2103_17238_amd import inputs as I

    if name == "grid256":
        return I.grid_256x256(), "grid256x256_poisson256_geometric_adaptive_A6"
    if name == "grid64":
        return I.grid_64x64(), "grid64x64_poisson128cap200_geometric_A3"
    if name == "golovin":
        return I.golovin_box(2 ** 13, replicas=1024), "golovin_box_2^13_x1024_cells"
    if name == "geometric":
        return I.geometric_box(2 ** 17), "geometric_box_2^17"
    raise SystemExit(f"unknown workload {name}")


def kernel_source_sha():
    """Hash of the source the workgroup-per-cell kernel is built from: the
    kernel file up to its mid-size section (the generator, the collision
    kernels, the wave helpers, the cell kernel itself).  Committed traffic
    figures are used only while it matches."""
    with open(os.path.join(ROOT, "paper_2103_17238_amd", "csrc", "sdm_kernels.hip")) as fh:
        src = fh.read()
    return hashlib.sha256(src[: src.index("// Mid-size cells")].encode()).hexdigest()[:16]


def displace_source_sha():
    with open(os.path.join(ROOT, "paper_2103_17238_amd", "csrc", "sdm_displace.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def displace_traffic_from_profiles():
    """HBM bytes per displacement step from the committed rocprofv3 --pmc
    summary, if it was taken on the current source; else None."""
    path = os.path.join(PROFILES, "k_disp_grid256_single_eddy_pmc.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("displace_source_sha") != displace_source_sha():
        return None
    return (d["fetch_kib_per_step"] + d["write_kib_per_step"]) * 1024.0


def condense_source_sha():
    with open(os.path.join(ROOT, "paper_2103_17238_amd", "csrc", "sdm_condense.hip"), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def condense_valu_from_profiles(step_s):
    """VALU issue of the condensation step from the committed SQ counters of
    the same source, over the measured step time; None if they do not match."""
    try:
        d = json.load(open(os.path.join(PROFILES, "k_condense_grid256_pmc.json")))
    except (OSError, ValueError):
        return None
    if d.get("condense_source_sha") != condense_source_sha() or "sq_insts_valu_per_step" not in d:
        return None
    achieved = d["sq_insts_valu_per_step"] / step_s
    return {"bound": "valu-issue", "unit": "wave64 VALU instructions/s",
            "insts_per_step": d["sq_insts_valu_per_step"], "achieved": achieved,
            "peak": VALU_PEAK_WAVE_INSTS, "frac": achieved / VALU_PEAK_WAVE_INSTS}


def condense_traffic_from_profiles():
    """HBM bytes per condensation step from the committed rocprofv3 --pmc
    summary, if it was taken on the current source; else None."""
    try:
        d = json.load(open(os.path.join(PROFILES, "k_condense_grid256_pmc.json")))
    except (OSError, ValueError):
        return None
    if d.get("condense_source_sha") != condense_source_sha():
        return None
    return (d["fetch_kib_per_step"] + d["write_kib_per_step"]) * 1024.0


CLASS_CAPS = (64, 128, 256, 384, 512)


def launched_classes(state, mask):
    """Capacities of the workgroup-per-cell classes that get cells."""
    import numpy as np

    mask |= 0x10
    caps = [c for k, c in enumerate(CLASS_CAPS) if (mask >> k) & 1]
    n = np.diff(state.cell_off)
    n = n[(n > 0) & (n <= 512)]
    used = sorted({caps[int(np.searchsorted(caps, x))] for x in np.unique(n)})
    return used


def traffic_from_profiles(kernel_name, workload, launches_bytes, tuning=None):
    """HBM bytes per step (all launches of the step) from committed rocprofv3
    --pmc summaries, if they were taken on the current kernel source in the
    same launch shape; else None."""
    path = os.path.join(PROFILES, f"{kernel_name}_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_sha() or tuning is None:
        return None
    shape = d.get("shapes", {}).get(f"{tuning['wave_class_mask']:#x}/{tuning['waves_per_cell']}")
    if shape is None:
        return None
    # KiB per step, already scaled by the copy probe (see the json's commands)
    return (shape["fetch_kib_per_step"] + shape["write_kib_per_step"]) * 1024.0


# VALU issue ceiling: 256 CUs x 4 SIMDs, one wave64 VALU instruction per SIMD
# every 4 cycles (16 lanes per cycle), 2.4 GHz
VALU_PEAK_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def valu_from_profiles(tuning, substeps_per_cell_step, step_s):
    """VALU issue of the step from the committed SQ-counter summary of the same
    cell-kernel source and launch shape: instructions per step (the profiled
    count scaled by the substeps per cell-step of this run over the profiled
    run's) over the measured step time, against the issue ceiling; None if
    the summary does not match."""
    path = os.path.join(PROFILES, "k_cells_grid256_sq.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha") != kernel_source_sha() or tuning is None:
        return None
    if d.get("shape") != f"{tuning['wave_class_mask']:#x}/{tuning['waves_per_cell']}":
        return None
    insts = sum(k["SQ_INSTS_VALU"] for k in d["kernels"].values())
    waves = sum(k["SQ_WAVES"] for k in d["kernels"].values())
    lanes = sum(k["SQ_THREAD_CYCLES_VALU"] for k in d["kernels"].values()) / insts
    scale = substeps_per_cell_step / d["substeps_per_cell_step"]
    per_step = insts * scale
    achieved = per_step / step_s
    return {"bound": "valu-issue", "unit": "wave64 VALU instructions/s",
            "insts_per_step": per_step, "insts_per_cell_step": per_step / waves,
            "achieved": achieved, "peak": VALU_PEAK_WAVE_INSTS,
            "frac": achieved / VALU_PEAK_WAVE_INSTS, "lanes_active": lanes,
            "note": "counts from the committed rocprofv3 SQ summary of this kernel source and "
                    "shape, scaled by substeps per cell-step (profiled "
                    f"{d['substeps_per_cell_step']:.3f}); peak = 256 CUs x 4 SIMDs x 2.4 GHz "
                    "/ 4 cycles per wave64 instruction"}


def cpu_baseline(state, n_cells_sample, steps):
    """The CPU oracle, as it stands, on the first cells of the same workload."""
    import numpy as np

    import oracle
    from paper_2103_17238_amd import inputs as I

    C = min(n_cells_sample, state.n_cells)
    end = int(state.cell_off[C])
    sub = I.State(state.xi[:end].copy(), state.v[:end].copy(),
                  np.ascontiguousarray(state.attrs[:, :end]), state.cell_off[: C + 1].copy(),
                  state.dt, state.dv, state.kernel, state.b, state.adaptive, state.seed)
    threads = min(16, int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                  oracle.max_threads())
    cfg = oracle.OracleConfig(n_slots=sub.n_slots, n_cells=C, n_attr=sub.n_attr, dt=sub.dt,
                              dv=sub.dv, b=sub.b, kernel=sub.kernel, adaptive=sub.adaptive,
                              n_threads=threads, seed=sub.seed)
    live = 0
    t0 = time.perf_counter()
    for s in range(steps):
        out = oracle.step(cfg, sub.xi, sub.v, sub.attrs, sub.cell_off, s)
        live += int(out["tallies"][0])
    dt = time.perf_counter() - t0
    return {"value": live / dt, "unit": "SD-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"first {C} cells ({sub.n_slots} SD slots) of the same workload, "
                      f"{steps} steps, OpenMP over cells; {dt:.1f} s"}


def copy_bandwidth_gbs(gib=1.0, reps=5):
    """Measured device-to-device copy bandwidth (read + write bytes over the
    median copy time): a second, attainable denominator for the roofline."""
    import numpy as np
    import torch

    n = int(gib * 2 ** 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    del src, dst
    return 2 * n * 8 / float(np.median(times)) / 1e9


def batched_vs_separate(state, tuning, n_cells=256, steps=5):
    """The first n_cells cells of the workload as one simulation (one launch
    per step and class) against the same cells as n_cells simulations of one
    cell each (their own launches), same launch shape; SD-steps/s of both."""
    import torch

    from paper_2103_17238_amd import binding as B
    from paper_2103_17238_amd import inputs as I

    C = min(n_cells, state.n_cells)

    def sub(c0, c1):
        a, b = int(state.cell_off[c0]), int(state.cell_off[c1])
        return I.State(state.xi[a:b].copy(), state.v[a:b].copy(),
                       state.attrs[:, a:b].copy(), state.cell_off[c0:c1 + 1] - a,
                       state.dt, state.dv, state.kernel, state.b, state.adaptive, state.seed)

    def timed(sims):
        for s in sims:
            t = B.sdm_get_tuning(s.handle)
            t.wave_class_mask, t.waves_per_cell = tuning["wave_class_mask"], tuning["waves_per_cell"]
            B.sdm_set_tuning(s.handle, t)
            s.step(1)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            for s in sims:
                s.step(1)
        e1.record()
        torch.cuda.synchronize()
        live = sum(B.sdm_stats(s.handle)["live_sd_steps"] for s in sims)
        per_step = live / (steps + 1)
        return per_step * steps / (e0.elapsed_time(e1) / 1e3)

    one = [B.Sim(sub(0, C))]
    batched = timed(one)
    for s in one:
        s.close()
    many = [B.Sim(sub(c, c + 1)) for c in range(C)]
    separate = timed(many)
    for s in many:
        s.close()
    return {"cells": C, "steps": steps, "batched_sd_steps_per_s": batched,
            "separate_sd_steps_per_s": separate, "speedup": batched / separate}


def fused_vs_single(state, tuning, steps=40):
    """The same steps from the same state taken one call per step (one launch
    per step and class, as timed for `value`) and in one call (the library
    fuses up to 8 steps per launch, each cell kept in LDS across them);
    milliseconds per step of both.  A separate figure, never the headline."""
    import torch

    from paper_2103_17238_amd import binding as B

    out = {}
    for name in ("single", "fused"):
        sim = B.Sim(state)
        t = B.sdm_get_tuning(sim.handle)
        t.wave_class_mask, t.waves_per_cell = tuning["wave_class_mask"], tuning["waves_per_cell"]
        B.sdm_set_tuning(sim.handle, t)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        if name == "single":
            for _ in range(steps):
                sim.step(1)
        else:
            sim.step(steps)
        e1.record()
        torch.cuda.synchronize()
        out[name] = e0.elapsed_time(e1) / steps
        sim.close()
    return {"steps": steps, "single_ms_per_step": out["single"],
            "fused_ms_per_step": out["fused"], "speedup": out["single"] / out["fused"]}


def serving_c5(n_requests, rate, baseline_prefix, small_budget_prefix, steps=600):
    """The serving configuration: Poisson arrivals at `rate` per second,
    n_sd = round(2^U(10, 16)), Golovin or geometric with probability 1/2,
    `steps` steps each, HBM-budget admission (80 % of free HBM), continuous
    batching with shared launches.  Beside it: the one-at-a-time baseline
    (FIFO, each request alone with its own launches) on a prefix of the same
    trace, and a 64 MiB budget that forces queueing on a prefix.  p50/p99 of
    completion - arrival, and SD-steps/s over the run's wall time."""
    import torch

    from paper_2103_17238_amd import inputs as I
    from paper_2103_17238_amd.serving import GpuExecutor, Server, serve_one_at_a_time

    reqs = I.serving_requests(n_requests, rate_per_s=rate, n_steps=steps)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    # warm-up: kernels loaded, allocator primed (its own short trace)
    warm = I.serving_requests(16, rate_per_s=4000.0, n_steps=20, rng_seed=99)
    Server(GpuExecutor(), budget_bytes=budget, steps_per_tick=SERVE_TICK).run(warm, I.request_state)
    note(f"serving: {n_requests} requests at {rate:g}/s")
    ex = GpuExecutor()
    stats = Server(ex, budget_bytes=budget, steps_per_tick=SERVE_TICK).run(reqs, I.request_state)
    ex.close()
    served = stats.summary()
    served.update(requests=n_requests, budget_bytes=budget,
                  device_busy_s=stats.device_busy_s)
    note(f"serving: p50 {served['p50_s']:.3f} s p99 {served['p99_s']:.3f} s; "
         f"one-at-a-time on the first {baseline_prefix}")
    base = serve_one_at_a_time(reqs[:baseline_prefix], I.request_state, GpuExecutor()).summary()
    base.update(requests=baseline_prefix, note=f"first {baseline_prefix} requests of the trace")
    note(f"serving: 64 MiB budget on the first {small_budget_prefix}")
    ex = GpuExecutor()
    small = Server(ex, budget_bytes=64 * 2 ** 20, steps_per_tick=SERVE_TICK).run(
        reqs[:small_budget_prefix], I.request_state)
    ex.close()
    tight = small.summary()
    tight.update(requests=small_budget_prefix, budget_bytes=64 * 2 ** 20,
                 note=f"first {small_budget_prefix} requests of the trace, 64 MiB budget")
    same = {"served_sd_steps_per_s": served["sd_steps_per_s"]}
    # the baseline's throughput on its prefix against the served run's over
    # the whole trace (both over wall time, arrivals included)
    same["one_at_a_time_sd_steps_per_s"] = base["sd_steps_per_s"]
    return {"workload": f"serving_{n_requests}_requests_{rate:g}_per_s_nsd_2^10..2^16_"
                        f"{steps}_steps",
            "served": served, "one_at_a_time": base, "budget_64mib": tight,
            "throughput": same}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="grid256",
                    choices=["grid256", "grid64", "golovin", "geometric", "serving", "displace",
                             "kinematic", "condense"])
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner (also when the environment sets SDM_TUNE=0)")
    ap.add_argument("--mask", type=lambda x: int(x, 0), default=None,
                    help="fixed class mask (skips the autotuner; e.g. 0x18)")
    ap.add_argument("--waves", type=int, default=None,
                    help="fixed waves per cell (with --mask)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batching-check", action="store_true",
                    help="skip the batched-vs-separate comparison on a sample of cells")
    ap.add_argument("--cpu-cells", type=int, default=65536)
    ap.add_argument("--cpu-steps", type=int, default=30)
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="before timing, copy a buffer of this size 3 times (a plain copy "
                         "kernel of known traffic, to scale rocprofv3 FETCH/WRITE_SIZE)")
    ap.add_argument("--serve-requests", type=int, default=1024)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-baseline", type=int, default=128,
                    help="requests replayed one at a time for the baseline")
    ap.add_argument("--serve-small-budget", type=int, default=1024,
                    help="requests of the trace served under a 64 MiB budget")
    ap.add_argument("--no-serving", action="store_true",
                    help="default workload: skip the serving measurement")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(cells would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2103_17238_amd import binding as B

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe_gib > 0:
        n = int(args.copy_probe_gib * 2 ** 30) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "serving":
        return serve_bench(args)
    if args.workload == "displace":
        return displace_bench(args)
    if args.workload == "condense":
        return condense_bench(args)
    if args.workload == "kinematic":
        return kinematic_bench(args)
    note(f"workload {args.workload}: building the input")
    state, workload = make_state(args.workload)
    host_state = state.copy()
    sim = B.Sim(state)
    stream = torch.cuda.current_stream()

    tuning_note = "default"
    if os.environ.get("SDM_TUNE", "1").strip() == "0":
        args.no_tune = True
    if args.mask is not None:
        t = B.sdm_get_tuning(sim.handle)
        t.wave_class_mask = args.mask
        t.waves_per_cell = args.waves if args.waves else t.waves_per_cell
        B.sdm_set_tuning(sim.handle, t)
        tuning_note = "fixed"
    elif not args.no_tune and args.workload not in ("grid256", "grid64"):
        # boxes: the library's autotuner (cell paths, bucket sizes) on a scratch copy
        scratch = B.workspace_tensor(B.sdm_autotune_scratch_bytes(sim.handle))
        t = B.sdm_autotune(sim.handle, scratch, trial_steps=3, stream=stream)
        B.sdm_set_tuning(sim.handle, t)
        del scratch
        tuning_note = "autotuned"
    elif not args.no_tune:
        # shapes: every cell in the 512-slot class (one launch per step), or
        # cells of <= 256 slots in their own class on a second stream (two
        # concurrent launches); waves per cell
        trials = []
        for mask in (0x10, 0x14, 0x18, 0x1C):
            for wpb in (1, 2):
                t = B.sdm_get_tuning(sim.handle)
                t.wave_class_mask, t.waves_per_cell = mask, wpb
                # time on a scratch copy so the measured state is untouched
                probe = B.Sim(host_state)
                B.sdm_set_tuning(probe.handle, t)
                probe.step(2)
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(4):  # one call per step, as timed below
                    probe.step(1)
                e1.record(stream)
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / 4
                probe.close()
                trials.append((ms, len(launched_classes(state, mask)), mask, wpb))
        best = min(trials)
        t = B.sdm_get_tuning(sim.handle)
        t.wave_class_mask, t.waves_per_cell = best[2], best[3]
        B.sdm_set_tuning(sim.handle, t)
        tuning_note = "autotuned"
    tuning = B.sdm_get_tuning(sim.handle).as_dict()
    note(f"tuning {tuning} ({tuning_note}); timing {args.steps} steps")

    sim.step(args.warmup)
    torch.cuda.synchronize()
    B.sdm_reset_status(sim.handle)
    torch.cuda.synchronize()

    # the timed region: K steps, one call each, HIP events on the launch
    # stream around all of them (events between steps would add their own
    # commands to the stream, which shows on steps of a few microseconds)
    K = args.steps
    e_start, e_end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    e_start.record(stream)
    for k in range(K):
        sim.step(1)
    e_end.record(stream)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t_wall
    total_ms = float(e_start.elapsed_time(e_end))
    stats = B.sdm_stats(sim.handle)
    flags = B.sdm_status_word(sim.handle)
    # spread of single steps: a separate pass with an event after every step
    Kd = min(K, 50)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(Kd + 1)]
    evs[0].record(stream)
    for k in range(Kd):
        sim.step(1)
        evs[k + 1].record(stream)
    torch.cuda.synchronize()
    per_step_ms = np.array([evs[k].elapsed_time(evs[k + 1]) for k in range(Kd)])
    copy_gbs = copy_bandwidth_gbs()

    live = stats["live_sd_steps"]
    coll = stats["colliding_pairs"]
    A = state.n_attr
    alg_bytes = (16 * live + 8 * (K * state.n_slots - live) + (32 + 32 * A) * coll
                 + 8 * state.n_cells * K)
    value = live / (total_ms / 1e3)
    cell_grid = args.workload in ("grid256", "grid64")
    mode = "adaptive" if state.adaptive else "plain"
    caps = launched_classes(state, tuning["wave_class_mask"])
    two = len(caps) > 1
    if not cell_grid:
        kernel_name = "whole_step"
    else:  # the step's cell launches (concurrent when there are several)
        kernel_name = " || ".join(f"k_cells<{c},{tuning['waves_per_cell']},{mode}>" for c in caps)
    achieved = alg_bytes / K / (total_ms / K / 1e3) / 1e9
    traffic = traffic_from_profiles("k_cells", args.workload, alg_bytes / K, tuning)
    subs = stats["cell_substeps"] / max(stats["cell_steps"], 1)
    valu = (valu_from_profiles(tuning, subs, total_ms / K / 1e3)
            if args.workload == "grid256" else None)
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "SD-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": total_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded generators: Poisson cell sizes, lognormal radii)",
        "config": {
            "workload": workload,
            "cells": state.n_cells,
            "sd_slots": state.n_slots,
            "n_attr": A,
            "kernel": "geometric" if state.kernel == 1 else "golovin",
            "adaptive": bool(state.adaptive),
            "parallelism": ("1 GPU, concurrent cell launches per step (two of the library's streams)" if two
                            else "1 GPU, one fused launch per step") if cell_grid else "1 GPU",
            "tuning": tuning,
            "tuning_source": tuning_note,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": kernel_name,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes / K,
            "avg_launch_ms": total_ms / K,
            # from the separate pass with an event after every step
            "median_step_ms_evented": float(np.median(per_step_ms)),
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
        "valu": valu,
        "stats": {"live_sd_steps": live, "colliding_pairs": coll,
                  "cell_substeps": stats["cell_substeps"], "cell_steps": stats["cell_steps"],
                  # the adaptive load the timed steps carried (it grows as drops
                  # grow): compare runs at the same value
                  "substeps_per_cell_step": stats["cell_substeps"] / max(stats["cell_steps"], 1),
                  "status_flags": flags, "wall_s": t_wall},
    }
    sim.close()
    note(f"{total_ms / K:.4f} ms per step; batching and fusion figures")
    if cell_grid and not args.no_batching_check:
        line["batching"] = batched_vs_separate(host_state, tuning)
        # the whole timed job (the same number of steps from the initial
        # state) in one call, beside one call per step
        line["fusion"] = fused_vs_single(host_state, tuning, steps=args.steps)
    if not args.no_cpu_baseline:
        note("cpu baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(host_state, args.cpu_cells, args.cpu_steps)
    else:
        line["cpu_baseline"] = None
    if args.workload == "grid256" and not args.no_serving:
        line["serving"] = serving_c5(4096, args.serve_rate, args.serve_baseline,
                                     args.serve_small_budget)
    print(json.dumps(line), flush=True)


def displace_bench(args):
    """Displacement + re-segmentation of the 256 x 256 grid (16.8 M slots, 6
    attributes) in the single-eddy flow (20 m cells, w_max 0.6 m/s, dt 1 s):
    one step = one sdm_displace call (four kernels) from one set of state
    buffers into the other.  Algorithmic bytes per step: one read and one
    write of every slot's xi, v, attributes and position ((32 + 8 A) x 2 =
    160 B per slot), the cell offsets (16 B per cell) and the face Courant
    numbers."""
    import numpy as np
    import torch

    from paper_2103_17238_amd import binding as B
    from paper_2103_17238_amd import inputs as I

    st = I.grid_256x256()
    nx = nz = 256
    cx, cz = I.single_eddy_courant(nx, nz)
    pos = I.positions(st.n_slots)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    bufs = [[dev(st.xi), dev(st.v), dev(st.attrs), dev(pos), dev(st.cell_off)]]
    bufs.append([torch.empty_like(t) for t in bufs[0]])
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = B.workspace_tensor(B.sdm_displace_workspace_bytes(nx, nz))
    dcx, dcz = dev(cx), dev(cz)
    stream = torch.cuda.current_stream()
    k = [0]

    def one():
        a, b = bufs[k[0] & 1], bufs[(k[0] + 1) & 1]
        B.sdm_displace(nx, nz, dcx, dcz, *a, *b, status, ws, stream)
        k[0] += 1

    for _ in range(args.warmup):
        one()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    w0 = time.perf_counter()
    for e0, e1 in evs:
        e0.record(stream)
        one()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    per = [e0.elapsed_time(e1) / 1e3 for e0, e1 in evs]
    total_s = evs[0][0].elapsed_time(evs[-1][1]) / 1e3
    ms = total_s / args.steps * 1e3
    n, A, C = st.n_slots, st.n_attr, nx * nz
    alg = 2 * (32 + 8 * A) * n + 16 * (C + 1) + 8 * ((nx + 1) * nz + nx * (nz + 1))
    avg = float(np.mean(per))
    copy_gbs = copy_bandwidth_gbs()
    achieved = alg / avg / 1e9
    flags = int(status.item()) & 0xFFFFFFFF
    line = {
        "metric": "super-droplet steps/s (displacement + cell re-segmentation)",
        "value": n * args.steps / total_s, "unit": "SD-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (Poisson cell sizes, uniform positions, single-eddy face Courant numbers)",
        "config": {"workload": "displace_grid256x256_single_eddy_A6", "cells": C, "sd_slots": n,
                   "n_attr": A, "courant_max": float(max(np.abs(cx).max(), np.abs(cz).max())),
                   "parallelism": "1 GPU, one wavefront per cell"},
        "roofline": {"bound": "hbm", "kernel": "sdm_displace (k_disp_count, k_disp_offsets, "
                                                 "k_disp_scan, k_disp_scatter)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": displace_traffic_from_profiles(),
                     "alg_bytes_per_launch": alg, "avg_launch_ms": avg * 1e3,
                     "median_launch_ms": float(np.median(per)) * 1e3, "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs},
        "status_flags": flags, "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        from oracle import displacement as D

        ref = (st.xi, st.v, st.attrs, pos, st.cell_off)
        steps = 3
        t0 = time.perf_counter()
        for _ in range(steps):
            ref = D.displace_resegment(nx, nz, cx, cz, *ref[:5])
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": n * steps / dt, "unit": "SD-steps/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"the whole grid ({n} slots), {steps} steps, numpy "
                                          f"(one thread); {dt:.1f} s"}
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def condense_bench(args):
    """Condensation on the 256 x 256 grid (16.8 M slots: the coalescence
    grid's layout and cloud mode plus an aerosol population, dry volume and
    kappa x dry volume as attributes 0 and 1, a third of the SDs haze) with
    per-cell ambient states (T, p, S drawn per cell): one step = one
    sdm_condensation_step call, dt = 1 s.  Algorithmic bytes per step: 40 B
    per live slot (xi, v, dry volume, kappa dry volume read; v written),
    8 B per dead slot (xi), 16 B per cell offset and 24 B of ambient state
    per cell."""
    import numpy as np
    import torch

    from paper_2103_17238_amd import binding as B
    from paper_2103_17238_amd import inputs as I

    st = I.condensation_grid()
    amb = I.ambient(st.n_cells)
    sim = B.Sim(st)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
    T, p, S = dev(amb["T"]), dev(amb["p"]), dev(amb["S"])
    cc = B.sdm_cond_config(1.0, 0, 1, 0, 0)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        B.sdm_condensation_step(sim.handle, cc, T, p, S, stream)
    torch.cuda.synchronize()
    K = args.steps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    e0.record(stream)
    for _ in range(K):
        B.sdm_condensation_step(sim.handle, cc, T, p, S, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    total_s = e0.elapsed_time(e1) / 1e3
    n, C = st.n_slots, st.n_cells
    live = int((st.xi > 0).sum())
    alg = 40 * live + 8 * (n - live) + 16 * (C + 1) + 24 * C
    achieved = alg / (total_s / K) / 1e9
    copy_gbs = copy_bandwidth_gbs()
    sim.close()
    line = {
        "metric": "super-droplet steps/s (condensation)",
        "value": live * K / total_s, "unit": "SD-steps/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": total_s / K * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (Poisson cell sizes, lognormal cloud and aerosol modes, per-cell "
                "ambient states)",
        "config": {"workload": "condense_grid256x256_aerosol_A6", "cells": C, "sd_slots": n,
                   "n_attr": st.n_attr, "dt_s": 1.0,
                   "parallelism": "1 GPU, one block per cell and 1024-slot part"},
        "roofline": {"bound": "hbm", "kernel": "k_condense", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": condense_traffic_from_profiles(), "alg_bytes_per_launch": alg,
                     "avg_launch_ms": total_s / K * 1e3, "copy_gbs": copy_gbs,
                     "frac_of_copy": achieved / copy_gbs},
        "valu": condense_valu_from_profiles(total_s / K),
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        from oracle import condensation as cd

        cells = 4096
        m = int(st.cell_off[cells])
        v = st.v[:m].copy()
        t0 = time.perf_counter()
        cd.step(st.xi[:m], v, st.attrs[:, :m], st.cell_off[:cells + 1], amb["T"][:cells],
                amb["p"][:cells], amb["S"][:cells], 1.0, 0, 1)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": int((st.xi[:m] > 0).sum()) / dt, "unit": "SD-steps/s",
                                "cores": 1, "kind": "oracle",
                                "sample": f"the first {cells} cells ({m} slots), one step, numpy "
                                          f"(one thread); {dt:.1f} s"}
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


def kinematic_bench(args):
    """Coalescence with displacement on the 256 x 256 grid: per step one
    sdm_displace (single-eddy flow), one sdm_rebind (the launch tables
    rewritten on the device for the new layout; one stream synchronisation)
    and one coalescence step.  Reports the three parts' times.  Default shape
    0x18 (cells in the 384-slot class): cells of about 256 slots keep room to
    grow, so the rebind stays on the device."""
    import numpy as np
    import torch

    from paper_2103_17238_amd import binding as B
    from paper_2103_17238_amd import inputs as I

    st = I.grid_256x256()
    nx = nz = 256
    cx, cz = I.single_eddy_courant(nx, nz)
    sim = B.Sim(st, any_layout=True)
    t = B.sdm_get_tuning(sim.handle)
    t.wave_class_mask = args.mask if args.mask is not None else 0x18
    t.waves_per_cell = args.waves if args.waves else 1
    B.sdm_set_tuning(sim.handle, t)
    kin = B.Kinematic2D(sim, nx, nz, cx, cz, I.positions(st.n_slots))
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        kin.step(stream)
        sim.step(1, stream)
    torch.cuda.synchronize()
    t_disp = t_rebind = t_coal = 0.0
    w0 = time.perf_counter()
    for _ in range(args.steps):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        kin.displace(stream)
        e[1].record(stream)
        h0 = time.perf_counter()
        kin.rebind(stream)  # device-side table refresh, one stream synchronisation
        t_rebind += time.perf_counter() - h0
        e2 = torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        sim.step(1, stream)
        e[2].record(stream)
        torch.cuda.synchronize()
        t_disp += e[0].elapsed_time(e[1]) / 1e3
        t_coal += e2.elapsed_time(e[2]) / 1e3
    wall = time.perf_counter() - w0
    stats = B.sdm_stats(sim.handle)
    line = {
        "metric": "super-droplet steps/s (displacement + re-plan + coalescence)",
        "value": st.n_slots * args.steps / wall, "unit": "SD-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (grid of the coalescence benchmark, uniform positions, single eddy)",
        "config": {"workload": "kinematic_grid256x256_single_eddy_geometric_adaptive_A6",
                   "cells": nx * nz, "sd_slots": st.n_slots,
                   "tuning": B.sdm_get_tuning(sim.handle).as_dict(),
                   "parallelism": "1 GPU"},
        "parts_ms_per_step": {"displace": t_disp / args.steps * 1e3,
                              "rebind": t_rebind / args.steps * 1e3,
                              "coalescence": t_coal / args.steps * 1e3},
        "status_flags": kin.flags(), "colliding_pairs": stats["colliding_pairs"],
        "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def serve_bench(args):
    """Continuous batching of box requests (Poisson arrivals) against the
    one-at-a-time baseline on a prefix of the same trace."""
    import torch

    from paper_2103_17238_amd import inputs as I
    from paper_2103_17238_amd.serving import GpuExecutor, Server, serve_one_at_a_time

    reqs = I.serving_requests(args.serve_requests, rate_per_s=args.serve_rate)
    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    ex = GpuExecutor()
    srv = Server(ex, budget_bytes=budget, steps_per_tick=SERVE_TICK)
    # warm-up: kernels compiled / loaded, allocator primed
    Server(GpuExecutor(), budget_bytes=budget, steps_per_tick=SERVE_TICK).run(reqs[:8], I.request_state)
    stats = srv.run(reqs, I.request_state)
    ex.close()
    served = stats.summary()
    base_reqs = reqs[: args.serve_baseline]
    bstats = serve_one_at_a_time(base_reqs, I.request_state, GpuExecutor())
    base = bstats.summary()
    alg = 16 * served["sd_steps"]
    line = {
        "metric": METRIC,
        "value": served["sd_steps_per_s"],
        "unit": "SD-steps/s",
        "n_gpus": 1,
        "steps": args.serve_requests,
        "warmup": 8,
        "ms_per_step": None,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (Poisson arrivals, log-uniform SD counts, seeded)",
        "config": {
            "workload": f"serving_{args.serve_requests}_requests_{args.serve_rate:g}_per_s_"
                        "nsd_2^10..2^16_600_steps",
            "parallelism": "1 GPU, continuous batching, one shared launch per step",
            "budget_bytes": budget,
            "steps_per_tick": SERVE_TICK,
        },
        "serving": served,
        "one_at_a_time": dict(base, requests=len(base_reqs)),
        "roofline": {
            "bound": "hbm", "kernel": "whole_step", "unit": "GB/s", "peak": HBM_PEAK_GBS,
            "achieved": alg / stats.device_busy_s / 1e9 if stats.device_busy_s else None,
            "frac": alg / stats.device_busy_s / 1e9 / HBM_PEAK_GBS if stats.device_busy_s
            else None,
            "traffic": None, "note": "16 B per live SD-step over device-busy time",
        },
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
