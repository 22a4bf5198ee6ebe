#!/usr/bin/env python
"""Throughput of the boosted-frame laser-wakefield PIC step on one MI355X.

Workload (default): 2D boosted frame gamma = 13, 256 x 4096 cells, 16 macro-electrons per
cell at 1e18 cm^-3 (lab) with rigid ions, window pre-loaded with plasma (steady state of the
moving window), laser a0 = 2 w0 = 20 um through the lab-fixed antenna, CK2 solver with
Friedman theta = 0.1, 4 bilinear passes + compensation, 10-cell PML on every face, moving
window, FP32 fields/momenta with FP64 positions.  Inputs are synthetic and seeded.

One step = the whole PIC step of the library (Faraday, push, ions, antenna, filter, Ampere,
window/injection, periodic tile sort).  Launch configuration: the library's default 26 x 8
particle tile and a sort every 80 steps (the sort's amortised cost is inside the timed steps).
Prints ONE JSON line with the metric, the roofline of
the dominant kernel (gather/push/deposit, timed with HIP events on the library's stream) and
the FP64 CPU oracle timed on a bounded sample of the same workload.

Other workloads: --workload c3 (3D boosted frame gamma = 30, 128 x 128 x 1024, 8 ppc, 134 M
electrons + 134 M rigid ions, window pre-loaded, 8 x 8 x 10 tiles), c4 (the batched scan),
c5 (learned vs plain current filter).
"""
from __future__ import annotations

import argparse
import math
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E, published
PMC_FILE = os.path.join(ROOT, "profiles", "gpd_c2_pmc.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1009_2727_amd", "csrc", "bf_particles.hip")


GPD_SOURCES = ("bf_particles.hip", "bf_device.h", "bf_kernels.h")


def src_hash() -> str:
    """Hash of the sources the gather/push/deposit kernel is compiled from: stored counter
    totals are used only while it matches."""
    h = hashlib.sha256()
    for f in GPD_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1009_2727_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def bytes_model(ne: int, ni: int, nx: int, nz: int, real: int = 4):
    """Algorithmic HBM bytes.  Per electron (2D, FP32 momenta, FP64 positions): read x,z
    (16) + u (12) + w (4), write x,z,u (28) = 60 B.  Per rigid ion: read x, z0 (16) + w (4) =
    20 B.  Per interior cell and step: 51 words (Faraday+Friedman 12 read / 6 write, gather 9
    read, deposit flush 3 write, J clear 3, filter 3+3, Ampere 9 read / 3 write).  The
    gather/push/deposit kernel alone moves its particles plus the 9 staged field words and
    the 3 flushed current words per cell."""
    cells = nx * nz
    gpd = ne * (32 + 28) + cells * 12 * real
    step = ne * 60 + ni * 20 + cells * 51 * real
    return gpd, step


def bytes_model3(ne: int, ni: int, nx: int, ny: int, nz: int, real: int = 4):
    """Algorithmic HBM bytes of the 3D step.  Per electron (FP32 momenta, FP64 positions):
    read x,y,z (24) + u (12) + w (4), write x,y,z,u (36) = 76 B.  Per rigid ion: read x, y, z0
    (24) + w (4) = 28 B.  Per interior cell: Friedman 9 read / 6 write words, Faraday 6 / 6,
    gather 9 read, Ampere 9 / 6, filtered current 3 written, plus the FP64 current: cleared,
    deposited and read by the filter (3 x 8 B each).  The gather/push/deposit kernel alone moves
    its electrons, the 9 gathered field words and the 3 deposited FP64 words per cell."""
    cells = nx * ny * nz
    gpd = ne * 76 + cells * (9 * real + 24)
    step = ne * 76 + ni * 28 + cells * ((15 + 12 + 9 + 15 + 3) * real + 72)
    return gpd, step


def cpu_baseline3(args):
    """FP64 3D oracle on a bounded sample: a 32 x 32 x 64 slab of the same physics (8 ppc,
    pre-loaded, gamma = 30), a few steps, single thread."""
    import pic_inputs as pi
    from oracle.pic3 import Oracle3
    w = pi.c3(real="f64", nx=32, ny=32, nz=64, ppc=8, preload=True)
    o = Oracle3.from_workload(w)
    ne = len(o.particles(0)["id"])
    o.step(1)
    t0 = time.perf_counter()
    o.step(args.cpu_steps3)
    dt = time.perf_counter() - t0
    return {"value": ne * args.cpu_steps3 / dt, "unit": "electron pushes/s", "cores": 1, "kind": "oracle",
            "sample": f"32x32x64 slab of the same 3D workload, 8 ppc pre-loaded ({ne} electrons), "
                      f"{args.cpu_steps3} steps after one untimed step, FP64, single thread"}


def bench_3d(args):
    """The 3D boosted run (gamma = 30, 128 x 128 x 1024, 8 ppc, window pre-loaded) timed over
    the whole step; the roofline is that of the 3D gather/push/deposit kernel."""
    import torch
    import pic_inputs as pi
    from paper_1009_2727_amd import Sim
    w = pi.c3(real="f32", preload=True)
    cfg = w["config"]
    sim = Sim.from_workload(w, sort_every=args.sort_every, timers=True)
    stream = sim.stream
    sim.step(args.warmup)
    torch.cuda.synchronize()
    c0 = sim.counts()
    sim.timers(reset=True)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    sim.step(args.steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    status = sim.sync_status()
    c1 = sim.counts()
    timers = sim.timers(reset=True)
    ne = 0.5 * (c0[0] + c1[0])
    ni = 0.5 * (c0[1] + c1[1])
    ms_step = ms / args.steps
    gpd_bytes, step_bytes = bytes_model3(int(ne), int(ni), cfg["nx"], cfg["ny"], cfg["nz"])
    push_ms, push_n = timers["push"]
    gpd_ms = push_ms / max(push_n, 1)
    achieved = gpd_bytes / (gpd_ms / 1e3) / 1e9
    out = {
        "metric": "particle pushes/s",
        "value": ne * args.steps / (ms / 1e3),
        "unit": "electron pushes/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": w["name"], "grid": f"{cfg['nx']}x{cfg['ny']}x{cfg['nz']}", "ppc": 8,
                   "gamma_boost": cfg["gamma_boost"], "electrons": int(ne), "rigid_ions": int(ni),
                   "positions": "f64", "current_accumulation": "f64", "compact_every": sim.info()["sort_every"],
                   "status": status},
        "hbm_gbps_per_step": step_bytes / (ms_step / 1e3) / 1e9,
        "phases_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in timers.items()},
        "roofline": {"bound": "hbm", "kernel": "k3_gpd (gather + push + deposit)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": gpd_bytes, "avg_launch_ms": gpd_ms,
                     "limiter": "LDS: 8-byte current adds and gather reads, with bank conflicts "
                                "(rocprofv3 counters in profiles/)"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline3(args)
    return out


def cpu_baseline(args):
    """FP64 oracle on a bounded sample of the workload: a 256 x 256 slab of the same
    physics (16 ppc, pre-loaded), a few steps, single thread."""
    import pic_inputs as pi
    from oracle import Oracle
    w = pi.c2(real="f64", nx=256, nz=256, ppc=16, preload=True)
    o = Oracle.from_workload(w)
    ne = o.num_particles(0)
    o.step(1)       # first step outside the timing (allocations)
    t0 = time.perf_counter()
    o.step(args.cpu_steps)
    dt = time.perf_counter() - t0
    return {"value": ne * args.cpu_steps / dt, "unit": "particle pushes/s", "cores": 1,
            "kind": "oracle",
            "sample": f"256x256 slab of the same workload, 16 ppc pre-loaded ({ne} electrons), "
                      f"{args.cpu_steps} steps after one untimed step, FP64, single thread"}


def learned_filter_leg(args, w, plain_filter_ms):
    """The same workload and steps with the learned current filter (BF16 MFMA convolutions)
    in place of the bilinear one.  Its weights are the exact factorisation of the 4-pass +
    compensation filter, so the physics is the plain filter's and only the cost differs."""
    import torch
    import copy
    from paper_1009_2727_amd import Sim, bilinear_factor_params
    w2 = copy.deepcopy(w)
    w2["config"]["filter_kind"] = 1
    cfg = w2["config"]
    sim = Sim.from_workload(w2, sort_every=args.sort_every, timers=True)
    sim.set_learned_filter(bilinear_factor_params(cfg["filter_npass"], bool(cfg["filter_compensate"])))
    sim.step(args.warmup)
    torch.cuda.synchronize()
    c0 = sim.counts()
    sim.timers(reset=True)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(sim.stream)
    sim.step(args.steps)
    t1.record(sim.stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1)
    c1 = sim.counts()
    tm = sim.timers(reset=True)
    ne = 0.5 * (c0[0] + c1[0])
    return {"value": ne * args.steps / (ms / 1e3), "unit": "electron pushes/s",
            "ms_per_step": ms / args.steps, "filter_ms_per_step": tm["filter"][0] / args.steps,
            "plain_filter_ms_per_step": plain_filter_ms, "status": sim.sync_status(),
            "weights": "exact factorisation of the 4-pass + compensation filter"}


def bench_scan(args):
    """The batched scan: independent boosted runs of uneven grid, boost, density, time step
    and ppc.  Tiles and sort cadence per run class come from the autotuner.  The same runs are
    timed stepped one after another (one launch per phase and run) and as one batch (one
    persistent launch per heavy phase for all runs)."""
    import torch
    import pic_inputs as pi
    from paper_1009_2727_amd import Batch, Sim
    from paper_1009_2727_amd.autotune import Autotuner
    runs = pi.c4(nruns=args.c4_runs, scale=args.c4_scale)
    t0 = time.perf_counter()
    tuner = None if args.no_autotune else Autotuner()
    picks = tuner.tune_all(runs) if tuner else [{"tile": (26, 8), "sort_every": 80}] * len(runs)
    tune_s = time.perf_counter() - t0
    print(f"[scan] autotuned {len(runs)} runs in {tune_s:.1f} s", file=sys.stderr, flush=True)
    sims = [Sim.from_workload(w, tile=tuple(c["tile"]), sort_every=c["sort_every"]) for w, c in zip(runs, picks)]
    stream = torch.cuda.current_stream()
    print(f"[scan] created {len(sims)} runs", file=sys.stderr, flush=True)
    for s in sims:
        s.step(args.warmup)
    torch.cuda.synchronize()
    ne = sum(s.counts()[0] for s in sims)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for s in sims:
        s.step(args.steps)
    b.record(stream)
    torch.cuda.synchronize()
    single_ms = a.elapsed_time(b)
    batch = Batch(sims, stream=stream)
    batch.step(args.warmup)
    torch.cuda.synchronize()
    print("[scan] one-at-a-time and batched warm-up done", file=sys.stderr, flush=True)
    a.record(stream)
    batch.step(args.steps)
    b.record(stream)
    torch.cuda.synchronize()
    batch_ms = a.elapsed_time(b)
    status = [s.sync_status() for s in sims]
    ne2 = sum(s.counts()[0] for s in sims)
    ne_avg = 0.5 * (ne + ne2)
    value = ne_avg * args.steps / (batch_ms / 1e3)
    return {
        "metric": "particle pushes/s", "value": value, "unit": "electron pushes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": batch_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"batched scan of {len(runs)} independent 2D boosted runs (grid scale "
                               f"{args.c4_scale:g}), pre-loaded, CK2 + Friedman 0.1, 4+comp filter",
                   "electrons": int(ne_avg), "runs": len(runs), "status_ok": all(x == 0 for x in status)},
        "one_at_a_time": {"value": ne_avg * args.steps / (single_ms / 1e3), "ms_per_step": single_ms / args.steps},
        "batched_over_one_at_a_time": single_ms / batch_ms,
        "autotune": {"seconds": tune_s, "classes": {str(k): v for k, v in (tuner.cache.items() if tuner else [])}},
    }


def _axis_ez(sim, nx):
    return sim.field("Ez")[:, nx // 2 + sim.info()["pml_x"]]


def bench_learned_filter_study(args):
    """The learned filter against the plain 4-pass + compensation filter.
    - Training: Adam from a random start on (raw J, filtered J) patch pairs cut from three seeded
      runs of the wake family, plus band-limited probes at |k| > pi/2 whose targets are the plain
      filter's output (the spectral term).
    - Gain: max |G_learned - G_plain| for |k| < 4 k_p and over the whole band.
    - Growth: slope per step of ln(high-k E_z energy) in the boosted instability family with no
      filter, the plain filter and the learned one.
    - Wake error: on-axis E_z after 700 steps of the wake family (plain / learned) against an
      unfiltered FP64 run at twice the resolution, max |dE_z| / max |E_z,ref|."""
    import torch
    import pic_inputs as pi
    from paper_1009_2727_amd import Sim, bilinear_factor_params, filter_training as ft

    t0 = time.perf_counter()
    X, Y = [], []
    for s in (1, 2, 3):
        x, y = ft.current_pairs(pi.c5_wake(seed=1015 + s), steps=420, every=30, per_component=32, seed=s)
        X.append(x)
        Y.append(y)
    X, Y = np.concatenate(X), np.concatenate(Y)
    print(f"[c5] {len(X)} training pairs", file=sys.stderr, flush=True)
    probes = ft.band_probes(1024)
    lf, hist = ft.train(X, Y, probes, probe_weight=1.0, steps=args.c5_train_steps, lr=2e-3, batch=64,
                        log_every=max(args.c5_train_steps // 10, 1))
    params = lf.params.cpu().numpy()
    print(f"[c5] trained, loss {hist[-1][1]:.3g}", file=sys.stderr, flush=True)
    plain = bilinear_factor_params(4, True)

    w = pi.c5_wake()
    info = Sim.from_workload(w, laser=False).info()
    kp = math.sqrt(info["n0_norm"]) * w["config"]["dz_um"]    # plasma wavenumber in grid units
    gain = {"k_below_4kp": ft.gain_error(params, 4 * kp), "whole_band": ft.gain_error(params, math.pi),
            "plain_vs_exact_factorisation": ft.gain_error(plain, math.pi)}

    growth = {}
    for name, npass, p in (("none", 0, None), ("plain", 4, None), ("learned", 4, params)):
        g = pi.c5_growth(npass=npass, comp=1 if npass else 0)
        growth[name] = ft.growth_rate(g, p, steps=g["steps"], every=20)[0]
    print(f"[c5] growth {growth}", file=sys.stderr, flush=True)

    def wake(params_or_none):
        w2 = pi.c5_wake()
        if params_or_none is not None:
            w2["config"]["filter_kind"] = 1
        sim = Sim.from_workload(w2)
        if params_or_none is not None:
            sim.set_learned_filter(params_or_none)
        sim.step(w2["steps"])
        return _axis_ez(sim, w2["config"]["nx"])

    ez_plain, ez_learned = wake(None), wake(params)
    ref = pi.c5_wake(real="f64", refine=2)
    rsim = Sim.from_workload(ref)
    rsim.step(ref["steps"])
    ez_ref_f = _axis_ez(rsim, ref["config"]["nx"])
    # E_z sits at half rows: coarse (k + 1/2) d = mean of fine rows 2k + 1/2 and 2k + 3/2
    pz_c, pz_f = info["pml_z"], rsim.info()["pml_z"]
    nz = w["config"]["nz"]
    fine = ez_ref_f[pz_f:pz_f + 2 * nz]
    ez_ref = 0.5 * (fine[0::2] + fine[1::2])
    sl = slice(pz_c, pz_c + nz)
    scale = np.abs(ez_ref).max()
    err = {"plain": float(np.abs(ez_plain[sl] - ez_ref).max() / scale),
           "learned": float(np.abs(ez_learned[sl] - ez_ref).max() / scale)}
    equal = err["learned"] <= 1.1 * err["plain"] + 1e-3
    return {
        "metric": "learned vs plain filter at equal wake error", "data": "synthetic",
        "wake_error": err, "equal_wake_error": bool(equal),
        "growth_rate_per_step": growth,
        "growth_within_5pct_of_plain": bool(growth["learned"] <= growth["plain"] + 0.05 * abs(growth["plain"])),
        "gain_error": gain,
        "train": {"pairs": int(len(X)), "probes": int(len(probes[0])), "steps": args.c5_train_steps,
                  "loss_history": hist},
        "seconds": time.perf_counter() - t0,
    }


def read_pmc():
    if not os.path.exists(PMC_FILE):
        return None
    try:
        d = json.load(open(PMC_FILE))
    except Exception:
        return None
    if d.get("source_hash") != src_hash():
        return None          # kernels changed since the counters were taken
    return d


def summarize_pmc(fetch_dir: str, write_dir: str, copy_bytes: int, out: str):
    """Reduces two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) to per-launch HBM bytes
    of the gather/push/deposit kernel, scaled by what the counters read for a plain device
    copy of copy_bytes in the same process."""
    import csv

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(f) as fh:
                for r in csv.DictReader(fh):
                    if r.get("Counter_Name") == counter:
                        rows.append((r.get("Kernel_Name", ""), float(r["Counter_Value"])))
        return rows

    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = load(d, counter)
        gpd = [v for k, v in rows if "k_gpd" in k]
        copies = [v for k, v in rows if ("copy" in k.lower() or "elementwise" in k.lower()) and v > 0]
        if not gpd or not copies:
            raise SystemExit(f"no {counter} rows for k_gpd / copy in {d}")
        cal = max(copies) * 1024.0 / copy_bytes     # counter KiB vs true bytes
        res[counter] = {"gpd_kib_per_launch": sum(gpd) / len(gpd), "copy_kib": max(copies),
                        "calibration": cal,
                        "gpd_bytes_per_launch": sum(gpd) / len(gpd) * 1024.0 / cal}
    res["source_hash"] = src_hash()
    res["traffic_bytes_per_launch"] = (res["FETCH_SIZE"]["gpd_bytes_per_launch"]
                                       + res["WRITE_SIZE"]["gpd_bytes_per_launch"])
    json.dump(res, open(out, "w"), indent=1)
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--sort-every", type=int, default=80,
                    help="steps between particle sorts (the particle order lasts: the plasma drifts rigidly)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned-filter", action="store_true",
                    help="skip the second run with the learned (MFMA) current filter")
    ap.add_argument("--cpu-steps", type=int, default=16)
    ap.add_argument("--calib-copy-gib", type=float, default=0.0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_GIB"))
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5"], default="c2",
                    help="c2: the 256x4096 boosted run (default); c3: the 3D 128x128x1024 boosted run; "
                         "c4: the batched scan of independent boosted runs (persistent batched launch "
                         "vs one run at a time); c5: learned vs plain current filter")
    ap.add_argument("--cpu-steps3", type=int, default=8)
    ap.add_argument("--c4-runs", type=int, default=64)
    ap.add_argument("--c4-scale", type=float, default=1.0, help="grid scale of the scan's runs")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--c5-train-steps", type=int, default=3000)
    args = ap.parse_args()

    if args.summarize_pmc:
        f, wdir, gib = args.summarize_pmc
        summarize_pmc(f, wdir, int(float(gib) * 2 ** 30), PMC_FILE)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU: the boosted-frame PIC hot path is "
                          "measured on one MI355X (multi-GPU sharding is described, not built)",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import pic_inputs as pi
    from paper_1009_2727_amd import Sim

    if args.workload == "c4":
        print(json.dumps(bench_scan(args)), flush=True)
        return
    if args.workload == "c3":
        print(json.dumps(bench_3d(args)), flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(bench_learned_filter_study(args)), flush=True)
        return

    if args.calib_copy_gib > 0:
        n = int(args.calib_copy_gib * 2 ** 30)
        src = torch.empty(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    w = pi.c2(real="f32", preload=True)
    cfg = w["config"]
    sim = Sim.from_workload(w, sort_every=args.sort_every, timers=True)
    stream = sim.stream
    sim.step(args.warmup)
    torch.cuda.synchronize()
    c0 = sim.counts()
    sim.timers(reset=True)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    sim.step(args.steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms = t_start.elapsed_time(t_end)
    status = sim.sync_status()
    c1 = sim.counts()
    timers = sim.timers(reset=True)
    ne = 0.5 * (c0[0] + c1[0])
    ni = 0.5 * (c0[1] + c1[1])
    ms_step = ms / args.steps
    value = ne * args.steps / (ms / 1e3)
    gpd_bytes, step_bytes = bytes_model(int(ne), int(ni), cfg["nx"], cfg["nz"])
    push_ms, push_n = timers["push"]
    gpd_ms = push_ms / max(push_n, 1)
    achieved = gpd_bytes / (gpd_ms / 1e3) / 1e9
    pmc = read_pmc()
    traffic = pmc["traffic_bytes_per_launch"] if pmc else None

    out = {
        "metric": "particle pushes/s",
        "value": value,
        "unit": "electron pushes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "grid": f"{cfg['nx']}x{cfg['nz']}", "ppc": 16,
                   "gamma_boost": cfg["gamma_boost"], "electrons": int(ne), "rigid_ions": int(ni),
                   "positions": "f64", "sort_every": sim.info()["sort_every"],
                   "status": status},
        "hbm_gbps_per_step": step_bytes / (ms_step / 1e3) / 1e9,
        "phases_ms_per_step": {k: v[0] / max(args.steps, 1) for k, v in timers.items()},
        "roofline": {"bound": "hbm", "kernel": "k_gpd (gather + push + deposit)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": gpd_bytes, "avg_launch_ms": gpd_ms},
    }
    if not args.no_learned_filter:
        del sim
        torch.cuda.empty_cache()
        out["learned_filter"] = learned_filter_leg(args, w, timers["filter"][0] / max(args.steps, 1))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
