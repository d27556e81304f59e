"""Throughput of the coupled Maxwell-LLG step on one MI355X.

    python bench.py [--steps K] [--warmup W] [--start S] [--workload filter512] [--no-cpu]
    python bench.py --config-table     # oracle vs GPU on the paper-shaped grids

A step is one full coupled time step (Step 1 H-M sub-step, Step 2 E update
with the soft source, Step 3 H-M sub-step, probe sampling) on the
512 x 256 x 256 tunable-filter-like grid (33.5M cells, two ferrite bars,
16 lossy dielectric boxes), fields resident in HBM.  The run is first
advanced S untimed steps (default 600) so that the K timed steps fall in
the part of the 1000-step run where the port pulse drives the ferrite and
the H-M iteration takes its usual 2-3 iterations.  The FP64 run is the
headline; the FP32 bulk mode runs the same workload afterwards, and its
error against the FP64 oracle is taken on the 1000-step crop run whose
oracle results are stored in tests/golden.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2103_12819_amd", "csrc", f) for f in ("kernels.h", "hm_fused.h")]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "pmc_traffic.json")


def _kernels_h_sha256():
    """SHA-256 of the kernel sources (kernels.h, then hm_fused.h)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def measured_traffic(kernel, cells_per_launch):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (scaled by a plain copy's reading), or None when the
    kernel source has changed since they were taken or the record covers a
    different number of cells per launch."""
    try:
        rec = json.load(open(TRAFFIC_JSON))
        sha = _kernels_h_sha256()
    except (OSError, ValueError):
        return None
    if sha != rec.get("kernels_h_sha256"):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if k is None or k.get("cells_per_launch", k.get("faces_per_launch")) != cells_per_launch:
        return None
    return k["traffic_bytes_per_launch"]


# kernel names in the counter databases -> the names used here (h_far is the
# two-half-step instantiation of h_bulk)
_PMC_NAMES = (("e_update", "e_update<double"), ("h_far", "h_bulk<double, false, 2>"),
              ("h_bulk", "h_bulk<double, false, 1>"), ("h_half", "h_half_db<double"),
              ("hm_fused", "hm_fused<double"), ("hm_more", "hm_more<double"),
              ("hm_pre", "hm_pre<double"), ("hm_step", "hm_step<double"), ("hm_finish", "hm_finish<double"),
              ("hm_commit", "hm_commit<double"), ("probe_flux", "probe_flux<double"))


def write_traffic_record(pmc_dir, workload="filter512"):
    """Turn the four rocprofv3 counter runs under `pmc_dir` (FETCH_SIZE and
    WRITE_SIZE of `bench.py --steps 3 --warmup 1 --no-cpu --no-fp32
    --no-adjoint`, whose 600 set-up steps reach the part of the run where the
    H-M iteration takes 3 iterations, and of `bench.py --calibrate-copy`) into
    the traffic record and a markdown table; CPU only.  Counter values are
    KiB per dispatch."""
    import sqlite3

    def per_kernel(db):
        rows = sqlite3.connect(db).execute(
            "select kernel_name, counter_name, value from counters_collection").fetchall()
        acc = {}
        for name, _ctr, val in rows:
            acc.setdefault(name, []).append(float(val))
        return {n: (len(v), sum(v) / len(v)) for n, v in acc.items()}

    def one(ctr, kind):
        d = os.path.join(pmc_dir, f"{ctr}_{kind}")
        dbs = [os.path.join(d, f) for f in os.listdir(d) if f.endswith("_results.db")]
        if len(dbs) != 1:
            raise SystemExit(f"expected one *_results.db under {d}, found {dbs}")
        return per_kernel(dbs[0])

    copy_bytes = 1 << 30
    scale = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        c = one(ctr, "copy")
        (n, kib), = [v for k, v in c.items() if "copyBuffer" in k]
        scale[ctr] = copy_bytes / (kib * 1024)
    cfg = W.CONFIGS[workload]()
    tiles = json.load(open(os.path.join(pmc_dir, "tiles.json")))
    cells = {"e_update": cfg.cells, "h_far": tiles["far_cells"], "h_half": tiles["near_cells"]}
    faces = tiles.get("n_mag")
    fetch, write = one("FETCH_SIZE", "bench"), one("WRITE_SIZE", "bench")
    rec = {"kernels_h_sha256": _kernels_h_sha256(),
           "workload": f"{cfg.name} {cfg.n[0]}x{cfg.n[1]}x{cfg.n[2]} fp64",
           "command": "bench.py --steps 3 --warmup 1 --no-cpu --no-fp32 --no-adjoint",
           "fetch_scale": scale["FETCH_SIZE"], "write_scale": scale["WRITE_SIZE"], "kernels": {}}
    lines = ["| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read GB | write GB | "
             "algorithmic GB | traffic / algorithmic |", "|---|---|---|---|---|---|---|---|"]
    for short, pat in _PMC_NAMES:
        # one class may run as several instantiations (e_update over tile
        # pairs and over unpaired tiles), each dispatched once per launch of
        # the class: their per-dispatch means add up
        fk = sorted(k for k in fetch if pat in k)
        wk = sorted(k for k in write if pat in k)
        if not fk or len(fk) != len(wk) or len({fetch[k][0] for k in fk}) != 1:
            continue
        nf = fetch[fk[0]][0]
        f = sum(fetch[k][1] for k in fk)
        w = sum(write[k][1] for k in wk)
        rd, wr = f * 1024 * scale["FETCH_SIZE"], w * 1024 * scale["WRITE_SIZE"]
        ent = {"instantiation": " + ".join(k.split("(")[0] for k in fk), "dispatches": nf,
               "read_bytes_per_launch": int(rd), "write_bytes_per_launch": int(wr),
               "traffic_bytes_per_launch": int(rd + wr)}
        algo = "-"
        ratio = "-"
        b = None
        if short in cells:
            ent["cells_per_launch"] = cells[short]
            b = bytes_per_cell("h_bulk" if short == "h_half" else short, 8, tiles, cfg) * cells[short]
        elif short == "hm_fused" and faces:
            ent["faces_per_launch"] = faces
            b = hm_bytes_per_face(8) * faces
        if b is not None:
            ent["algorithmic_bytes_per_launch"] = int(b)
            algo = f"{b / 1e9:.3f}"
            ratio = f"{(rd + wr) / b:.3f}"
        rec["kernels"][short] = ent
        lines.append(f"| `{ent['instantiation']}` | {nf} | {f:.1f} | {w:.1f} | {rd / 1e9:.3f} | "
                     f"{wr / 1e9:.3f} | {algo} | {ratio} |")
    with open(TRAFFIC_JSON, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(f"fetch scale {scale['FETCH_SIZE']:.4f}, write scale {scale['WRITE_SIZE']:.4f}")
    print("\n".join(lines))


BULK_KERNELS = ("h_bulk", "h_far", "e_update")

# Algorithmic HBM bytes per cell-step of the whole step (compulsory traffic of
# the three phases, each reading its inputs once and writing its outputs
# once, on the 3.1 %-magnetic filter grid): FP64 and FP32 bulk storage.
STEP_BYTES_PER_CELL = {"fp64": 242.5, "fp32": 126.5}

# profile class -> kernel name, per sub-step form
_CLASS_NAMES_FUSED = {"hm_pre": "hm_fused", "hm_step": "hm_more", "h_bulk": "h_half"}


def fused_form(kern, steps):
    """The run took the fused H-M sub-step (one hm_fused and one hm_more per
    sub-step, no hm_finish / hm_commit)."""
    return kern["hm_finish"][1] == 0 and kern["hm_commit"][1] == 0 and kern["hm_pre"][1] == 2 * steps


def hm_bytes_per_face(s):
    """Algorithmic bytes per evolving magnetic face and sub-step of the H-M
    iteration with its iterations fused: H^s read and H written (s each),
    one E component read per face (three per cell), M^s read and M written
    (24 B each, FP64), the face constants (Ms, alpha, gamma: 24 B per cell,
    8 per face)."""
    return 3 * s + 56


def bytes_per_cell(kernel, s, tiles, cfg):
    """Algorithmic HBM bytes per cell for one launch of a bulk kernel with
    storage elements of s bytes: h_bulk and h_far read E(3) + H(3) and write
    H(3) (the fused pass reads and writes each value once); e_update reads
    E(3) + H(3) and the materials (eps_r and, when some cell conducts, sigma
    maps, or one byte of material id) and writes E(3)."""
    if kernel in ("h_bulk", "h_far"):
        return 9 * s
    has_sig = cfg.sigma is not None and bool(np.any(np.asarray(cfg.sigma) != 0))
    return 9 * s + (1 if tiles["materials"] > 0 else s * (2 if has_sig else 1))


def cells_per_launch(kernel, kern, tiles, cells, steps):
    """Cells one launch of `kernel` covers, averaged over the timed call of
    `steps` steps: e_update every cell; h_far the far tiles; h_bulk every
    tile in the call's first Step 1 and last Step 3, the near tiles in the
    other 2 * steps - 2 half steps."""
    if kernel == "e_update":
        return cells
    if kernel == "h_far":
        return tiles["far_cells"]
    total = 2 * cells + (2 * steps - 2) * tiles["near_cells"]
    return total / max(1, kern["h_bulk"][1])


def kernel_table(kern, info, cfg, s, steps):
    """Per profile class: time per step, launches per step, average launch,
    algorithmic bytes per launch and the achieved fraction of the HBM peak."""
    tiles = info["tiles"]
    cells = cfg.cells
    fused = fused_form(kern, steps)
    out = {}
    for k, (ms, n) in kern.items():
        if n == 0:
            continue
        name = _CLASS_NAMES_FUSED.get(k, k) if fused else k
        row = {"ms_per_step": round(ms / steps, 4), "launches_per_step": round(n / steps, 3),
               "avg_launch_ms": round(ms / n, 4)}
        b = None
        if k in BULK_KERNELS:
            nc = cells_per_launch(k, kern, tiles, cells, steps)
            row["cells_per_launch"] = nc if k != "h_bulk" else round(nc, 1)
            b = bytes_per_cell(k, s, tiles, cfg) * nc
        elif k == "hm_pre" and fused:
            row["faces_per_launch"] = info["n_mag"]
            b = hm_bytes_per_face(s) * info["n_mag"]
        if b is not None:
            gbs = b / (ms / n / 1e3) / 1e9
            row.update({"algorithmic_bytes_per_launch": int(round(b)), "GB/s": round(gbs, 1),
                        "frac": round(gbs / HBM_PEAK_GBS, 4)})
        out[name] = row
    return out


def fp32_vs_oracle():
    """The 128 x 64 x 64 crop of the filter grid, 1000 steps, FP32 bulk mode,
    against the FP64 oracle's stored run (tests/golden, written by a script
    that runs the oracle alone): every probe series and integral, and E, H
    and M - M0 on the stored sample of each field."""
    import gzip
    import paper_2103_12819_amd as mm
    path = os.path.join(ROOT, "tests", "golden", "filter_crop_oracle.json.gz")
    if not os.path.exists(path):
        return None
    gold = json.load(gzip.open(path, "rt"))
    cfg = W.filter_crop(seed=0, steps=gold["steps"])
    init = mm.from_config(cfg)
    sim = mm.from_config(cfg, precision="fp32")
    sim.step(cfg.steps)
    errs = {}
    groups = {"E": ("Ex", "Ey", "Ez"), "H": ("Hx", "Hy", "Hz"),
              "M-M0": tuple("M" + f + c for f in "xyz" for c in "xyz")}
    for gname, names in groups.items():
        num = den = 0.0
        for nm in names:
            ref = gold["fields"][nm]
            idx = np.array(ref["sample_idx"])
            r = np.array([float.fromhex(v) for v in ref["sample"]])
            got = sim.field(nm).reshape(-1)[idx]
            if gname == "M-M0":
                m0 = init.field(nm).reshape(-1)[idx]
                r, got = r - m0, got - m0
            num += float(np.sum((got - r) ** 2))
            den += float(np.sum(r ** 2))
        errs[gname] = float(f"{np.sqrt(num / den):.3e}")
    for pid, p in enumerate(gold["probes"]):
        r = np.array([float.fromhex(v) for v in p["series"]])
        S_ref = float.fromhex(p["sum"])
        sr, S = sim.probe(pid)
        errs[f"probe{pid}"] = float(f"{np.linalg.norm(sr - r) / np.linalg.norm(r):.3e}")
        errs[f"sum{pid}"] = float(f"{abs(S - S_ref) / max(abs(S_ref), cfg.dt * float(np.sum(np.abs(r)))):.3e}")
    sim.close()
    init.close()
    return {"workload": "filter crop 128x64x64, 1000 steps (FP32 bulk, FP64 M and accumulators)",
            "reference": "FP64 oracle, stored run", "fields_on": "512 stored samples per field",
            "rel_l2": errs}


def run_gpu(cfg, precision, steps, warmup, start):
    """Headline pass: `steps` steps bracketed by events on the library's
    stream, with no per-kernel events (each adds a gap to the stream, about
    0.1 ms per step in all).  Then a profiled pass of `steps` more steps with
    an event pair around every kernel launch: the per-kernel durations (the
    roofline of the dominant kernel and the breakdown) come from it."""
    import torch
    import paper_2103_12819_amd as mm

    sim = mm.from_config(cfg, precision=precision)
    info = sim.info()
    info["tiles"] = sim.tiles()
    stream = torch.cuda.current_stream()
    sim.step(start)      # set-up: advance the run to the window that is timed
    sim.step(warmup)
    sim.sync()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    sim.step(steps)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    iters = sim.stats()
    sim.profile(True)
    sim.profile_read()
    p0 = torch.cuda.Event(enable_timing=True)
    p1 = torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    sim.step(steps)
    p1.record(stream)
    kern = sim.profile_read()
    sim.profile(False)
    info["profiled_ms"] = p0.elapsed_time(p1)
    info["profiled_iters"] = sim.stats()[len(iters):]
    sim.sync()
    return sim, info, ms, wall, kern, iters


def run_adjoint_cost(steps=4000, ckpt=100):
    """Forward time of the 128x64x64 design grid (smooth random eps_r, Ms) over
    `steps` steps with checkpoints, then the time of mm_adjoint (segment
    recompute + reverse sweep) for the gradient of the integrated flux."""
    import torch
    import paper_2103_12819_amd as mm

    cfg = W.design128(seed=0, steps=steps)
    sim = mm.from_config(cfg)
    sim.enable_adjoint(ckpt)
    sim.step(5)          # warm-up of the launch path (part of the differentiated run)
    sim.sync()
    t0 = time.perf_counter()
    sim.step(steps - 5)
    sim.sync()
    t_fwd = time.perf_counter() - t0
    t1 = time.perf_counter()
    ge, gm = sim.adjoint(0)
    t_adj = time.perf_counter() - t1
    _, L = sim.probe(0)
    sim.close()
    torch.cuda.synchronize()
    per_fwd = t_fwd / (steps - 5)
    return {"workload": f"design128 128x64x64, {steps} steps, checkpoints every {ckpt}",
            "forward_ms_per_step": round(per_fwd * 1e3, 4),
            "adjoint_ms_per_step": round(t_adj / steps * 1e3, 4),
            "adjoint_over_forward": round((t_adj / steps) / per_fwd, 3),
            "loss": L, "max_abs_grad_eps_r": float(np.abs(ge).max()),
            "max_abs_grad_Ms": float(np.abs(gm).max())}


def run_scale(steps=500, ckpt=100, inner=34):
    """The 1024x512x512 grid (268M cells) in FP32: forward `steps` steps with
    two-level adjoint checkpoints, then the adjoint of the time-integrated
    flux; per-kernel times of the first 100 forward steps, the forward rate
    of the rest, and the peak device memory."""
    import torch
    import paper_2103_12819_amd as mm

    t0 = time.perf_counter()
    cfg = W.scale1024(seed=0, steps=steps)
    torch.cuda.reset_peak_memory_stats()
    sim = mm.from_config(cfg, precision="fp32")
    sim.enable_adjoint(ckpt, inner)
    sim.sync()
    setup = time.perf_counter() - t0
    tiles = sim.tiles()
    # per-kernel durations from the first 100 steps (event pair around every
    # launch); the forward rate from the other steps, without those events
    prof_steps = min(100, steps // 2)
    sim.profile(True)
    sim.profile_read()
    sim.step(prof_steps)
    kern = sim.profile_read()
    sim.profile(False)
    sim.sync()
    t1 = time.perf_counter()
    sim.step(steps - prof_steps)
    sim.sync()
    fwd = (time.perf_counter() - t1) * steps / (steps - prof_steps)
    t2 = time.perf_counter()
    ge, gm = sim.adjoint(0)
    adj = time.perf_counter() - t2
    _, L = sim.probe(0)
    info = sim.info()
    iters = sim.stats()
    sim.close()
    peak = torch.cuda.max_memory_allocated()
    cells = cfg.cells
    rl = {}
    for k in BULK_KERNELS:
        ms, n = kern[k]
        if n:
            nc = cells_per_launch(k, kern, tiles, cells, prof_steps)
            b = bytes_per_cell(k, 4, tiles, cfg) * nc
            rl[k] = {"avg_launch_ms": round(ms / n, 4), "GB/s": round(b / (ms / n / 1e3) / 1e9, 1)}
    return {"workload": f"scale1024 {cfg.n[0]}x{cfg.n[1]}x{cfg.n[2]} ({cells} cells), 3 ferrite inclusions, "
                        f"64 dielectric boxes, FP32, {steps} steps, checkpoints every {ckpt} (inner {inner})",
            "setup_s": round(setup, 1),
            "forward_ms_per_step": round(fwd / steps * 1e3, 4),
            "forward_Mcell_per_s": round(cells * steps / fwd / 1e6, 1),
            "adjoint_s": round(adj, 2),
            "adjoint_over_forward": round(adj / fwd, 3),
            "kernels_ms_per_step": {k: round(v[0] / prof_steps, 4) for k, v in kern.items()},
            "bulk_roofline": rl,
            "iterations_per_substep": {str(k): int(v) for k, v in zip(*np.unique(iters, return_counts=True))},
            "peak_device_GB": round(peak / 1e9, 1),
            "context_device_GB": round(info["device_bytes"] / 1e9, 1),
            "loss": L, "max_abs_grad_eps_r": float(np.abs(ge).max()),
            "max_abs_grad_Ms": float(np.abs(gm).max())}


def cpu_baseline(budget_s=15.0, cfg=None, label="the 128x64x64 crop of the filter grid", warm=True,
                 max_steps=2000):
    """The oracle on `cfg` (default: the 128x64x64 crop of the same grid), as
    many steps as fit in the time budget (at least 2).  warm: one step
    before the timing (allocation warm-up)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import from_config as oracle_from_config
    if cfg is None:
        cfg = W.filter_crop(seed=0, steps=1)
    sim = oracle_from_config(cfg)
    if warm:
        sim.step(1)
    n = 0
    t0 = time.perf_counter()
    while True:
        sim.step(1)
        n += 1
        el = time.perf_counter() - t0
        if (el > budget_s and n >= 2) or n >= max_steps:
            break
    return {"value": cfg.cells * n / el / 1e6, "unit": "Mcell-updates/s", "cores": 1,
            "kind": "oracle", "steps": n, "seconds": round(el, 2),
            "sample": f"oracle (numpy FP64, 1 thread) on {label}, {n} steps in {el:.1f} s"}


# Paper-shaped configurations and their step counts for the oracle-vs-GPU table
TABLE = [("slab64", lambda: W.slab64(), 200), ("filter_crop128", lambda: W.filter_crop(seed=0), 1000),
         ("waveguide256", lambda: W.waveguide256(seed=0), 2000), ("design128", lambda: W.design128(seed=0), 400)]


def run_table(budget_s, with_cpu):
    """One JSON line per configuration: the GPU (FP64) over the whole step
    count in one call, and with_cpu: the oracle over its first steps (as many
    as fit in budget_s, from step 0) with the GPU timed over the same steps."""
    import torch
    import paper_2103_12819_amd as mm

    def gpu_seconds(cfg, steps):
        sim = mm.from_config(cfg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        el = time.perf_counter() - t0
        iters = np.asarray(sim.stats())
        sim.close()
        return el, iters

    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    print(json.dumps({"host": {"cpu_model": model, "logical_cpus": os.cpu_count(),
                               "oracle_threads": 1, "device": torch.cuda.get_device_name(0)}}), flush=True)
    gpu_seconds(W.slab64(), 3)     # first launches (code objects) outside the table
    for name, make, steps in TABLE:
        cfg = make()
        el, iters = gpu_seconds(cfg, steps)
        row = {"config": name, "n": list(cfg.n), "cells": cfg.cells, "steps": steps,
               "gpu_fp64_s": round(el, 4), "gpu_fp64_Mcell_per_s": round(cfg.cells * steps / el / 1e6, 1),
               "mean_iterations_per_substep": round(float(iters.mean()), 2)}
        if with_cpu:
            cb = cpu_baseline(budget_s, cfg=make(), label=f"{name}, from step 0", warm=False, max_steps=steps)
            el_n, it_n = gpu_seconds(make(), cb["steps"])
            row["oracle"] = cb
            row["gpu_same_steps_Mcell_per_s"] = round(cfg.cells * cb["steps"] / el_n / 1e6, 1)
            row["gpu_over_oracle_same_steps"] = round(row["gpu_same_steps_Mcell_per_s"] / cb["value"], 1)
            row["mean_iterations_same_steps"] = round(float(it_n.mean()), 2)
        print(json.dumps(row), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="filter512")
    ap.add_argument("--start", type=int, default=600,
                    help="untimed steps before the warm-up: the default window lies in the part of "
                         "the 1000-step filter run where the port pulse drives the ferrite bars")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--scale", action="store_true",
                    help="also run the 1024x512x512 FP32 forward + two-level adjoint (about 2 minutes, "
                         "~250 GB of device memory)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy 5 times (scale reference for HBM counters)")
    ap.add_argument("--tiles-json", default=None,
                    help="write the workload's tile counts to this file and exit (GPU)")
    ap.add_argument("--config-table", action="store_true",
                    help="only time the paper-shaped configurations (GPU FP64, whole runs) and, without "
                         "--no-cpu, the oracle on each one's first steps (one JSON line each)")
    ap.add_argument("--traffic-record", default=None, metavar="PMC_DIR",
                    help="write profiles/pmc_traffic.json from the counter runs under PMC_DIR (CPU)")
    args = ap.parse_args()
    if args.traffic_record:
        write_traffic_record(args.traffic_record, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is described in the design notes only)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py: no HIP device", file=sys.stderr)
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        print(json.dumps({"calibrate_copy_bytes_read": src.numel() * 4, "bytes_written": dst.numel() * 4,
                          "launches": 6, "avg_ms": round(ms, 4),
                          "GB/s": round(2 * src.numel() * 4 / (ms / 1e3) / 1e9, 1)}), flush=True)
        return
    if args.config_table:
        run_table(30.0, not args.no_cpu)
        return
    if args.tiles_json:
        import paper_2103_12819_amd as mm
        sim = mm.from_config(W.CONFIGS[args.workload](), with_probes=False)
        json.dump(dict(sim.tiles(), n_mag=sim.info()["n_mag"]), open(args.tiles_json, "w"))
        sim.close()
        return

    cfg = W.CONFIGS[args.workload]()
    cells = cfg.cells
    print(f"[bench] {cfg.name} {cfg.n} fp64: start {args.start}, warmup {args.warmup}, steps {args.steps}",
          flush=True)
    sim64, info64, ms64, wall64, kern64, it64 = run_gpu(cfg, "fp64", args.steps, args.warmup, args.start)
    per_step = ms64 / args.steps
    value = cells * args.steps / (ms64 / 1e3) / 1e6
    table64 = kernel_table(kern64, info64, cfg, 8, args.steps)
    # dominant kernel (largest share of the step, every class) and its roofline
    dom = max(table64, key=lambda k: table64[k]["ms_per_step"])
    d = table64[dom]
    traffic = measured_traffic(dom, d.get("cells_per_launch", d.get("faces_per_launch")))
    step_bytes = STEP_BYTES_PER_CELL["fp64"] * cells
    print(f"[bench] fp64 {per_step:.3f} ms/step, {value:.1f} Mcell/s, kernels {kern64}", flush=True)

    out = {
        "metric": "coupled Mcell-updates/s (FP64; FP32 bulk mode alongside with its L2 error vs the FP64 oracle)",
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{cfg.name} {cfg.n[0]}x{cfg.n[1]}x{cfg.n[2]} ({cells} cells), "
                               "2 ferrite bars + 16 seeded lossy dielectric boxes, Jz port, PEC",
                   "cells": cells, "magnetic_faces": info64["n_mag"], "parallelism": "single GPU",
                   "timed_steps": [args.start + args.warmup, args.start + args.warmup + args.steps]},
        "profiled_pass": {"steps": [args.start + args.warmup + args.steps, args.start + args.warmup + 2 * args.steps],
                          "ms_per_step": round(info64["profiled_ms"] / args.steps, 4),
                          "note": "event pair around every kernel launch; kernel durations and roofline from here",
                          "iterations_per_substep": {str(k): int(v) for k, v in
                                                     zip(*np.unique(info64["profiled_iters"], return_counts=True))}},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": d["GB/s"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": d["frac"],
                     "traffic": traffic, "avg_launch_ms": d["avg_launch_ms"],
                     "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"],
                     "step": {"bytes_per_cell": STEP_BYTES_PER_CELL["fp64"],
                              "algorithmic_bytes_per_step": int(step_bytes),
                              "achieved": round(step_bytes / (per_step / 1e3) / 1e9, 1),
                              "frac": round(step_bytes / (per_step / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}},
        "tiles": info64["tiles"],
        "kernels_fp64": table64,
        "kernels_fp64_ms_per_step": {k: v["ms_per_step"] for k, v in table64.items()},
        "iterations_per_substep": {str(k): int(v) for k, v in
                                   zip(*np.unique(it64[-2 * args.steps:], return_counts=True))},
    }
    if not args.no_fp32:
        print("[bench] fp32 run", flush=True)
        sim32, info32, ms32, wall32, kern32, it32 = run_gpu(cfg, "fp32", args.steps, args.warmup, args.start)
        v32 = cells * args.steps / (ms32 / 1e3) / 1e6
        p32 = ms32 / args.steps
        sb32 = STEP_BYTES_PER_CELL["fp32"] * cells
        table32 = kernel_table(kern32, info32, cfg, 4, args.steps)
        out["fp32"] = {"value": round(v32, 2), "ms_per_step": round(p32, 4),
                       "roofline_step": {"bytes_per_cell": STEP_BYTES_PER_CELL["fp32"],
                                         "achieved": round(sb32 / (p32 / 1e3) / 1e9, 1),
                                         "frac": round(sb32 / (p32 / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
                       "kernels": table32,
                       "kernels_ms_per_step": {k: v["ms_per_step"] for k, v in table32.items()}}
        print(f"[bench] fp32 {p32:.3f} ms/step, {v32:.1f} Mcell/s", flush=True)
        sim32.close()
        print("[bench] fp32 error against the oracle (stored 1000-step crop run)", flush=True)
        out["fp32"]["error_vs_fp64_oracle"] = fp32_vs_oracle()
    sim64.close()
    if not args.no_adjoint:
        print("[bench] adjoint cost (design128)", flush=True)
        out["adjoint"] = run_adjoint_cost()
        print(f"[bench] adjoint {out['adjoint']}", flush=True)
    if args.scale:
        print("[bench] scale (1024x512x512 FP32, forward + adjoint)", flush=True)
        out["scale"] = run_scale()
        print(f"[bench] scale {out['scale']}", flush=True)
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", flush=True)
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
