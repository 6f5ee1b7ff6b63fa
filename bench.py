"""Benchmark of the MI355X MHD update step (one JSON line on stdout).

A step is one full update of the method: the FP64 CFL max-reduction on the
device and the 12 operators F_x M_x F_y M_y F_z M_z M_z F_z M_y F_y M_x F_x
(dt kept on the device, as mhd_step_auto enqueues it).  The default
workload is the 256^3 FP32 run of seeded random-phase solenoidal turbulence
(P(k) ~ k^-4, 1 <= k <= 8, rms Mach 1, beta 1, B0 along z).  The state is
resident in HBM before the timed region starts.

Also reported:
 * roofline of the dominant kernel: algorithmic bytes per launch divided by
   its average duration, timed with HIP events on the solver's stream;
 * every operator kernel's average duration and bandwidth;
 * cpu_baseline: the FP64 CPU oracle on one full step of the same workload
   on the host cores (a bounded sample), scaled to Mcell-updates/s.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload turb256|ot512|ot1024|turb256-f64] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-updates/s/GPU + %HBM roofline; learned-coarse vs plain at equal L1"
HBM_PEAK_GBS = 8000.0

# algorithmic bytes per cell of one launch, in units of the element size:
# fluid reads rho, m (3), e and the three face fields it averages into the
# cell-centred field, writes rho, m, e; magnetic reads rho, m_d and b (3),
# writes b (3); the CFL reads the 8 fields.
ALG_WORDS = {"fluid": 8 + 5, "magnetic": 5 + 3, "cfl": 8}
STEP_WORDS = 6 * (8 + 8) + 8   # fused-sweep lower bound: 8r + 8w per sweep, + CFL

WORKLOADS = {
    "turb256": dict(n=256, prec="f32", ic="turbulence",
                    desc="random-phase solenoidal turbulence 256^3, P(k)~k^-4 (1<=k<=8), "
                         "rms Mach 1, beta 1, B0 || z, seed 2, FP32 state"),
    "turb256-f64": dict(n=256, prec="f64", ic="turbulence",
                        desc="random-phase solenoidal turbulence 256^3, FP64 state"),
    "ot512": dict(n=512, prec="f32", ic="orszag_tang",
                  desc="3D Orszag-Tang-type 512^3, FP32 state"),
    "ot1024": dict(n=1024, prec="f32", ic="orszag_tang",
                   desc="3D Orszag-Tang-type 1024^3, FP32 state (2 x 34.4 GB)"),
    "ensemble64": dict(n=0, prec="f32", ic="ensemble",
                       desc="64 periodic boxes, sizes drawn from {32,48,64,96,128,192,256}^3 "
                            "(seed 4), per-box turbulence with Mach in [0.5,3], beta in "
                            "[0.1,10]; one persistent launch per operator, per-box dt, "
                            "HIP-graph replay, autotuned launch shape; FP32"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_state_device(wl, torch):
    """Initial state as a device tensor (built on the host in numpy for
    sizes up to 512^3, field by field on the device above that)."""
    from paper_1004_1680_amd import inputs as I
    n = wl["n"]
    dt = torch.float64 if wl["prec"] == "f64" else torch.float32
    if wl["ic"] == "turbulence":
        s = I.turbulence((n, n, n), seed=2)
    else:
        s = I.orszag_tang((n, n, n))
    t = torch.from_numpy(s).to(device="cuda", dtype=dt)
    del s
    return t


def time_operator(S, op, d, dt, reps, stream, torch):
    """average duration (ms) of one launch of an operator kernel, HIP events
    on the solver's stream around `reps` back-to-back launches"""
    f = S.fluid if op == "fluid" else S.magnetic
    f(d, dt)                          # scalars already on the device
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        f(d, dt)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(wl):
    import oracle
    from paper_1004_1680_amd import inputs as I
    n = wl["n"]
    ncell = n ** 3
    if ncell > 256 ** 3:             # keep the sample bounded: 256^3 of the family
        n = 256
        ncell = n ** 3
    s = I.turbulence((n, n, n), seed=2) if wl["ic"] == "turbulence" else I.orszag_tang((n, n, n))
    oracle.load()
    t0 = time.perf_counter()
    dt, vmax = oracle.cfl(s)
    oracle.step(s, dt, vmax)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": round(ncell / el / 1e6, 4), "unit": "Mcell-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"1 full step (CFL + 12 operators) of the same initial state at {n}^3, "
                      f"FP64, OpenMP over pencils; {el:.2f} s wall"}


def run_ensemble(args, wl, torch, mhd):
    from paper_1004_1680_amd import autotune
    from paper_1004_1680_amd import inputs as I
    spec = I.ensemble_spec(nbox=64, seed=4)
    dims = [(n, n, n) for n, _, _, _ in spec]
    B = mhd.Batch(dims, prec=wl["prec"])
    ncell = B.ncell
    for i, (n, m, b, sd) in enumerate(spec):
        B.set_state(i, I.turbulence((n, n, n), seed=sd, mach=m, beta=b))
        log(f"[bench] box {i} ({n}^3, Mach {m:.2f}, beta {b:.2f}) resident")
    log("[bench] autotune")
    shape = autotune.tune_batch(B, args.cfl, use_cache=False)
    log(f"[bench] launch shape {shape}; warm-up")
    B.run(args.warmup, args.cfl, graph=True)
    B.status(raise_on_nonphysical=False)
    log(f"[bench] timing {args.steps} graph-replayed steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.run(args.steps, args.cfl, graph=True)
    B.status(raise_on_nonphysical=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    steps, nonphys = B.status(raise_on_nonphysical=False)
    ms_per_step = el * 1e3 / args.steps
    value = ncell * args.steps / el / 1e6
    step_alg = STEP_WORDS * 4 * ncell / (ms_per_step * 1e-3) / 1e9
    split = (6 * (ALG_WORDS["fluid"] + ALG_WORDS["magnetic"]) + ALG_WORDS["cfl"]) * 4 * ncell
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "boxes": len(dims), "cells": ncell, "cfl": args.cfl,
                   "launch": shape, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "whole step (split operator kernels)",
                     "achieved": round(split / (ms_per_step * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(split / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "step_hbm_frac": round(step_alg / HBM_PEAK_GBS, 4),
        "boxes_nonphysical": int((nonphys != 0).sum()),
    }
    B.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="turb256", choices=sorted(WORKLOADS))
    ap.add_argument("--cfl", type=float, default=0.7)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU decomposition is a design in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1004_1680_amd import mhd

    wl = WORKLOADS[args.workload]
    if wl["ic"] == "ensemble":
        return run_ensemble(args, wl, torch, mhd)
    n = wl["n"]
    ncell = n ** 3
    esize = 8 if wl["prec"] == "f64" else 4
    stream = torch.cuda.current_stream()
    log(f"[bench] workload {args.workload}: {wl['desc']}")
    S = mhd.Solver((n, n, n), prec=wl["prec"], stream=stream)
    st = make_state_device(wl, torch)
    S.set_state_tensor(st)
    del st
    torch.cuda.synchronize()
    log("[bench] state resident; warm-up")

    for _ in range(args.warmup):
        S.step_auto(args.cfl)
    S.status()
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        S.step_auto(args.cfl)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    nsteps_ok = S.status()
    ms_per_step = el * 1e3 / args.steps
    value = ncell * args.steps / el / 1e6

    # per-kernel durations (HIP events on the solver's stream); the state is
    # restored before each operator so that repeated launches with a frozen
    # dt never run away from the CFL condition
    log("[bench] per-kernel timing")
    saved = S.get_state_tensor()
    kern = {}
    for op in ("fluid", "magnetic"):
        for d in range(3):
            S.set_state_tensor(saved)
            dt = S.cfl_dt(args.cfl) * 0.25
            ms = time_operator(S, op, d, dt, args.kernel_reps, stream, torch)
            gbs = ALG_WORDS[op] * esize * ncell / (ms * 1e-3) / 1e9
            kern[f"{op}_{'xyz'[d]}"] = {"ms": round(ms, 5), "alg_GBs": round(gbs, 1)}
    # CFL (partial + final reduction)
    S.set_state_tensor(saved)
    del saved
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        S.cfl_dt(args.cfl)
    e1.record(stream)
    e1.synchronize()
    ms_cfl_sync = e0.elapsed_time(e1) / args.kernel_reps
    kern["cfl(sync)"] = {"ms": round(ms_cfl_sync, 5),
                         "alg_GBs": round(ALG_WORDS["cfl"] * esize * ncell / (ms_cfl_sync * 1e-3) / 1e9, 1)}
    # dominant kernel: largest time per step (each operator runs twice a step)
    dom = max((k for k in kern if k != "cfl(sync)"), key=lambda k: kern[k]["ms"])
    op = dom.split("_")[0]
    bytes_per_launch = ALG_WORDS[op] * esize * ncell
    achieved = bytes_per_launch / (kern[dom]["ms"] * 1e-3) / 1e9
    # measured HBM traffic of that kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE,
    # copy-calibrated), valid only while the kernel sources are unchanged
    traffic = None
    tpath = os.path.join(ROOT, "profiles", f"sweeps_{args.workload}_{wl['prec']}_hbm_traffic.md".replace("_f32_", "_fp32_").replace("_f64_", "_fp64_"))
    if not os.path.exists(tpath):
        tpath = os.path.join(ROOT, "profiles", f"sweeps_{args.workload}_hbm_traffic.md")
    from paper_1004_1680_amd.profile_summary import read_traffic
    tmap = read_traffic(tpath)
    tname = {"x": "{op}_x_kernel<{t}>", "y": "{op}_march_kernel<{t}, 1>",
             "z": "{op}_march_kernel<{t}, 2>"}[dom[-1]].format(
        op="fluid" if op == "fluid" else "mag", t="double" if esize == 8 else "float")
    if tname in tmap:
        traffic = tmap[tname]
    step_alg = STEP_WORDS * esize * ncell / (ms_per_step * 1e-3) / 1e9

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if wl["prec"] == "f64" else "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "grid": [n, n, n], "cfl": args.cfl,
                   "step": "CFL (FP64) + F_x M_x F_y M_y F_z M_z M_z F_z M_y F_y M_x F_x",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "alg_bytes_per_cell": ALG_WORDS[op] * esize},
        "step_hbm_frac": round(step_alg / HBM_PEAK_GBS, 4),
        "kernels": kern,
        "steps_completed": nsteps_ok,
    }
    S.close()
    if args.calibrate_copy:
        # a plain copy kernel of known size: 1 GiB read + 1 GiB written
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
