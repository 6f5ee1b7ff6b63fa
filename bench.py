"""Benchmark of the MI355X MHD update step (one JSON line on stdout).

A step is one full update of the method: the FP64 CFL max-reduction on the
device and the 12 operators F_x M_x F_y M_y F_z M_z M_z F_z M_y F_y M_x F_x
(dt kept on the device, as mhd_step_auto enqueues it).  In FP32 each
reverse-half pair (M_d F_d) runs as one fused kernel, so a step is 9
launches, and the CFL maximum of the next step is found by the last one.  The default
workload is the 512^3 FP32 run of the 3D Orszag-Tang-type state (the size at
which the HBM-roofline target is stated); ot1024, turb256 (seeded
random-phase solenoidal turbulence, P(k) ~ k^-4, 1 <= k <= 8, rms Mach 1,
beta 1, B0 along z) and the others are selectable.  The state is resident in
HBM before the timed region starts.

Also reported:
 * roofline of the dominant kernel: algorithmic bytes per launch divided by
   its average duration, timed with HIP events on the solver's stream;
 * every operator kernel's average duration and bandwidth;
 * cpu_baseline: the FP64 CPU oracle on full steps of the same initial
   state on the host cores (median of 3 one-step runs; states above 512^3
   are sampled at 512^3), scaled to Mcell-updates/s, with the CPU model and
   the threads used;
 * power: GPU board power sampled over a separate window of at least 2 s
   of the same steps (energy per step);
 * copy_ceiling: a plain streaming copy kernel of the library
   (mhd_stream_copy) on 2 GiB buffers, the practical HBM bandwidth that
   the sweep kernels are compared with.

The closure128 workload times the learned coarse step on a 128^3 grid (plain
step + BF16 MFMA network + gate + projection + guard) and a training step,
with the MFMA roofline of the network's forward pass; with --closure-eval it
also rolls out trained weights against the restricted 1024^3 solution and
plain 128^3 / 256^3 / 512^3 runs (learned vs plain at equal L1).

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
                       [--workload ot512|ot1024|turb256|turb256-f64|ensemble64|closure128]
                       [--no-cpu] [--closure-weights W.npz [--closure-eval]]
       python bench.py --precision-report all|2|3
           (FP32 and FP64 on the GPU against the FP64 oracle: 256^3 turbulence
            over 100 steps; 1024^3 FP32 against FP64 over 50 steps)
       python bench.py --size-sweep default|16,32,... [--sweep-prec f32|f64]
           (ms per step against n^3 with the paper's four criteria: code and
            fractional speed-up against the one-thread oracle, FLOPS and
            bandwidth fractions from the paper's per-cell counts)
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
BF16_PEAK_TFLOPS = 2500.0          # dense MFMA, MI355X
# closure network: 27 offsets x (8*32 + 32*32 + 32*8) multiply-adds per cell
CLOSURE_FLOP_PER_CELL = 2 * 27 * (8 * 32 + 32 * 32 + 32 * 8)

# algorithmic bytes per cell of one launch, in units of the element size:
# fluid reads rho, m (3), e and the three face fields it averages into the
# cell-centred field, writes rho, m, e; magnetic reads rho, m_d and b (3),
# writes b (3); the fused reverse pair (magnetic then fluid) reads and writes
# the 8 fields; the CFL reads the 8 fields.
ALG_WORDS = {"fluid": 8 + 5, "magnetic": 5 + 3, "pair": 8 + 8, "middle": 8 + 8, "cfl": 8}
STEP_WORDS = 6 * (8 + 8) + 8   # fused-sweep lower bound: 8r + 8w per sweep, + CFL

LIMITERS = {"vanleer": 0, "minmod": 1, "mc": 2, "superbee": 3}

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
    "closure128": dict(n=128, prec="f32", ic="closure",
                       desc="learned coarse step on 128^3 (8x restriction of 1024^3): plain FP32 "
                            "step + 3-layer 3^3 conv net 8->32->32->8 (BF16 MFMA, FP32 accumulate), "
                            "roughness gate, conservative projection, guard; Orszag-Tang-type "
                            "state (seed 200)"),
    "ensemble64": dict(n=0, prec="f32", ic="ensemble",
                       desc="64 periodic boxes, sizes drawn from {32,48,64,96,128,192,256}^3 "
                            "(seed 4), per-box turbulence with Mach in [0.5,3], beta in "
                            "[0.1,10]; one persistent launch per operator, per-box dt, "
                            "HIP-graph replay, autotuned launch shape; FP32"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


class PowerSampler:
    """Board power of the GPU over a timed region: the amdgpu hwmon reading
    (power1_average, else power1_input; microwatts) of the device's PCI
    function, sampled every `period` seconds on a host thread.  result() is
    None when no such file is readable."""

    def __init__(self, torch, period=0.01):
        import threading
        self.period = period
        self.path = self._find(torch)
        self.samples = []
        self._stop = threading.Event()
        self._thread = None

    @staticmethod
    def _find(torch):
        import glob
        try:
            p = torch.cuda.get_device_properties(torch.cuda.current_device())
            dev = f"/sys/bus/pci/devices/{p.pci_domain_id:04x}:{p.pci_bus_id:02x}:{p.pci_device_id:02x}.0"
        except Exception:
            return None
        for name in ("power1_average", "power1_input"):
            for f in sorted(glob.glob(f"{dev}/hwmon/hwmon*/{name}")):
                try:
                    with open(f) as fh:
                        if int(fh.read().strip()) > 0:
                            return f
                except (OSError, ValueError):
                    continue
        return None

    def _run(self):
        while not self._stop.is_set():
            try:
                with open(self.path) as fh:
                    self.samples.append(int(fh.read().strip()) * 1e-6)
            except (OSError, ValueError):
                pass
            self._stop.wait(self.period)

    def __enter__(self):
        import threading
        if self.path:
            self._thread = threading.Thread(target=self._run, daemon=True)
            self._thread.start()
        return self

    def __exit__(self, *exc):
        if self._thread:
            self._stop.set()
            self._thread.join()

    def result(self, seconds, steps, cells, what="GPU board power (hwmon), mean over the timed region"):
        if not self.samples:
            return None
        w = sum(self.samples) / len(self.samples)
        return {"avg_W": round(w, 1), "J_per_step": round(w * seconds / steps, 4),
                "Mcell_updates_per_J": round(cells * steps / (w * seconds) / 1e6, 2),
                "samples": len(self.samples), "window_s": round(seconds, 3), "steps": steps,
                "min_W": round(min(self.samples), 1), "max_W": round(max(self.samples), 1),
                "period_s": self.period, "source": self.path,
                "reading": os.path.basename(self.path) if self.path else None,
                "what": what}


def energy_window(S, cfl, cells, torch, seconds=2.0):
    """board power over a window of at least `seconds` of device-dt steps of
    the solver's current state (energy per step; the timed region of the
    throughput figure is too short for a stable power reading)"""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step_auto(cfl)
    torch.cuda.synchronize()
    per = max(time.perf_counter() - t0, 1e-4)
    steps = max(10, int(seconds / per) + 1)
    with PowerSampler(torch) as power:
        t0 = time.perf_counter()
        for _ in range(steps):
            S.step_auto(cfl)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
    S.status()
    return power.result(el, steps, cells, what=f"GPU board power (hwmon), mean over {steps} steps "
                                             "run for this reading after the timed region")


def copy_ceiling(torch, mhd, stream, gib=2, reps=10):
    """bandwidth of the library's plain streaming copy (mhd_stream_copy) and
    of torch's device copy on gib-GiB buffers: read + write bytes / time"""
    n = (gib << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    out = {}
    for name, fn in (("mhd_stream_copy", lambda: mhd.stream_copy(src, dst, stream)),
                     ("torch_copy", lambda: dst.copy_(src))):
        fn()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 4), "GBs": round(2 * 4 * n / (ms * 1e-3) / 1e9, 1)}
    assert torch.equal(src, dst)
    del src, dst
    torch.cuda.empty_cache()
    best = out["mhd_stream_copy"]["GBs"]
    return {"kernel": "mhd_stream_copy", "bytes_moved": 2 * 4 * n, "GBs": best,
            "frac": round(best / HBM_PEAK_GBS, 4), "torch_copy_GBs": out["torch_copy"]["GBs"],
            "what": f"{gib} GiB read + {gib} GiB written per copy, mean of {reps}"}


def cpu_info():
    """host CPU model string and the OpenMP threads the oracle uses"""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or avail
    return model, threads, avail


def make_state_device(wl, torch):
    """Initial state as a device tensor: turbulence is built on the host
    (numpy FFTs), the Orszag-Tang-type state directly on the device (equal
    to the host generator bit for bit; 1024^3 would need 69 GB of host
    memory in FP64)."""
    from paper_1004_1680_amd import inputs as I
    n = wl["n"]
    dt = torch.float64 if wl["prec"] == "f64" else torch.float32
    if wl["ic"] == "turbulence":
        s = I.turbulence((n, n, n), seed=2)
        t = torch.from_numpy(s).to(device="cuda", dtype=dt)
        del s
        return t
    return I.orszag_tang_torch((n, n, n), seed=0, dtype=dt)


def time_operator(S, op, d, dt, reps, stream, torch):
    """average duration (ms) of one launch of an operator kernel, HIP events
    on the solver's stream around `reps` back-to-back launches (op "pair":
    the fused reverse-half pair M_d F_d)"""
    if op == "pair":
        def f(d, dt):
            S.sweep(3 + d, dt)
    elif op == "pair+cfl":
        def f(d, dt):
            S.sweep(6, dt)
    elif op == "middle":
        def f(d, dt):
            S.sweep(7, dt)
    else:
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


def time_components(S, n, prec, stream, reps, torch, mhd):
    """restriction by 8 (fine -> (n/8)^3, the closure's coarsening) and the
    conservation / div b diagnostics: average duration (ms, HIP events on
    the solver's stream) and algorithmic bandwidth.  Restriction reads the 5
    cell fields and the face values lying on coarse faces (1 in 8 of each
    face field) and writes the 8 coarse fields; diagnostics read 8 fields."""
    esize = 8 if prec == "f64" else 4
    ncell = n ** 3
    out = {}
    r = 8
    if n % (4 * r) == 0:
        C = mhd.Solver((n // r,) * 3, prec=prec, stream=stream)
        S.restrict_to(C)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            S.restrict_to(C)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        alg = ((5 + 3 / r) * ncell + 8 * ncell / r ** 3) * esize
        out[f"restrict_{n}_to_{n // r}"] = {"ms": round(ms, 5), "alg_GBs": round(alg / (ms * 1e-3) / 1e9, 1),
                                            "alg_bytes": int(alg)}
        C.close()
    S.diag()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        S.diag()
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    out["diag(sync)"] = {"ms": round(ms, 5), "alg_GBs": round(8 * esize * ncell / (ms * 1e-3) / 1e9, 1)}
    return out


def step_launches(S, n, esize, fused, w32, lim=0, middle=False):
    """(kernel name, grid threads) of every sweep launch of one step of an
    n^3 grid, in the profiler's naming: the template arguments as the
    demangled names print them (the slope limiter; the fluid kernels' freezing
    speed, 0 for the step's; the 32-bit offsets flag of the x kernels last)"""
    t = "double" if esize == 8 else "float"
    tpr = n // 4
    rpw = max(1, 256 // tpr)
    xgrid = -(-(n * n) // rpw) * rpw * tpr

    def march(chunk):
        lanes = n * n * (n // chunk)
        return -(-lanes // 256) * 256

    fx = (f"fluid_x_kernel<{t}, false, {lim}, 0, {w32}>", xgrid)
    mx = (f"mag_x_kernel<{t}, {lim}, {w32}>", xgrid)
    fy = (f"fluid_march_kernel<{t}, 1, {w32}, {lim}, 0>", march(S.chunk(1)))
    my = (f"mag_march_kernel<{t}, 1, {w32}, {lim}>", march(S.chunk(1)))
    fz = (f"fluid_march_kernel<{t}, 2, {w32}, {lim}, 0>", march(S.chunk(2)))
    mz = (f"mag_march_kernel<{t}, 2, {w32}, {lim}>", march(S.chunk(2)))
    if middle:
        from paper_1004_1680_amd import mhd
        return [fx, mx, fy, my, fz,
                (f"magmagfluid_march_kernel<{t}, 2, {w32}, {lim}>", march(S.launch(mhd.MHD_TUNE_MIDDLE_CHUNK))),
                (f"magfluid_march_kernel<{t}, 1, {w32}, {lim}>", march(S.pair_chunk(1))),
                (f"magfluid_x_kernel<{t}, true, {lim}, {w32}>", xgrid)]
    if fused:
        return [fx, mx, fy, my, fz, mz,
                (f"magfluid_march_kernel<{t}, 2, {w32}, {lim}>", march(S.pair_chunk(2))),
                (f"magfluid_march_kernel<{t}, 1, {w32}, {lim}>", march(S.pair_chunk(1))),
                (f"magfluid_x_kernel<{t}, true, {lim}, {w32}>", xgrid)]
    return [fx, mx, fy, my, fz, mz, mz, fz, my, fy, mx, (f"fluid_x_kernel<{t}, true, {lim}, 0, {w32}>", xgrid)]


def cpu_baseline(wl, reps=3):
    """the oracle on the workload's initial state (states above 512^3, whose
    FP64 copies would not fit host memory, at 512^3 of the same family):
    `reps` full steps (CFL + 12 operators), each from that state, on all
    host threads; the median time"""
    import oracle
    from paper_1004_1680_amd import inputs as I
    n = min(wl["n"], 512)
    ncell = n ** 3
    s = I.turbulence((n, n, n), seed=2) if wl["ic"] == "turbulence" else I.orszag_tang((n, n, n))
    oracle.load()
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        dt, vmax = oracle.cfl(s)
        oracle.step(s, dt, vmax)
        times.append(time.perf_counter() - t0)
    el = float(np.median(times))
    model, threads, avail = cpu_info()
    same = "the same" if n == wl["n"] else f"a {n}^3 sample of the same family as the"
    out = {"value": round(ncell / el / 1e6, 4), "unit": "Mcell-updates/s", "cores": threads,
           "kind": "oracle", "cpu_model": model, "host_threads_available": avail,
           "omp_num_threads": os.environ.get("OMP_NUM_THREADS"),
           "sample": f"median of {reps} full steps (CFL + 12 operators), each from {same} "
                     f"initial state at {n}^3, FP64, OpenMP over pencils; wall "
                     + ", ".join(f"{t:.2f}" for t in times) + " s"}
    out["single_thread"] = cpu_baseline_single_thread(wl)
    return out


def cpu_baseline_single_thread(wl, n=128):
    """the oracle on one host thread, one full step of the same family at
    128^3 (a single-core reference like the paper's one-core x86 figure),
    in a child process started with OMP_NUM_THREADS=1"""
    import subprocess
    code = (
        "import sys, time\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import oracle\n"
        "from paper_1004_1680_amd import inputs as I\n"
        f"n = {n}\n"
        + ("s = I.turbulence((n, n, n), seed=2)\n" if wl["ic"] == "turbulence" else "s = I.orszag_tang((n, n, n))\n")
        + "oracle.load()\n"
        "t0 = time.perf_counter()\n"
        "dt, vmax = oracle.cfl(s)\n"
        "oracle.step(s, dt, vmax)\n"
        "print(time.perf_counter() - t0)\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=120, check=True)
        el = float(r.stdout.strip().splitlines()[-1])
    except (subprocess.SubprocessError, ValueError) as e:
        return {"error": str(e)[:200]}
    return {"value": round(n ** 3 / el / 1e6, 4), "unit": "Mcell-updates/s", "cores": 1,
            "sample": f"1 full step at {n}^3, FP64, one thread; {el:.2f} s wall"}


def run_ensemble(args, wl, torch, mhd):
    from paper_1004_1680_amd import autotune
    from paper_1004_1680_amd import inputs as I
    spec = I.ensemble_spec(nbox=64, seed=4)
    dims = [(n, n, n) for n, _, _, _ in spec]
    B = mhd.Batch(dims, prec=wl["prec"])
    B.set_limiter(LIMITERS[args.limiter])
    ncell = B.ncell
    for i, (n, m, b, sd) in enumerate(spec):
        B.set_state(i, I.turbulence((n, n, n), seed=sd, mach=m, beta=b))
        log(f"[bench] box {i} ({n}^3, Mach {m:.2f}, beta {b:.2f}) resident")
    log("[bench] autotune")
    shape = autotune.tune_batch(B, args.cfl, use_cache=False)
    if args.middle:
        B.set_launch(mhd.MHD_BATCH_MIDDLE, args.middle)
    shape["middle"] = B.launch(mhd.MHD_BATCH_MIDDLE)
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
    fused = shape["reverse"] == 1
    middle = fused and shape["middle"] == 1
    # bytes of the launches a step runs: 6 or 3 split operator pairs, 0 or 3
    # fused reverse pairs (each box's CFL maximum is found by the last launch);
    # the middle M_z M_z F_z in one launch drops the forward M_z's bytes
    nsplit = 3 if fused else 6
    split = (nsplit * (ALG_WORDS["fluid"] + ALG_WORDS["magnetic"]) + (6 - nsplit) * ALG_WORDS["pair"]
             - (ALG_WORDS["magnetic"] if middle else 0)) * 4 * ncell
    out = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "boxes": len(dims), "cells": ncell, "cfl": args.cfl,
                   "limiter": args.limiter, "launch": shape, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm",
                     "kernel": "whole step (" + ("5 forward operators, M_z M_z F_z in one launch, 2 fused reverse pairs"
                                                 if middle else "3 split pairs, 3 fused reverse pairs" if fused
                                                 else "12 split operators") + ", per-box CFL in the last launch)",
                     "achieved": round(split / (ms_per_step * 1e-3) / 1e9, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(split / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                     "traffic": None},
        "step_hbm_frac": round(step_alg / HBM_PEAK_GBS, 4),
        "boxes_nonphysical": int((nonphys != 0).sum()),
    }
    B.close()
    print(json.dumps(out), flush=True)


def run_closure(args, wl, torch, mhd):
    from paper_1004_1680_amd import closure_train as CT
    from paper_1004_1680_amd import inputs as I
    n = wl["n"]
    ncell = n ** 3
    stream = torch.cuda.current_stream()
    C = mhd.Solver((n, n, n), prec="f32", stream=stream)
    u0 = I.orszag_tang_torch((n, n, n), seed=200)
    C.set_state_tensor(u0)
    if args.closure_weights:
        cl, scales, meta = CT.load(args.closure_weights, (n, n, n), stream)
        wdesc = f"trained weights {os.path.basename(args.closure_weights)}"
    else:
        # untrained network with the scales of the state itself: the cost of a
        # step does not depend on the weights
        cl = mhd.Closure((n, n, n), stream=stream)
        cl.set_params(CT.init_params(0))
        st = cl.stats(u0, u0)
        mean = st[0] / ncell
        std = np.sqrt(np.maximum(st[1] / ncell - mean ** 2, 0.0)) + 1e-6
        cl.set_scales(mean, std, np.full(8, 1e-4), np.full(8, 1e-4))
        # one pooled mean roughness for all fields (fields that start flat,
        # like the density here, would otherwise get a huge gate)
        cl.set_gate(np.full(8, max(float(np.mean(st[4])) / ncell, 1e-30)))
        wdesc = "untrained weights (timing only)"
    log(f"[bench] closure {n}^3, {wdesc}; warm-up")
    for _ in range(args.warmup):
        cl.step(C, args.cfl)
    C.status()
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} learned steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        cl.step(C, args.cfl)
    C.status()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_learned = el * 1e3 / args.steps
    value = ncell * args.steps / el / 1e6
    # plain step at the same size, same state
    C.set_state_tensor(u0)
    for _ in range(args.warmup):
        C.step_auto(args.cfl)
    C.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        C.step_auto(args.cfl)
    C.status()
    torch.cuda.synchronize()
    ms_plain = (time.perf_counter() - t0) * 1e3 / args.steps
    # network forward pass (3 MFMA convolutions + gate + projection), HIP
    # events on the closure's stream
    u = C.get_state_tensor()
    out = torch.empty_like(u)
    cl.forward(u, out)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        cl.forward(u, out)
    e1.record(stream)
    e1.synchronize()
    ms_fwd = e0.elapsed_time(e1) / args.kernel_reps
    # training step (forward, loss, backward, Adam), no host synchronisation
    tgt = torch.zeros_like(u)
    saved = cl.params()
    cl.train_step(u, tgt, 1e-6, want_loss=False)
    e0.record(stream)
    for _ in range(args.kernel_reps):
        cl.train_step(u, tgt, 1e-6, want_loss=False)
    e1.record(stream)
    e1.synchronize()
    ms_train = e0.elapsed_time(e1) / args.kernel_reps
    cl.set_params(saved)
    tflops = CLOSURE_FLOP_PER_CELL * ncell / (ms_fwd * 1e-3) / 1e12
    out_line = {
        "metric": METRIC, "value": round(value, 2), "unit": "Mcell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_learned, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16/f32",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "grid": [n, n, n], "cfl": args.cfl, "weights": wdesc,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "kernel": "closure forward (conv 8->32, 32->32, 32->8 + gate + projection)",
                     "achieved": round(tflops, 1), "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(tflops / BF16_PEAK_TFLOPS, 4), "traffic": None,
                     "alg_flop_per_cell": CLOSURE_FLOP_PER_CELL},
        "plain_ms_per_step": round(ms_plain, 4),
        "forward_ms": round(ms_fwd, 4),
        "train_step_ms": round(ms_train, 4),
        "train_tflops": round(3 * CLOSURE_FLOP_PER_CELL * ncell / (ms_train * 1e-3) / 1e12, 1),
        "fallbacks": cl.fallbacks(), "reduced": cl.reduced(),
    }
    C.close()
    if args.closure_eval:
        if not args.closure_weights:
            raise SystemExit("--closure-eval needs --closure-weights")
        log("[bench] learned vs plain rollout against the restricted 1024^3 solution")
        res = CT.evaluate(cl, 1024, 8, 200, 200, torch, stream, args.cfl,
                          log=lambda m: log(m), checkpoints=[10, 25, 50, 100, 150, 200])
        out_line["learned_vs_plain"] = {k: res[k] for k in ("T", "compared_steps", "learned", "plain_128",
                                                             "plain_256", "plain_512", "plain_wall_at_equal_L1_s",
                                                             "speedup_at_equal_L1", "checkpoints") if k in res}
    cl.close()
    if not args.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out_line["cpu_baseline"] = cpu_baseline_closure()
    print(json.dumps(out_line), flush=True)


def cpu_baseline_closure():
    """the oracle's plain step and FP64 network forward (with gate and
    projection) on a 64^3 sample"""
    import oracle
    from oracle import closure as OC
    from paper_1004_1680_amd import inputs as I
    n = 64
    s = I.orszag_tang((n, n, n))
    oracle.load()
    ps = OC.init_params(0)
    u = s.reshape(8, -1)
    mean, std = u.mean(axis=1), u.std(axis=1) + 1e-6
    t0 = time.perf_counter()
    dt, vmax = oracle.cfl(s)
    s1 = oracle.step(s, dt, vmax)
    u1 = s1.reshape(8, -1)
    g = OC.gate(u1, np.ones(8), (n, n, n))
    OC.forward(OC.normalize(u1, mean, std), ps, np.full(8, 1e-4), (n, n, n), g=g)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    return {"value": round(n ** 3 / el / 1e6, 4), "unit": "Mcell-updates/s", "cores": cores,
            "kind": "oracle",
            "sample": f"1 learned step at {n}^3 (plain FP64 step + FP64 network forward, gate, "
                      f"projection); {el:.2f} s wall"}


FAMILIES = {"rho": [0], "m": [1, 2, 3], "e": [4], "b": [5, 6, 7]}


def family_l1(diff_sums, ref_sums):
    """relative L1 of a field family, pooled over its fields: sum |a - ref|
    / sum |ref| (a small member, such as b_z of the Orszag-Tang state, which
    starts at zero and grows from roundoff-sized values, does not dominate)"""
    return float(sum(diff_sums) / sum(ref_sums))


def family_errors(a, ref):
    """per field family: max |a - ref| / max |ref| and the relative L1"""
    out = {}
    for k, idx in FAMILIES.items():
        den = np.abs(ref[idx]).max()
        l1 = family_l1([float(np.abs(a[f] - ref[f]).sum()) for f in idx],
                       [float(np.abs(ref[f]).sum()) for f in idx])
        out[k] = {"max_rel": float(np.abs(a[idx] - ref[idx]).max() / den), "l1": l1}
    return out


def precision_config2(args, torch, mhd, checkpoints=(1, 10, 50, 100)):
    """256^3 random-phase solenoidal turbulence (rms Mach 1, beta 1, B0 || z,
    seed 2): FP32 GPU, FP64 GPU and the FP64 oracle over 100 steps (each
    with its own CFL time steps, device dt on the GPU), errors at the
    checkpoints"""
    import oracle
    from paper_1004_1680_amd import inputs as I
    n = (256, 256, 256)
    s = I.turbulence(n, seed=2)
    gpu = {}
    for prec in ("f64", "f32"):
        S = mhd.Solver(n, prec=prec)
        S.set_state(s)
        k, states = 0, {}
        t0 = time.perf_counter()
        for c in checkpoints:
            while k < c:
                S.step_auto(args.cfl)
                k += 1
            S.status()
            states[c] = (S.get_state(), S.time())
        log(f"[precision] config 2 {prec}: {k} steps in {time.perf_counter() - t0:.1f} s")
        S.close()
        gpu[prec] = states
    oracle.load()
    o, t, k = s, 0.0, 0
    rows = []
    t0 = time.perf_counter()
    for c in checkpoints:
        while k < c:
            dt, vmax = oracle.cfl(o, args.cfl)
            o = oracle.step(o, dt, vmax)
            t += 2.0 * dt
            k += 1
            if k % 5 == 0:
                log(f"[precision] config 2 oracle step {k} ({time.perf_counter() - t0:.0f} s)")
        g64, t64 = gpu["f64"][c]
        g32, t32 = gpu["f32"][c]
        rows.append({"step": c, "time_oracle": t, "time_f64": t64, "time_f32": t32,
                     "f64_vs_oracle": family_errors(g64, o), "f32_vs_oracle": family_errors(g32, o),
                     "f32_vs_f64": family_errors(g32, g64)})
    return {"workload": "random-phase solenoidal turbulence 256^3, P(k)~k^-4 (1<=k<=8), rms Mach 1, "
                        "beta 1, B0 || z, seed 2", "cfl": args.cfl, "checkpoints": rows}


def precision_config3(args, torch, mhd, checkpoints=(1, 10, 25, 50)):
    """1024^3 Orszag-Tang-type state, FP32 against FP64 on the GPU over 50
    steps (the oracle would need 137 GB of host memory per state).  The FP64
    state is read back as float32 through host memory (its rounding, 6e-8,
    is far below the differences measured), the FP32 state on the device;
    errors per field family at the checkpoints"""
    from paper_1004_1680_amd import inputs as I
    n = (1024, 1024, 1024)
    S64 = mhd.Solver(n, prec="f64")
    t = I.orszag_tang_torch(n, seed=0, dtype=torch.float64)
    S64.set_state_tensor(t)
    torch.cuda.synchronize()
    del t
    torch.cuda.empty_cache()
    S32 = mhd.Solver(n, prec="f32")
    t = I.orszag_tang_torch(n, seed=0, dtype=torch.float32)
    S32.set_state_tensor(t)
    torch.cuda.synchronize()
    del t
    torch.cuda.empty_cache()
    rows, k = [], 0
    el = {"f64": 0.0, "f32": 0.0}
    for c in checkpoints:
        for name, S in (("f64", S64), ("f32", S32)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(c - k):
                S.step_auto(args.cfl)
            S.status()
            torch.cuda.synchronize()
            el[name] += time.perf_counter() - t0
        k = c
        ref = S64.get_state_tensor(dtype=torch.float32).cpu()
        torch.cuda.empty_cache()
        g = S32.get_state_tensor()
        fams = {}
        for fam, idx in FAMILIES.items():
            mx, den, dsum, rsum = 0.0, 0.0, [], []
            for f in idx:
                r = ref[f].cuda()
                d = (g[f] - r).abs_()
                mx = max(mx, float(d.max()))
                den = max(den, float(r.abs().max()))
                dsum.append(float(d.sum(dtype=torch.float64)))
                rsum.append(float(r.abs().sum(dtype=torch.float64)))
                del r, d
            fams[fam] = {"max_rel": mx / den if den > 0 else mx, "l1": family_l1(dsum, rsum)}
        del g, ref
        torch.cuda.empty_cache()
        rows.append({"step": c, "time_f64": S64.time(), "time_f32": S32.time(), "f32_vs_f64": fams})
        log(f"[precision] config 3 step {c}: {fams}")
    S64.close()
    S32.close()
    return {"workload": "3D Orszag-Tang-type 1024^3", "cfl": args.cfl, "checkpoints": rows,
            "ms_per_step": {p: round(1e3 * el[p] / checkpoints[-1], 2) for p in el}}


def run_precision_report(args, torch, mhd):
    """FP32 and FP64 on the GPU against the oracle over many steps: config 2
    (256^3 turbulence, 100 steps, with the oracle) and config 3 (1024^3,
    50 steps, FP32 against FP64)"""
    rep = {"metric": "precision of the FP32 and FP64 GPU tiers over many steps", "unit": "relative error",
           "higher_is_better": False, "n_gpus": 1, "data": "synthetic"}
    which = args.precision_report
    if which in ("all", "2"):
        rep["config2_turb256_100_steps"] = precision_config2(args, torch, mhd)
    if which in ("all", "3"):
        rep["config3_ot1024_50_steps"] = precision_config3(args, torch, mhd)
    print(json.dumps(rep), flush=True)


SWEEP_SIZES = (16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
ORACLE_1CORE_SIZES = (16, 32, 64, 128)   # the sizes of the paper's one-core x86 column


def cpu_baseline_sizes(ic, sizes=ORACLE_1CORE_SIZES):
    """the oracle on one host thread, one full step at each size (the
    counterpart of the paper's one-core x86 times), in a child process
    started with OMP_NUM_THREADS=1; returns {n: ms}"""
    import subprocess
    code = (
        "import sys, time\n"
        f"sys.path.insert(0, {ROOT!r})\n"
        "import oracle\n"
        "from paper_1004_1680_amd import inputs as I\n"
        "oracle.load()\n"
        f"for n in {tuple(sizes)!r}:\n"
        + ("    s = I.turbulence((n, n, n), seed=2)\n" if ic == "turbulence"
           else "    s = I.orszag_tang((n, n, n))\n")
        + "    t0 = time.perf_counter()\n"
        "    dt, vmax = oracle.cfl(s)\n"
        "    oracle.step(s, dt, vmax)\n"
        "    print(n, (time.perf_counter() - t0) * 1e3, flush=True)\n")
    env = dict(os.environ, OMP_NUM_THREADS="1")
    try:
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                           timeout=300, check=True)
    except subprocess.SubprocessError as e:
        log(f"[sweep] one-core oracle failed: {str(e)[:200]}")
        return {}
    out = {}
    for line in r.stdout.splitlines():
        a = line.split()
        if len(a) == 2:
            out[int(a[0])] = float(a[1])
    return out


def run_size_sweep(args, torch, mhd):
    """Time per full step against box length n^3 (the paper's Fig. 1 and
    Table 3) with the four criteria of its section IV.A at each size."""
    from paper_1004_1680_amd import autotune
    from paper_1004_1680_amd import criteria as C
    prec = args.sweep_prec
    esize = 8 if prec == "f64" else 4
    sizes = SWEEP_SIZES if args.size_sweep == "default" else tuple(int(x) for x in args.size_sweep.split(","))
    stream = torch.cuda.current_stream()
    peak = C.FP64_VECTOR_PEAK_GFLOPS if prec == "f64" else C.FP32_VECTOR_PEAK_GFLOPS
    core_peak, core_desc = C.host_core_peak_gflops()
    one_core = {} if args.no_cpu else cpu_baseline_sizes("orszag_tang")
    recs = []
    for n in sizes:
        ncell = n ** 3
        log(f"[sweep] n={n} {prec}")
        S = mhd.Solver((n, n, n), prec=prec, stream=stream)
        if args.middle:
            S.set_launch(mhd.MHD_TUNE_MIDDLE, args.middle)
        st = make_state_device(dict(n=n, prec=prec, ic="orszag_tang"), torch)
        S.set_state_tensor(st)
        torch.cuda.synchronize()
        if not args.no_tune:
            autotune.tune_solver(S, args.cfl, use_cache=False)
        S.set_state_tensor(st)
        for _ in range(3):
            S.step_auto(args.cfl)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            S.step_auto(args.cfl)
        torch.cuda.synchronize()
        est = (time.perf_counter() - t0) / 3
        k = int(min(500, max(10, args.sweep_seconds / est)))
        # timed in blocks of at most 50 steps, each from the initial state
        # (restored outside the timed region; its first step makes a separate
        # CFL pass): the Orszag-Tang flow stays smooth over a block, while
        # hundreds of steps carry a small box into its current-sheet phase
        el, done = 0.0, 0
        while done < k:
            b = min(50, k - done)
            S.set_state_tensor(st)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(b):
                S.step_auto(args.cfl)
            torch.cuda.synchronize()
            el += time.perf_counter() - t0
            S.status()
            done += b
        S.close()
        del st
        torch.cuda.empty_cache()
        ms = el * 1e3 / k
        t1 = one_core.get(n)
        c = C.criteria(ms, t1, ncell, peak, C.HBM_PEAK_GBS, core_peak,
                       bytes_per_cell=esize * C.PAPER_FLOATS_PER_CELL_STEP)
        recs.append({"n": n, "steps": k, "ms_per_step": ms, "mcell_s": ncell * k / el / 1e6,
                     "alg_hbm_frac": STEP_WORDS * esize * ncell / (ms * 1e-3) / 1e9 / C.HBM_PEAK_GBS,
                     "oracle_1core_ms": t1, "criteria": c})
        log(f"[sweep] n={n}: {ms:.4f} ms/step over {k} steps")
    big = [r for r in recs if r["n"] >= args.sweep_slope_from]
    rec = {
        "command": "python3 bench.py " + " ".join(sys.argv[1:]),
        "workload": "3D Orszag-Tang-type state at each n^3",
        "dtype": prec,
        "sizes": recs,
        "slope_all": C.size_slope([r["n"] for r in recs], [r["ms_per_step"] for r in recs]) if len(recs) > 1 else None,
        "slope_from": args.sweep_slope_from,
        "slope_large": C.size_slope([r["n"] for r in big], [r["ms_per_step"] for r in big]) if len(big) > 1 else None,
        "peak_gflops": peak, "peak_gbs": C.HBM_PEAK_GBS,
        "host_core": core_desc, "host_core_gflops": core_peak,
        "units": "decimal (1e9) throughout; the paper's own totals use 2^30",
    }
    out = {"metric": "ms per full step vs box size; the paper's four criteria", "unit": "ms/step",
           "higher_is_better": False, "n_gpus": 1, "dtype": prec, "data": "synthetic",
           "config": {"workload": rec["workload"], "sizes": list(sizes), "cfl": args.cfl},
           "size_sweep": rec}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="ot512", choices=sorted(WORKLOADS))
    ap.add_argument("--cfl", type=float, default=0.7)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-tune", action="store_true", help="keep the built-in march chunks")
    ap.add_argument("--closure-weights", default=None, help="trained closure (.npz) for closure128")
    ap.add_argument("--closure-eval", action="store_true",
                    help="closure128: also evaluate learned vs plain against the 1024^3 solution")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    ap.add_argument("--limiter", default="vanleer", choices=sorted(LIMITERS),
                    help="slope limiter of the operators (the paper's: vanleer)")
    ap.add_argument("--middle", type=int, default=0, choices=(0, 1, 2),
                    help="M_z M_z F_z of a step: 1 one launch, 2 M_z and the z pair, 0 built-in")
    ap.add_argument("--row-group", type=int, default=None, metavar="ROWS",
                    help="x sweeps: most rows along y in one group of the tile order (0 built-in, ny linear)")
    ap.add_argument("--size-sweep", default=None, metavar="SIZES",
                    help="time a full step at each n^3 (comma list, or 'default': "
                         + ",".join(map(str, SWEEP_SIZES)) + ") with the paper's four criteria")
    ap.add_argument("--sweep-prec", default="f32", choices=("f32", "f64"))
    ap.add_argument("--sweep-seconds", type=float, default=0.5,
                    help="size sweep: timed seconds per size (10..500 steps)")
    ap.add_argument("--sweep-slope-from", type=int, default=128,
                    help="size sweep: smallest n of the large-box slope fit")
    ap.add_argument("--precision-report", default=None, choices=("all", "2", "3"),
                    help="FP32 / FP64 GPU against the oracle over many steps: 256^3 turbulence "
                         "for 100 steps (2), 1024^3 FP32 against FP64 for 50 steps (3)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(a multi-GPU decomposition is designed, not implemented)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1004_1680_amd import mhd

    if args.size_sweep:
        return run_size_sweep(args, torch, mhd)
    if args.precision_report:
        return run_precision_report(args, torch, mhd)
    wl = WORKLOADS[args.workload]
    if wl["ic"] == "ensemble":
        return run_ensemble(args, wl, torch, mhd)
    if wl["ic"] == "closure":
        return run_closure(args, wl, torch, mhd)
    n = wl["n"]
    ncell = n ** 3
    esize = 8 if wl["prec"] == "f64" else 4
    stream = torch.cuda.current_stream()
    log(f"[bench] workload {args.workload}: {wl['desc']}")
    S = mhd.Solver((n, n, n), prec=wl["prec"], stream=stream)
    lim = LIMITERS[args.limiter]
    S.set_limiter(lim)
    if args.middle:
        S.set_launch(mhd.MHD_TUNE_MIDDLE, args.middle)
    if args.row_group is not None:
        S.set_launch(mhd.MHD_TUNE_ROW_GROUP, args.row_group)
    st = make_state_device(wl, torch)
    S.set_state_tensor(st)
    del st
    torch.cuda.synchronize()
    if not args.no_tune:
        from paper_1004_1680_amd import autotune
        chunks = autotune.tune_solver(S, args.cfl, use_cache=False)
        log(f"[bench] autotuned march chunks: {chunks}")
    log("[bench] state resident; warm-up")

    for _ in range(args.warmup):
        S.step_auto(args.cfl)
    S.status()
    torch.cuda.synchronize()

    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    with PowerSampler(torch) as power:
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
    fused = S.reverse() == 1
    middle = S.launch(mhd.MHD_TUNE_MIDDLE) == 1
    ops = ("fluid", "magnetic", "pair") if fused else ("fluid", "magnetic")
    for op in ops:
        for d in range(3):
            if op == "pair" and d == 0:
                # the x pair runs once a step, as the last launch, with the
                # fused CFL epilogue (sweep code 6)
                S.set_state_tensor(saved)
                dt = S.cfl_dt(args.cfl) * 0.25
                ms = time_operator(S, "pair+cfl", 0, dt, args.kernel_reps, stream, torch)
                gbs = ALG_WORDS["pair"] * esize * ncell / (ms * 1e-3) / 1e9
                kern["pair_x+cfl"] = {"ms": round(ms, 5), "alg_GBs": round(gbs, 1)}
            S.set_state_tensor(saved)
            dt = S.cfl_dt(args.cfl) * 0.25
            ms = time_operator(S, op, d, dt, args.kernel_reps, stream, torch)
            gbs = ALG_WORDS[op] * esize * ncell / (ms * 1e-3) / 1e9
            kern[f"{op}_{'xyz'[d]}"] = {"ms": round(ms, 5), "alg_GBs": round(gbs, 1)}
    if middle:
        # M_z M_z F_z in one launch (sweep code 7), run once a step in place of
        # M_z and the z pair
        S.set_state_tensor(saved)
        dt = S.cfl_dt(args.cfl) * 0.25
        ms = time_operator(S, "middle", 2, dt, args.kernel_reps, stream, torch)
        kern["middle_z"] = {"ms": round(ms, 5),
                            "alg_GBs": round(ALG_WORDS["middle"] * esize * ncell / (ms * 1e-3) / 1e9, 1)}
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
    components = time_components(S, n, wl["prec"], stream, min(args.kernel_reps, 10), torch, mhd)
    log("[bench] energy window")
    energy = energy_window(S, args.cfl, ncell, torch)
    # dominant kernel: largest time per step (with fused reverse pairs every
    # kernel runs once a step, otherwise each operator runs twice)
    skip = {"cfl(sync)"} | ({"pair_x"} if fused else set()) | ({"magnetic_z", "pair_z"} if middle else set())
    dom = max((k for k in kern if k not in skip), key=lambda k: kern[k]["ms"])
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
    kname = {"fluid": "fluid", "magnetic": "mag", "pair": "magfluid", "middle": "magmagfluid"}[op]
    # march kernels carry their addressing (32-bit byte offsets when a field
    # is under 4 GiB) as a third template argument
    w32 = "true" if ncell * esize <= 2 ** 32 else "false"
    axis = dom.split("_")[1][0]
    cfl_x = dom.endswith("+cfl")
    # the profiler's names (as in step_launches): the slope limiter, the
    # fluid kernels' freezing speed (0), the x kernels' 32-bit offsets flag
    t = "double" if esize == 8 else "float"
    cf = "true" if cfl_x else "false"
    if axis == "x":
        tname = {"fluid": f"fluid_x_kernel<{t}, {cf}, {lim}, 0, {w32}>",
                 "magnetic": f"mag_x_kernel<{t}, {lim}, {w32}>",
                 "pair": f"magfluid_x_kernel<{t}, {cf}, {lim}, {w32}>"}[op]
    else:
        dd = 1 if axis == "y" else 2
        tname = f"{kname}_march_kernel<{t}, {dd}, {w32}, {lim}" + (", 0>" if op == "fluid" else ">")
    if tname in tmap:
        traffic = tmap[tname]
    step_alg = STEP_WORDS * esize * ncell / (ms_per_step * 1e-3) / 1e9
    # measured HBM bytes of a whole step: the profiled traffic of each launch
    # the step makes, at its launch grid (null if any is missing)
    step_traffic = None
    if tmap:
        tot = 0
        for name, grid in step_launches(S, n, esize, fused, w32, lim, middle):
            b = tmap.get(f"{name} @ {grid}", tmap.get(name))
            if b is None:
                tot = None
                break
            tot += b
        step_traffic = tot

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
                   "step": ("CFL (FP64) + F_x M_x F_y M_y F_z M_z M_z F_z M_y F_y M_x F_x; "
                            + ("8 launches: M_z M_z F_z in one, the reverse pairs M_y F_y, M_x F_x "
                               "fused, CFL in the last" if middle else
                               "9 launches: each reverse pair M_d F_d fused, CFL in the last"
                               if fused else "12 launches")),
                   "limiter": args.limiter,
                   "march_chunks": [S.chunk(1), S.chunk(2)],
                   "pair_chunks": [S.pair_chunk(1), S.pair_chunk(2)] if fused else None,
                   "middle_chunk": S.launch(mhd.MHD_TUNE_MIDDLE_CHUNK) if middle else None,
                   "x_row_group": S.launch(mhd.MHD_TUNE_ROW_GROUP),
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "alg_bytes_per_cell": ALG_WORDS[op] * esize},
        "step_hbm_frac": round(step_alg / HBM_PEAK_GBS, 4),
        "step_traffic": None if step_traffic is None else {
            "bytes": int(step_traffic),
            "achieved_GBs": round(step_traffic / (ms_per_step * 1e-3) / 1e9, 1),
            "frac": round(step_traffic / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
        "kernels": kern,
        "components": components,
        "power": energy,
        "power_timed_region": power.result(el, args.steps, ncell),
        "steps_completed": nsteps_ok,
    }
    S.close()
    log("[bench] copy ceiling")
    out["copy_ceiling"] = copy_ceiling(torch, mhd, stream)
    out["step_frac_of_copy"] = round(step_alg / out["copy_ceiling"]["GBs"], 4)
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
