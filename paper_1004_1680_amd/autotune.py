"""Launch-shape autotuner for the MHD kernels.

Results never depend on the launch shape (the tests check this bit for bit),
only the time does.  The tuner times a few steps of each candidate shape on
the live state and keeps the fastest; choices are cached in a JSON file
(``$MHD_AUTOTUNE_CACHE``, default ``~/.cache/mhd_autotune.json``) keyed by
device, problem and precision.

* single grid: the march chunk length along y and z of the single
  operators and of the fused reverse-half pairs, and along z of the fused
  middle of a step (M_z M_z F_z) when it is on (the x sweeps hold whole
  rows and have no shape to choose);
* batched ensemble: the persistent grid of the operator launches, the
  target march chunk, whether the reverse-half pairs run fused (fused
  pairs pay a 13-cell warm-up per chunk, heavy for small boxes) and, fused,
  their chunk and whether the middle M_z M_z F_z runs as one launch.

The state is saved before tuning and restored afterwards, so tuning does not
advance the simulation.
"""
import json
import os
import time

from . import mhd

CACHE = os.environ.get("MHD_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "mhd_autotune.json"))


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    try:
        os.makedirs(os.path.dirname(CACHE), exist_ok=True)
        tmp = CACHE + ".tmp"
        with open(tmp, "w") as f:
            json.dump(db, f, indent=1, sort_keys=True)
        os.replace(tmp, CACHE)
    except OSError:
        pass


def _device_tag():
    try:
        import torch
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "gfx950"


def divisors(n, lo=8):
    return [d for d in range(lo, n + 1) if n % d == 0]


def chunk_candidates(n):
    """divisors of n near powers of two, plus the whole pencil"""
    out = set()
    for p in (16, 32, 64, 128, 256, 512, 1024):
        ds = [d for d in divisors(n) if d <= p]
        if ds:
            out.add(max(ds))
    out.add(n)
    return sorted(out)


def tune_solver(S, cfl=0.7, steps=4, repeats=2, use_cache=True):
    """Choose the march chunks of a Solver along y and z: those of the single
    operators and, when the reverse-half pairs run fused, those of the fused
    pairs (one parameter at a time, the others held).  Each candidate is
    timed over `steps` steps, best of `repeats`.  Returns {key: chunk} with
    keys (kind, axis), kind "op" or "pair"."""
    fused = S.reverse() == 1
    middle = S.launch(mhd.MHD_TUNE_MIDDLE) == 1
    kinds = ("op", "pair") if fused else ("op",)
    if middle:
        kinds += ("mid",)
    key = (f"{_device_tag()}:single:{S.n[0]}x{S.n[1]}x{S.n[2]}:"
           f"{'f64' if S.prec == mhd.MHD_F64 else 'f32'}:{'fused' if fused else 'separate'}"
           f"{':middle' if middle else ''}")
    setter = {"op": S.set_chunk, "pair": S.set_pair_chunk,
              "mid": lambda axis, ch: S.set_launch(mhd.MHD_TUNE_MIDDLE_CHUNK, ch)}
    db = _load()
    if use_cache and key in db:
        best = {(k, int(a)): v for k, av in db[key].items() for a, v in av.items()}
        for (k, a), v in best.items():
            setter[k](a, v)
        return best
    saved = S.get_state_tensor()

    def timed():
        S.set_state_tensor(saved)
        S.step_auto(cfl)
        S.status()
        t = float("inf")
        for _ in range(repeats):
            t0 = time.perf_counter()
            for _ in range(steps):
                S.step_auto(cfl)
            S.status()
            t = min(t, time.perf_counter() - t0)
        return t

    best = {}
    for kind in kinds:
        for axis in ((2,) if kind == "mid" else (1, 2)):
            timings = {}
            for ch in chunk_candidates(S.n[axis]):
                setter[kind](axis, ch)
                timings[ch] = timed()
            best[(kind, axis)] = min(timings, key=timings.get)
            setter[kind](axis, best[(kind, axis)])
    S.set_state_tensor(saved)
    db[key] = {k: {str(a): v for (kk, a), v in best.items() if kk == k} for k in kinds}
    _store(db)
    return best


def tune_batch(B, cfl=0.7, steps=3, grids=(512, 1024, 2048), chunks=(16, 32, 64, 128),
               reverse=(1, 2), pair_chunks=(64, 128, 256), use_cache=True):
    """Choose the persistent grid, the target chunk, whether the reverse-half
    pairs run fused (1) or as two operators (2) and, fused, the target chunk
    of the pairs and whether the middle M_z M_z F_z runs as one launch (1) or
    not (2; FP32 only), for a Batch.  A few steps run first so the device
    clocks have settled; each shape is timed twice and keeps the faster.  A
    box that leaves the physical range takes the cheap skip path of every
    later step, which would favour the shapes timed after it: the saved
    state is then restored and the shape timed again."""
    sig = ",".join(str(n[0]) + "x" + str(n[1]) + "x" + str(n[2]) for n in B.dims)
    key = f"{_device_tag()}:batch:{hash(sig) & 0xffffffff:08x}:{len(B.dims)}:{'f64' if B.prec == mhd.MHD_F64 else 'f32'}"
    db = _load()
    def apply(g, c, r, pc, m):
        for k in (mhd.MHD_BATCH_GRID_X, mhd.MHD_BATCH_GRID_Y, mhd.MHD_BATCH_GRID_Z):
            B.set_launch(k, g)
        B.set_launch(mhd.MHD_BATCH_CHUNK, c)
        B.set_launch(mhd.MHD_BATCH_REVERSE, r)
        B.set_launch(mhd.MHD_BATCH_PAIR_CHUNK, pc)
        B.set_launch(mhd.MHD_BATCH_MIDDLE, m)

    def result(g, c, r, pc, m):
        return {"grid": g, "chunk": c, "reverse": r, "pair_chunk": pc, "middle": B.launch(mhd.MHD_BATCH_MIDDLE)}

    if use_cache and key in db and "middle" in db[key]:
        e = db[key]
        apply(e["grid"], e["chunk"], e["reverse"], e["pair_chunk"], e["middle"])
        return result(e["grid"], e["chunk"], e["reverse"], e["pair_chunk"], e["middle"])
    saved = [B.get_state(i) for i in range(B.nbox)]

    def restore():
        for i, s in enumerate(saved):
            B.set_state(i, s)

    B.run(steps, cfl, graph=True)
    B.status(raise_on_nonphysical=False)
    mids = (1, 2) if B.prec == mhd.MHD_F32 else (2,)
    timings = {}
    for r in reverse:
        for g in grids:
            for c in chunks:
                # the pair chunk and the middle matter only when the pairs run fused
                for pc in (pair_chunks if r == 1 else (pair_chunks[0],)):
                    for m in (mids if r == 1 else (2,)):
                        apply(g, c, r, pc, m)
                        for attempt in range(2):
                            B.run(1, cfl, graph=True)
                            B.status(raise_on_nonphysical=False)
                            best = None
                            for _ in range(2):
                                t0 = time.perf_counter()
                                B.run(steps, cfl, graph=True)
                                _, nonphys = B.status(raise_on_nonphysical=False)
                                t = time.perf_counter() - t0
                                best = t if best is None else min(best, t)
                            if not nonphys.any():
                                break
                            restore()
                        timings[(g, c, r, pc, m)] = best
    # the four fastest shapes again, from the saved state, over more steps
    final = {}
    for cand in sorted(timings, key=timings.get)[:4]:
        apply(*cand)
        restore()
        B.run(1, cfl, graph=True)
        B.status(raise_on_nonphysical=False)
        t0 = time.perf_counter()
        B.run(3 * steps, cfl, graph=True)
        B.status(raise_on_nonphysical=False)
        final[cand] = time.perf_counter() - t0
    g, c, r, pc, m = min(final, key=final.get)
    apply(g, c, r, pc, m)
    restore()
    db[key] = {"grid": g, "chunk": c, "reverse": r, "pair_chunk": pc, "middle": m,
               "timings_ms": {"/".join(map(str, k)): round(v * 1e3 / steps, 3) for k, v in timings.items()}}
    _store(db)
    return result(g, c, r, pc, m)
    saved = [B.get_state(i) for i in range(B.nbox)]
    timings = {}
    for r in reverse:
        for g in grids:
            for c in chunks:
                # the pair chunk matters only when the pairs run fused
                for pc in (pair_chunks if r == 1 else (pair_chunks[0],)):
                    apply(g, c, r, pc)
                    B.run(1, cfl, graph=True)
                    B.status(raise_on_nonphysical=False)
                    t0 = time.perf_counter()
                    B.run(steps, cfl, graph=True)
                    B.status(raise_on_nonphysical=False)
                    timings[(g, c, r, pc)] = time.perf_counter() - t0
    g, c, r, pc = min(timings, key=timings.get)
    apply(g, c, r, pc)
    for i, s in enumerate(saved):
        B.set_state(i, s)
    db[key] = {"grid": g, "chunk": c, "reverse": r, "pair_chunk": pc,
               "timings_ms": {"/".join(map(str, k)): round(v * 1e3 / steps, 3) for k, v in timings.items()}}
    _store(db)
    return {"grid": g, "chunk": c, "reverse": r, "pair_chunk": pc}
