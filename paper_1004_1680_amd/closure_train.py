"""Training data, training and evaluation of the learned coarse closure.

Every numerical step runs in the library's kernels through the C ABI: the
fine and coarse solvers (mhd_step, mhd_cfl_dt), the restriction operator
(mhd_restrict), and the closure's MFMA forward/backward and Adam
(mhd_closure_*).  PyTorch holds device tensors and forms the per-pair
target difference and the normalisation statistics of the training set.

Data (one pair per coarse step of a fine trajectory):
  u_c      = R u_f(t)                  restriction by r of the fine state
  u_plain  = plain coarse step of u_c  (dt_c from the coarse CFL condition)
  target   = R u_f(t + 2 dt_c) - u_plain, the fine run stepped to exactly
             t + 2 dt_c (last fine step shortened)
The closure learns u_plain -> target; its learned coarse step is
u_plain + correction, with the plain step kept when the corrected state is
not physical.

Evaluation: from a held-out initial state, the learned coarse solver, the
plain coarse solver and plain solvers at 2x and 4x the coarse resolution run
to the same final time; each is restricted to the coarse grid and compared
with the restricted fine solution (relative L1 averaged over the 8 fields),
together with its wall time.
"""
import json
import time

import numpy as np

from . import inputs as I
from . import mhd

FAMILIES = {1: [0], 2: [1, 2, 3], 3: [4], 4: [5, 6, 7]}


def l1_rel(a, b):
    """mean over the 8 fields of mean|a - b| / mean|b| (a zero reference
    field uses the scale of its family)"""
    errs = []
    for idx in FAMILIES.values():
        fam = float(np.mean(np.abs(b[idx])))
        for f in idx:
            den = float(np.mean(np.abs(b[f])))
            if den == 0.0:
                den = fam if fam > 0 else 1.0
            errs.append(float(np.mean(np.abs(a[f] - b[f]))) / den)
    return float(np.mean(errs))


def _sync(torch):
    torch.cuda.synchronize()


def advance_to(S, t_end, cfl=0.7, t0=0.0, log=None, every=200):
    """host-dt steps of S from time t0 to exactly t_end; returns steps"""
    t, k = t0, 0
    while t < t_end * (1.0 - 1e-12):
        dt = min(S.cfl_dt(cfl), 0.5 * (t_end - t))
        S.step(dt)
        t += 2.0 * dt
        k += 1
        if log and k % every == 0:
            log(f"[closure] {S.n[0]}^3 run: step {k}, t = {t:.4f} of {t_end:.4f}")
    return k


class PairSet:
    """Training pairs of one coarse grid, kept as (u_c, u_ref, dt, c): the
    restricted fine state at t, the restricted fine state at t + 2 dt and
    the coarse step's dt and relaxation speed (half the memory of storing
    the plain step as well).  pair(i) runs the plain coarse step (library
    step on the device) and returns (u_plain, target = u_ref - u_plain,
    residual kernel)."""

    def __init__(self, cl, nc, stream):
        self.cl = cl
        self.C = mhd.Solver((nc,) * 3, prec="f32", stream=stream)
        self.items = []
        self.seeds = []          # trajectories that gave at least one pair

    def add(self, u_c, u_ref, dt, c):
        self.items.append((u_c, u_ref, dt, c))

    def pair(self, i):
        u_c, u_ref, dt, c = self.items[i]
        self.C.set_state_tensor(u_c)
        self.C.set_relaxation_speed(c)
        self.C.step(dt)
        u_plain = self.C.get_state_tensor()
        return u_plain, self.cl.residual(u_ref, u_plain)

    def __len__(self):
        return len(self.items)

    def __getitem__(self, i):
        if isinstance(i, slice):
            return [self.pair(j) for j in range(*i.indices(len(self)))]
        return self.pair(i)

    def __iter__(self):
        for i in range(len(self)):
            yield self.pair(i)

    def extend(self, other):
        self.items.extend(other.items)
        self.seeds.extend(other.seeds)


def generate_pairs(cl, nf, r, seeds, steps_per_traj, stream, cfl=0.7, log=print, rollout=False, deadline=None):
    """training pairs from fine trajectories of the Orszag-Tang family (one
    per seed), as a PairSet; cl: the Closure of the coarse grid, whose
    residual kernel forms the targets.  Within a trajectory the restricted
    state that ends one pair starts the next and is stored once.

    deadline: a time.perf_counter() value after which no further pair is
    generated (the pairs so far are returned).

    rollout: also pairs whose input is the state of a plain coarse run
    started from the restricted initial state and stepped with the same
    coarse time steps (and relaxation speeds), paired with the same
    restricted fine state: the coarse states a rollout actually visits,
    whose correction includes pulling the accumulated error back toward the
    fine solution."""
    nc = nf // r
    F = mhd.Solver((nf,) * 3, prec="f32", stream=stream)
    C = mhd.Solver((nc,) * 3, prec="f32", stream=stream)
    Rr = mhd.Solver((nc,) * 3, prec="f32", stream=stream) if rollout else None
    pairs = PairSet(cl, nc, stream)
    for sd in seeds:
        if deadline is not None and time.perf_counter() > deadline:
            log(f"[closure] time budget reached before seed {sd}: {len(pairs)} pairs")
            break
        F.set_state_tensor(I.orszag_tang_torch((nf,) * 3, seed=sd))
        t = 0.0
        roll_alive = rollout
        u_ref = None
        for k in range(steps_per_traj):
            if deadline is not None and time.perf_counter() > deadline:
                log(f"[closure] time budget reached at seed {sd}, coarse step {k}: {len(pairs)} pairs")
                break
            try:
                F.restrict_to(C)
                u_c = C.get_state_tensor().clone() if u_ref is None else u_ref
                dtc = C.cfl_dt(cfl)
                c = C.relaxation_speed()
                nfine = advance_to(F, t + 2.0 * dtc, cfl, t0=t)
            except mhd.NonPhysicalState as e:
                # the plain scheme does not guarantee positivity: the
                # trajectory ends here, its earlier pairs are kept
                log(f"[closure] seed {sd} ends at coarse step {k} (t = {t:.4f}): {e}")
                break
            t += 2.0 * dtc
            F.restrict_to(C)
            u_ref = C.get_state_tensor().clone()
            pairs.add(u_c, u_ref, dtc, c)
            if not pairs.seeds or pairs.seeds[-1] != sd:
                pairs.seeds.append(sd)
            if roll_alive:
                if k == 0:
                    Rr.set_state_tensor(u_c)
                else:
                    try:
                        Rr.cfl_dt(cfl)             # raises once the plain run is non-physical
                        pairs.add(Rr.get_state_tensor().clone(), u_ref, dtc, c)
                    except mhd.NonPhysicalState:
                        log(f"[closure] seed {sd}: plain coarse rollout non-physical at step {k}")
                        roll_alive = False
                if roll_alive:
                    Rr.set_relaxation_speed(c)
                    Rr.step(dtc)
            if k % 8 == 0:
                log(f"[closure] seed {sd} coarse step {k}: dt_c {dtc:.3e}, {nfine} fine steps")
    F.close()
    C.close()
    if Rr is not None:
        Rr.close()
    return pairs


def fit_scales(cl, pairs, mode="family"):
    """Normalisation of the closure from the training set (FP64 per-field
    sums from the library's statistics kernel).

    in_mean, in_std: per-channel mean and standard deviation of the inputs.
    out_scale: mean |target| pooled over each field family (density,
      momentum, energy, magnetic field), so the network output is O(1) and
      the three axes are treated alike.
    target_scale (the loss weight 1 / s^2 of each field):
      "family": the same pooled mean |target|;
      "state":  mean |u| pooled over the family, i.e. the loss measures the
                error relative to the size of the field, as the relative L1
                error of the evaluation does."""
    tot = np.zeros((5, 8))
    n = 0
    for u, t in pairs:
        tot += cl.stats(u, t)
        n += u[0].numel()
    mean = tot[0] / n
    var = np.maximum(tot[1] / n - mean * mean, 0.0)
    in_std = np.sqrt(var) + 1e-6 * (np.abs(mean) + 1e-6)
    uabs = tot[2] / n
    tabs = tot[3] / n
    out_scale = np.empty(8)
    state_scale = np.empty(8)
    for idx in FAMILIES.values():
        out_scale[idx] = max(float(np.mean(tabs[idx])), 1e-12)
        state_scale[idx] = max(float(np.mean(uabs[idx])), 1e-12)
    if mode == "family":
        target_scale = out_scale.copy()
    elif mode == "state":
        target_scale = state_scale
    else:
        raise ValueError(f"unknown scale mode {mode!r}")
    return mean, in_std, out_scale, target_scale


def fit_gate(cl, pairs):
    """training-set mean roughness per field (floored at 1e-6 of the
    largest, so a field that stays flat does not dominate the gate)"""
    tot = np.zeros(8)
    n = 0
    for u, t in pairs:
        tot += cl.stats(u, t)[4]
        n += u[0].numel()
    R = tot / n
    return np.maximum(R, 1e-6 * max(R.max(), 1e-30))


def init_params(seed=0):
    """He-normal weights, zero biases; the last layer starts small so the
    untrained closure is close to the plain step"""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in ((8, 32), (32, 32), (32, 8)):
        w = rng.normal(0.0, np.sqrt(2.0 / (27 * cin)), size=(27, cin, cout))
        if cout == 8:
            w *= 0.01
        out += [w.ravel(), np.zeros(cout)]
    return np.concatenate(out).astype(np.float32)


def pair_scales(cl, pairs):
    """per pair, mean |target| pooled over each field family (8-vector)"""
    out = []
    for u, t in pairs:
        tabs = cl.stats(u, t)[3] / u[0].numel()
        s = np.empty(8)
        for idx in FAMILIES.values():
            s[idx] = max(float(np.mean(tabs[idx])), 1e-30)
        out.append(s)
    return out


def train(cl, pairs, val, epochs, lr, log=print, seed=0, lr_min_frac=0.05, scales=None, weighting="global"):
    """Adam over shuffled pairs, cosine learning-rate decay from lr to
    lr * lr_min_frac over all steps; returns (mean train loss, validation
    loss) per epoch.

    weighting: the loss scale of each pair (the target_scale of the closure
      during its step):
      "global": the training-set scales (set on the closure beforehand);
      "pair":   the pair's own mean |target| per family, so that a smooth
                early state with a small correction weighs as much as a
                state with shocks;
      "sqrt":   the geometric mean of the two."""
    rng = np.random.default_rng(seed)
    hist = []
    total = max(1, epochs * len(pairs))
    step = 0
    t_start = time.perf_counter()
    if weighting != "global":
        if scales is None:
            raise ValueError("per-pair weighting needs the training-set scales")
        ps = pair_scales(cl, pairs)
        vs = pair_scales(cl, val) if val else []
        g = np.asarray(scales[3], dtype=np.float64)
        if weighting == "sqrt":
            ps = [np.sqrt(p * g) for p in ps]
            vs = [np.sqrt(p * g) for p in vs]
        elif weighting != "pair":
            raise ValueError(f"unknown weighting {weighting!r}")

    def set_ts(ts):
        cl.set_scales(scales[0], scales[1], scales[2], ts)

    for ep in range(epochs):
        order = rng.permutation(len(pairs))
        tr = []
        for i in order:
            if weighting != "global":
                set_ts(ps[i])
            f = 0.5 * (1.0 + np.cos(np.pi * step / total))
            u, t = pairs[i]
            tr.append(cl.train_step(u, t, lr * (lr_min_frac + (1 - lr_min_frac) * f)))
            step += 1
        vl = []
        for j, (u, t) in enumerate(val or []):
            if weighting != "global":
                set_ts(vs[j])
            vl.append(cl.grad(u, t)[0])
        hist.append((float(np.mean(tr)), float(np.mean(vl)) if vl else None))
        log(f"[closure] epoch {ep}: train loss {hist[-1][0]:.4f}"
            + (f", validation loss {hist[-1][1]:.4f}" if vl else "")
            + f" ({time.perf_counter() - t_start:.1f} s)")
    if weighting != "global":
        set_ts(scales[3])
    return hist


def field_errors(cl, pairs):
    """per-field one-step residual ratio sum|target - delta| / sum|target|
    over pairs (below 1: the correction moves the plain step toward the
    restricted fine solution)"""
    num = np.zeros(8)
    den = np.zeros(8)
    for u, t in pairs:
        d = cl.forward(u)
        num += cl.stats(u, cl.residual(t, d))[3]
        den += cl.stats(u, t)[3]
    return num / np.maximum(den, 1e-300)


def _timed_auto(S, u0, k, cfl, torch):
    """wall time of k device-dt steps of S from state u0 (one sync at the end)"""
    S.set_state_tensor(u0)
    _sync(torch)
    t0 = time.perf_counter()
    for _ in range(k):
        S.step_auto(cfl)
    S.status()
    _sync(torch)
    return time.perf_counter() - t0


def _equal_l1_wall(plains, L):
    """plain wall time at L1 = L, log-log interpolated between the two plain
    resolutions whose L1 brackets L (None outside their range)"""
    for (l0, w0), (l1, w1) in zip(plains, plains[1:]):
        if l1 <= L <= l0 and l0 > l1:
            a = (np.log(l0) - np.log(L)) / (np.log(l0) - np.log(l1))
            return float(np.exp((1 - a) * np.log(w0) + a * np.log(w1)))
    return None


def evaluate(cl, nf, r, seed, nsteps, torch, stream, cfl=0.7, log=print, checkpoints=None):
    """learned vs plain coarse solvers against the restricted fine truth.

    The learned solver takes nsteps closure steps (device dt); the times it
    reaches after the checkpoint step counts (default: nsteps only) are the
    comparison times.  The fine solver and the plain solvers at nc, 2nc, 4nc
    (below the fine size) advance through those times exactly (host dt, the
    step before each time shortened); each solution is restricted to nc and
    compared with the restricted fine solution (relative L1 over the 8
    fields).  Should the fine run leave the physical range, the comparison
    ends at the last time it reached.  Wall times are those of device-dt
    steps with one synchronisation at the end: the learned run as timed
    between checkpoints, a plain run as the same number of plain steps it
    needed to reach the last compared time.  Returns a dict with one entry
    per checkpoint and the summary of the last one at top level."""
    nc = nf // r
    checkpoints = sorted(set(checkpoints or [nsteps]) | {nsteps})
    levels = []
    m = 1
    while nc * m < nf and m <= 4:
        levels.append(nc * m)
        m *= 2
    F = mhd.Solver((nf,) * 3, prec="f32", stream=stream)
    F.set_state_tensor(I.orszag_tang_torch((nf,) * 3, seed=seed))
    ics = {}
    for n in levels:
        P = mhd.Solver((n,) * 3, prec="f32", stream=stream)
        F.restrict_to(P)
        ics[n] = P.get_state_tensor().clone()
        P.close()

    # learned rollout, states kept at the checkpoints
    C = mhd.Solver((nc,) * 3, prec="f32", stream=stream)
    C.set_state_tensor(ics[nc])
    learned, times, walls = [], [], []
    done, wall = 0, 0.0
    for ck in checkpoints:
        _sync(torch)
        t0 = time.perf_counter()
        try:
            for _ in range(ck - done):
                cl.step(C, cfl)
            C.status()
        except mhd.NonPhysicalState as e:
            log(f"[closure] learned run left the physical range before step {ck}: {e}")
            break
        _sync(torch)
        wall += time.perf_counter() - t0
        done = ck
        learned.append(C.get_state())
        times.append(C.time())
        walls.append(wall)
    if not times:
        C.close()
        F.close()
        raise mhd.MHDError(mhd.MHD_ENONPHYS, "learned run failed before the first comparison time")
    checkpoints = checkpoints[:len(times)]
    fallbacks, reduced = cl.fallbacks(), cl.reduced()
    log(f"[closure] learned {nc}^3: {done} steps to t = {times[-1]:.4f} in {wall:.4f} s "
        f"({reduced} reduced, {fallbacks} dropped corrections)")

    # fine truth through the checkpoint times
    truth, nfine, t = [], 0, 0.0
    try:
        for T in times:
            nfine += advance_to(F, T, cfl, t0=t, log=log)
            t = T
            F.restrict_to(C)
            truth.append(C.get_state())
    except mhd.NonPhysicalState as e:
        log(f"[closure] fine run left the physical range after t = {t:.4f}: {e}")
    F.close()
    ncmp = len(truth)
    if ncmp == 0:
        C.close()
        raise mhd.MHDError(mhd.MHD_ENONPHYS, "fine run failed before the first comparison time")

    per = [{"steps": checkpoints[i], "t": times[i], "learned_L1": l1_rel(learned[i], truth[i]),
            "learned_wall_s": walls[i]} for i in range(ncmp)]
    plain_summary = {}
    for n in levels:
        P = mhd.Solver((n,) * 3, prec="f32", stream=stream)
        P.set_state_tensor(ics[n])
        k, t = 0, 0.0
        try:
            for i in range(ncmp):
                k += advance_to(P, times[i], cfl, t0=t, log=log)
                t = times[i]
                if n != nc:
                    P.restrict_to(C)
                    st = C.get_state()
                else:
                    st = P.get_state()
                per[i][f"plain_{n}_L1"] = l1_rel(st, truth[i])
                per[i][f"plain_{n}_steps"] = k
        except mhd.NonPhysicalState as e:
            log(f"[closure] plain {n}^3 left the physical range after t = {t:.4f}: {e}")
        wall_n = _timed_auto(P, ics[n], k, cfl, torch) if k else None
        P.close()
        plain_summary[n] = (k, wall_n)
        last = per[ncmp - 1].get(f"plain_{n}_L1")
        log(f"[closure] plain {n}^3: L1 {last if last is None else f'{last:.4e}'}, {k} steps in "
            f"{wall_n if wall_n is None else f'{wall_n:.4f}'} s")
    C.close()
    for i in range(ncmp):
        log(f"[closure] t = {per[i]['t']:.4f} ({per[i]['steps']} steps): learned L1 {per[i]['learned_L1']:.4e}, "
            + ", ".join(f"plain {n}^3 {per[i][f'plain_{n}_L1']:.4e}" for n in levels
                        if f"plain_{n}_L1" in per[i]))

    fin = per[ncmp - 1]
    res = {"T": fin["t"], "compared_steps": fin["steps"], "checkpoints": per,
           "fine": {"n": nf, "steps": nfine},
           "learned": {"n": nc, "L1": fin["learned_L1"], "wall_s": fin["learned_wall_s"], "steps": fin["steps"],
                       "fallbacks": fallbacks, "reduced": reduced}}
    for n in levels:
        k, w = plain_summary[n]
        if f"plain_{n}_L1" in fin:
            res[f"plain_{n}"] = {"n": n, "L1": fin[f"plain_{n}_L1"], "wall_s": w, "steps": k}
    plains = [(res[f"plain_{n}"]["L1"], res[f"plain_{n}"]["wall_s"]) for n in levels if f"plain_{n}" in res]
    eq = _equal_l1_wall(plains, res["learned"]["L1"])
    res["plain_wall_at_equal_L1_s"] = eq
    res["speedup_at_equal_L1"] = (eq / res["learned"]["wall_s"]) if eq else None
    return res


def save(path, cl, scales, meta=None, gate=None):
    """trained closure -> .npz (parameters, the four scale vectors, the mean
    roughness of the gate (empty: no gate), metadata as a JSON string)"""
    np.savez(path, params=cl.params(), in_mean=np.asarray(scales[0]), in_std=np.asarray(scales[1]),
             out_scale=np.asarray(scales[2]), target_scale=np.asarray(scales[3]),
             gate=np.asarray(gate if gate is not None else [], dtype=np.float64),
             meta=np.array(json.dumps(meta or {})))


def load(path, n, stream=None):
    """Closure of grid n with the parameters and scales stored by save()"""
    z = np.load(path, allow_pickle=False)
    cl = mhd.Closure(n, stream=stream)
    cl.set_params(z["params"])
    scales = (z["in_mean"], z["in_std"], z["out_scale"], z["target_scale"])
    cl.set_scales(*scales)
    if "gate" in z.files and z["gate"].size == 8:
        cl.set_gate(z["gate"])
    return cl, scales, json.loads(str(z["meta"]))


def train_closure(nf=256, r=8, train_seeds=tuple(range(1, 13)), val_seed=100, steps_per_traj=24,
                  val_steps=None, epochs=10, lr=1e-3, cfl=0.7, scale_mode="family", log=print,
                  weighting="global", gate=False, short_seeds=(), short_steps=0, rollout=False,
                  init=None, budget_s=None):
    """data generation and training; returns (closure, scales, info).
    short_seeds / short_steps: further trajectories of short_steps pairs
    each, which weight the early, smooth part of the flow more.

    init: a closure saved by save() to continue from: its parameters,
      scales and gate are kept (not fitted again; scale_mode and gate are
      then those it was saved with) and training goes on over the new pairs
      (Adam's moments start from zero); its metadata's pair count is carried
      into pairs_total, so a training set larger than one run can generate
      is covered in several runs over disjoint seeds.  val_loss_untrained
      is then the validation loss of the loaded parameters.
    budget_s: seconds from the start after which no further training pair
      is generated (the validation pairs come first)."""
    import torch
    stream = torch.cuda.current_stream()
    nc = nf // r
    cl = mhd.Closure((nc,) * 3, stream=stream)
    t0 = time.perf_counter()
    deadline = None if budget_s is None else t0 + budget_s
    val = generate_pairs(cl, nf, r, (val_seed,), val_steps or steps_per_traj, stream, cfl, log)
    pairs = generate_pairs(cl, nf, r, train_seeds, steps_per_traj, stream, cfl, log, rollout, deadline)
    if short_seeds and short_steps:
        pairs.extend(generate_pairs(cl, nf, r, short_seeds, short_steps, stream, cfl, log, deadline=deadline))
    _sync(torch)
    t_data = time.perf_counter() - t0
    log(f"[closure] {len(pairs)} training and {len(val)} validation pairs in {t_data:.1f} s")
    if len(pairs) == 0:
        raise ValueError("no training pairs were generated (time budget or trajectories too short)")
    before = {}
    if init is not None:
        z = np.load(init, allow_pickle=False)
        before = json.loads(str(z["meta"]))
        if (before.get("nf"), before.get("ratio")) != (nf, r):
            raise ValueError(f"{init} was trained for nf={before.get('nf')}, ratio={before.get('ratio')}")
        scales = (z["in_mean"], z["in_std"], z["out_scale"], z["target_scale"])
        R = z["gate"] if z["gate"].size == 8 else None
        scale_mode = before.get("scale_mode", scale_mode)
        cl.set_params(z["params"])
    else:
        scales = fit_scales(cl, pairs, scale_mode)
        R = fit_gate(cl, pairs) if gate else None
        cl.set_params(init_params(0))
    cl.set_scales(*scales)
    cl.set_gate(R)
    val_loss0 = float(np.mean([cl.grad(u, t)[0] for u, t in val]))
    t0 = time.perf_counter()
    hist = train(cl, pairs, val, epochs, lr, log, scales=scales, weighting=weighting)
    _sync(torch)
    t_train = time.perf_counter() - t0
    fe = field_errors(cl, val)
    log("[closure] validation one-step residual ratio per field: " + " ".join(f"{v:.3f}" for v in fe))
    # the same on up to 32 training pairs spread over the set (below 1 there
    # but not on the validation pairs: the fit does not carry over)
    idx = np.unique(np.linspace(0, len(pairs) - 1, min(32, len(pairs))).astype(int))
    fe_tr = field_errors(cl, (pairs[int(i)] for i in idx))
    log("[closure] training-pair one-step residual ratio per field: " + " ".join(f"{v:.3f}" for v in fe_tr))
    info = {"nf": nf, "ratio": r, "train_seeds": list(train_seeds), "steps_per_traj": steps_per_traj,
            "short_seeds": list(short_seeds), "short_steps": short_steps,
            "pairs": len(pairs), "data_s": t_data, "train_s": t_train, "epochs": epochs, "lr": lr,
            "train_steps": epochs * len(pairs), "val_loss_untrained": val_loss0, "history": hist,
            "val_field_residual": fe.tolist(), "train_field_residual": fe_tr.tolist(), "scale_mode": scale_mode, "weighting": weighting,
            "gate": None if R is None else np.asarray(R).tolist(), "rollout": rollout,
            "pairs_total": before.get("pairs_total", before.get("pairs", 0)) + len(pairs),
            "runs": before.get("runs", []) + [{"seeds": list(pairs.seeds), "pairs": len(pairs),
                                               "epochs": epochs, "lr": lr}]}
    del pairs, val
    return cl, scales, info


def run(nf=256, r=8, train_seeds=tuple(range(1, 13)), val_seed=100, test_seed=200, steps_per_traj=24,
        epochs=10, lr=1e-3, eval_steps=24, cfl=0.7, scale_mode="family", log=print, weighting="global",
        gate=False):
    """train then evaluate; returns (result dict, closure)"""
    import torch
    stream = torch.cuda.current_stream()
    cl, scales, info = train_closure(nf, r, train_seeds, val_seed, steps_per_traj, None, epochs, lr, cfl,
                                     scale_mode, log, weighting, gate)
    res = evaluate(cl, nf, r, test_seed, eval_steps, torch, stream, cfl, log)
    res.update(info)
    res["scales"] = [np.asarray(v).tolist() for v in scales]
    return res, cl


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="train / evaluate the learned coarse closure")
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--nf", type=int, default=256)
    t.add_argument("--ratio", type=int, default=8)
    t.add_argument("--seeds", type=int, default=12, help="training trajectories (seeds 1..N)")
    t.add_argument("--steps", type=int, default=24, help="coarse steps (pairs) per trajectory")
    t.add_argument("--val-steps", type=int, default=None)
    t.add_argument("--epochs", type=int, default=10)
    t.add_argument("--lr", type=float, default=1e-3)
    t.add_argument("--weighting", default="global", choices=("global", "pair", "sqrt"))
    t.add_argument("--gate", action="store_true", help="roughness gate on the correction")
    t.add_argument("--short-seeds", type=int, default=0, help="extra short trajectories")
    t.add_argument("--short-steps", type=int, default=0)
    t.add_argument("--rollout", action="store_true",
                   help="also pairs from plain coarse rollouts (the states a rollout visits)")
    t.add_argument("--seed-start", type=int, default=1, help="first training seed")
    t.add_argument("--init", default=None, help="continue from this saved closure (its scales and gate kept)")
    t.add_argument("--budget-s", type=float, default=None, help="stop generating training pairs after this")
    t.add_argument("--out", required=True, help=".npz file for the trained closure")
    e = sub.add_parser("eval")
    e.add_argument("--weights", required=True)
    e.add_argument("--steps", type=int, default=200, help="learned coarse steps of the rollout")
    e.add_argument("--seed", type=int, default=200, help="held-out initial state")
    e.add_argument("--checkpoints", type=str, default="", help="comma-separated step counts")
    args = ap.parse_args()
    say = lambda m: print(m, flush=True)
    import torch
    stream = torch.cuda.current_stream()
    if args.cmd == "train":
        s0 = args.seed_start
        cl, scales, info = train_closure(args.nf, args.ratio, tuple(range(s0, s0 + args.seeds)),
                                         steps_per_traj=args.steps, val_steps=args.val_steps,
                                         epochs=args.epochs, lr=args.lr, log=say,
                                         weighting=args.weighting, gate=args.gate,
                                         short_seeds=tuple(range(s0 + args.seeds, s0 + args.seeds + args.short_seeds)),
                                         short_steps=args.short_steps, rollout=args.rollout,
                                         init=args.init, budget_s=args.budget_s)
        save(args.out, cl, scales, info, info["gate"])
        print(json.dumps(info))
    else:
        z = np.load(args.weights, allow_pickle=False)
        meta = json.loads(str(z["meta"]))
        nf, r = meta["nf"], meta["ratio"]
        cl, scales, meta = load(args.weights, (nf // r,) * 3, stream)
        cks = [int(v) for v in args.checkpoints.split(",") if v] or None
        res = evaluate(cl, nf, r, args.seed, args.steps, torch, stream, log=say, checkpoints=cks)
        res["training"] = {k: meta[k] for k in ("pairs", "pairs_total", "runs", "epochs", "train_steps",
                                                "data_s", "train_s") if k in meta}
        print(json.dumps(res))
