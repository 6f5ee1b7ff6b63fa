"""Summaries of rocprofv3 output for the MHD kernels.

  python -m paper_1004_1680_amd.profile_summary stats  <kernel_stats.csv> <command...>
  python -m paper_1004_1680_amd.profile_summary trace  <kernel_trace.csv> <command...>
  python -m paper_1004_1680_amd.profile_summary traffic <fetch.csv> <write.csv> <ncell> <esize> <command...>

``stats`` prints a per-kernel table (calls, average / min / max duration).
``trace`` does the same from the per-dispatch trace, split by launch grid,
so that the launches of one tuned shape are averaged apart from the
autotuner's trial shapes.
``counters`` turns two ``rocprofv3 --pmc`` runs of SQ counters and a kernel
trace into a per-kernel table for the MFMA kernels: MFMA-busy fraction of
the kernel's SIMD-cycles and LDS bank-conflict cycles per LDS-active cycle.
``traffic`` turns the FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch)
of two ``rocprofv3 --pmc`` runs into HBM bytes per launch, scaled by what
the same counters read for the plain 1 GiB copy that ``bench.py
--calibrate-copy`` runs (a kernel of known traffic), and prints them next to
the algorithmic bytes.  It also prints the hash of the kernel sources the
counters belong to; ``bench.py`` reports the traffic only while the sources
still hash to it.
"""
import collections
import csv
import hashlib
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/sweep_kernels.h", "csrc/mhd_device.h", "csrc/sweep_f32.hip",
                  "csrc/sweep_f64.hip", "csrc/reduce_kernels.hip"]
ALG_WORDS = {"fluid": 13, "mag": 8, "magfluid": 16, "cfl_partial": 8}
COPY_BYTES = 1 << 30


def source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short(name):
    name = name.replace("mhd::", "").replace("void ", "")
    return name.split("(")[0]


def stats(path, command):
    rows = list(csv.DictReader(open(path)))
    out = [f"command: {command}", "",
           "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out)


def trace(path, command):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        key = (short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        d[key].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in d.values())
    out = [f"command: {command}", "",
           "| kernel | grid threads | workgroup | calls | avg us | min us | max us | % time |",
           "|---|---|---|---|---|---|---|---|"]
    for key in sorted(d, key=lambda k: -sum(d[k])):
        v = d[key]
        out.append(f"| {key[0]} | {key[1]} | {key[2]} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | "
                   f"{max(v):.2f} | {100 * sum(v) / total:.2f} |")
    return "\n".join(out)


def per_kernel(path, counter):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            d[r["Kernel_Name"]].append((float(r["Counter_Value"]) * 1024.0, int(r["Grid_Size"])))
    return d


def copy_factor(d):
    """bytes moved / bytes counted for the 1 GiB copies that bench.py
    --calibrate-copy makes after all other work: the last three copy
    dispatches of the run (the median of them)"""
    vals = [v for k, lst in d.items() if "copyBuffer" in k for v, g in lst]
    last = sorted(vals[-3:])
    ref = last[len(last) // 2] if last else None
    return COPY_BYTES / ref if ref else None


def traffic(fetch_csv, write_csv, ncell, esize, command):
    F = per_kernel(fetch_csv, "FETCH_SIZE")
    W = per_kernel(write_csv, "WRITE_SIZE")
    ff, fw = copy_factor(F), copy_factor(W)
    out = [f"command: {command}", f"kernel source hash: {source_hash()}",
           f"copy calibration: reads x{ff:.3f}, writes x{fw:.3f} "
           f"(1 GiB copy: counters / known bytes)", "",
           "| kernel | read MiB/launch | write MiB/launch | algorithmic MiB | traffic / algorithmic |",
           "|---|---|---|---|---|"]
    for k in sorted(F):
        if "mhd::" not in k:
            continue
        s = short(k)
        kind = ("magfluid" if "magfluid" in s else "fluid" if "fluid" in s else "mag" if "mag" in s
                else "cfl_partial" if "cfl_partial" in s else None)
        if kind is None:
            continue
        rd = sum(v for v, g in F[k]) / len(F[k]) * ff
        wr = sum(v for v, g in W[k]) / len(W[k]) * fw if W.get(k) else 0.0
        alg = ALG_WORDS[kind] * esize * ncell
        out.append(f"| {s} | {rd / 2**20:.1f} | {wr / 2**20:.1f} | {alg / 2**20:.1f} | "
                   f"{(rd + wr) / alg:.3f} |")
        out.append(f"traffic_bytes[{s}] = {int(rd + wr)}")
        # per launch grid (a march kernel's traffic depends on its chunk length)
        for grid in sorted({g for v, g in F[k]}):
            r_g = [v for v, g in F[k] if g == grid]
            w_g = [v for v, g in W.get(k, []) if g == grid]
            tot = sum(r_g) / len(r_g) * ff + (sum(w_g) / len(w_g) * fw if w_g else 0.0)
            out.append(f"traffic_bytes[{s} @ {grid}] = {int(tot)}")
    return "\n".join(out)


SIMDS, CLOCK_HZ = 1024, 2.4e9     # MI355X: 256 CUs x 4 SIMDs


def counters(pmc1_csv, pmc2_csv, stats_csv, command):
    vals = collections.defaultdict(lambda: collections.defaultdict(list))
    for path in (pmc1_csv, pmc2_csv):
        with open(path) as f:
            for r in csv.DictReader(f):
                vals[short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = {}
    with open(stats_csv) as f:
        for r in csv.DictReader(f):
            dur[short(r["Name"])] = float(r["AverageNs"]) * 1e-9
    out = [f"command: {command}", "",
           "| kernel | MFMA busy / SIMD-cycles | LDS bank-conflict / LDS-active cycles | VALU insts / wave | LDS insts / wave |",
           "|---|---|---|---|---|"]
    for k in sorted(vals):
        v = {c: sum(x) / len(x) for c, x in vals[k].items()}
        if not v.get("SQ_VALU_MFMA_BUSY_CYCLES") or k not in dur:
            continue
        busy = v["SQ_VALU_MFMA_BUSY_CYCLES"] / (dur[k] * CLOCK_HZ * SIMDS)
        conf = v.get("SQ_LDS_BANK_CONFLICT", 0.0) / max(v.get("SQ_LDS_IDX_ACTIVE", 0.0), 1.0)
        waves = max(v.get("SQ_WAVES", 1.0), 1.0)
        out.append(f"| {k} | {busy:.3f} | {conf:.3f} | {v.get('SQ_INSTS_VALU', 0.0) / waves:.0f} | "
                   f"{v.get('SQ_INSTS_LDS', 0.0) / waves:.0f} |")
    return "\n".join(out)


def read_traffic(path):
    """{kernel: bytes per launch} (also {"kernel @ grid threads": bytes} per
    launch shape) from a traffic summary, or {} if the kernel sources have
    changed since it was written"""
    if not os.path.exists(path):
        return {}
    txt = open(path).read()
    want = f"kernel source hash: {source_hash()}"
    if want not in txt:
        return {}
    out = {}
    for line in txt.splitlines():
        if line.startswith("traffic_bytes["):
            k = line[len("traffic_bytes["):line.index("]")]
            out[k] = int(line.split("=")[1])
    return out


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "stats":
        print(stats(sys.argv[2], " ".join(sys.argv[3:])))
    elif mode == "trace":
        print(trace(sys.argv[2], " ".join(sys.argv[3:])))
    elif mode == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5]),
                      " ".join(sys.argv[6:])))
    elif mode == "counters":
        print(counters(sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:])))
    elif mode == "hash":
        print(source_hash())
