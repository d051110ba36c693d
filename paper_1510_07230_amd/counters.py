"""Summarise rocprofv3 counter runs of bench.py.

Usage:
  python -m paper_1510_07230_amd.counters FETCH_CSV WRITE_CSV BLOCK_BYTES \\
      [--json OUT.json] [--md OUT.md] [--norb N --n n]
  python -m paper_1510_07230_amd.counters --mfma COUNTER_CSV TRACE_CSV \\
      [--md OUT.md] [--norb N --n n] [--cmd "..."]

The --mfma form reads a run with SQ_INSTS_VALU_MFMA_MOPS_{BF16,F32,F64},
SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE and the kernel trace of the same
run, and reports per kernel the matrix-core FLOPs per dispatch (MOPS counters
count units of 512 FLOPs), the achieved FLOP rate over the traced duration
and its fraction of the dense MFMA peak of the dominant type, and the raw
ratio of SQ_VALU_MFMA_BUSY_CYCLES to GRBM_GUI_ACTIVE (the aggregation of the
busy counter over CUs and SIMDs is not documented here, so the FLOP-based
fraction is the utilisation figure).

  python -m paper_1510_07230_amd.counters --stats KERNEL_STATS_CSV --md OUT.md \\
      [--title T] [--cmd "..."] [--sources]

The --stats form turns a rocprofv3 --stats kernel table into a Markdown
summary (top kernels by total time) with the hashes of the HIP sources.

BLOCK_BYTES is the size of the plain copy (k_convert<float,float>) that the
--calibrate-copy run of bench.py performs: it reads and writes BLOCK_BYTES
once, which scales the counters (KiB per dispatch) to bytes.  The JSON holds,
per kernel group of the mixed-precision step, the scaled HBM bytes of one
launch, the algorithmic bytes and a hash of the kernel's source file, so a
reader can tell whether the figures still describe the current kernel.
"""
import argparse
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel group -> (kernel-name fragment of the mixed step, source file)
GROUP_KERNELS = {
    "trial": ("k_gram_small_bf16<8, 32, true>", "dense_kernels.hip"),
    "apply_gram": ("k_apply_gram8<8>", "dense_kernels.hip"),
    "apply": ("k_apply_s3<8>", "dense_kernels.hip"),
    "hamiltonian": ("k_hamiltonian<float>", "grid_kernels.hip"),
    "commit": ("k_commit<float>", "grid_kernels.hip"),
}


def algorithmic_bytes(group, N, ng, es=4):
    """Bytes a launch moves when each operand is read or written once (the
    accept kernel: the four blocks of the Barzilai-Borwein traces plus the
    write of the new iterate into the caller's block)."""
    B = N * ng * es
    return {"trial": 3 * B, "apply_gram": B, "apply": 2 * B + 8 * ng,
            "hamiltonian": 2 * B + es * ng, "commit": 5 * B}[group]


PEAK_TFLOPS = {"BF16": 2500.0, "F32": 157.3, "F64": 78.6}
MFMA_COUNTERS = ("SQ_INSTS_VALU_MFMA_MOPS_BF16", "SQ_INSTS_VALU_MFMA_MOPS_F32",
                 "SQ_INSTS_VALU_MFMA_MOPS_F64", "SQ_VALU_MFMA_BUSY_CYCLES", "GRBM_GUI_ACTIVE")


def mfma_summary(counter_csv, trace_csv, min_flops=1e9):
    """Per kernel: mean counters per dispatch, traced mean duration, MFMA FLOPs,
    achieved TFLOP/s and fraction of the peak of the type with most FLOPs."""
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(counter_csv)):
        vals[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    dur = defaultdict(list)
    for r in csv.DictReader(open(trace_csv)):
        dur[r["Kernel_Name"]].append((float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) * 1e-9)
    out = {}
    for k, cs in vals.items():
        mean = {c: sum(v) / len(v) for c, v in cs.items()}
        flops = {t: 512.0 * mean.get("SQ_INSTS_VALU_MFMA_MOPS_" + t, 0.0) for t in PEAK_TFLOPS}
        total = sum(flops.values())
        if total < min_flops or not dur.get(k):
            continue
        d = sorted(dur[k])[len(dur[k]) // 2]  # median traced duration
        top = max(flops, key=flops.get)
        busy = mean.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0)
        gui = mean.get("GRBM_GUI_ACTIVE", 0.0)
        out[k] = {"dispatches": len(next(iter(cs.values()))), "median_us": d * 1e6,
                  "mfma_flops": flops, "type": top,
                  "tflops": total / d / 1e12,
                  "frac_of_peak": flops[top] / d / 1e12 / PEAK_TFLOPS[top],
                  "busy_per_gui": busy / gui if gui > 0 else None}
    return out


def mfma_markdown(res, title, cmds):
    out = [f"# MFMA use per kernel from rocprofv3 counters ({title})", "",
           "Counter run (the program directly after `--`; $REPO: the repository root, "
           "$OUT: an output directory):", ""]
    out += ["    " + x for x in cmds]
    out += ["", "MOPS counters count units of 512 FLOPs (checked: the FP64 Gram of 128 "
                "orbitals over 96^3 points reports 36 tiles x 256 x 2 x 884,736 FLOPs).  Rate = "
                "FLOPs per dispatch / median traced duration of the same run (counter "
                "collection can lengthen a kernel, so the rate is a lower bound); peak = dense "
                "MFMA peak of the dominant type (BF16 2.5 PFLOP/s, FP32 157.3, FP64 78.6 "
                "TFLOP/s).  The FLOPs are the matrix-core FLOPs the kernel issues (whole "
                "diagonal tiles, all four split products), not the algorithmic N(N+1) Ng.  "
                "busy/gui = SQ_VALU_MFMA_BUSY_CYCLES / GRBM_GUI_ACTIVE, raw.", "",
            "| kernel | dispatches | median us | type | MFMA GFLOP/dispatch | TFLOP/s | frac of peak | busy/gui |",
            "|---|---:|---:|---|---:|---:|---:|---:|"]
    for k, r in sorted(res.items(), key=lambda kv: -sum(kv[1]["mfma_flops"].values())):
        b = "" if r["busy_per_gui"] is None else f"{r['busy_per_gui']:.1f}"
        out.append(f"| `{short(k)}` | {r['dispatches']} | {r['median_us']:.1f} | {r['type']} | "
                   f"{sum(r['mfma_flops'].values()) / 1e9:.2f} | {r['tflops']:.1f} | "
                   f"{r['frac_of_peak']:.3f} | {b} |")
    return "\n".join(out) + "\n"


def source_sha(name):
    path = os.path.join(HERE, "csrc", name)
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


def per_kernel(path):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def short(name):
    for pre in ("void pou::(anonymous namespace)::", "pou::(anonymous namespace)::"):
        if name.startswith(pre):
            name = ("void " if pre.startswith("void") else "") + name[len(pre):]
    return name[:80] + ("..." if len(name) > 80 else "")


def summarise(fetch_csv, write_csv, block, N, n):
    fetch = per_kernel(fetch_csv)
    write = per_kernel(write_csv)
    copy = [k for k in fetch if "k_convert<float, float>" in k][0]
    sf = block / (fetch[copy][0] * 1024.0)
    sw = block / (write[copy][0] * 1024.0)
    kernels = {}
    for k in fetch:
        f = fetch[k][0]
        w = write.get(k, (0.0, 0))[0]
        kernels[k] = {"fetch_kib": f, "write_kib": w, "dispatches": fetch[k][1],
                      "hbm_bytes": f * 1024 * sf + w * 1024 * sw}
    ng = n ** 3
    groups = {}
    for g, (frag, src) in GROUP_KERNELS.items():
        hits = [k for k in kernels if frag in k]
        if not hits:
            continue
        rec = kernels[hits[0]]
        alg = algorithmic_bytes(g, N, ng)
        groups[g] = {"kernel": frag, "fetch_kib_per_dispatch": round(rec["fetch_kib"], 1),
                     "write_kib_per_dispatch": round(rec["write_kib"], 1),
                     "bytes_per_launch": int(round(rec["hbm_bytes"])),
                     "algorithmic_bytes": alg,
                     "ratio_to_algorithmic": round(rec["hbm_bytes"] / alg, 3),
                     "source_file": src, "source_sha": source_sha(src)}
    calib = {"copy_kernel": short(copy), "block_bytes": block,
             "copy_fetch_kib": fetch[copy][0], "copy_write_kib": write[copy][0],
             "scale_fetch": sf, "scale_write": sw}
    return {"calibration": calib, "groups": groups, "kernels": kernels}


def markdown(res, cmds):
    c = res["calibration"]
    out = ["# HBM traffic per launch from FETCH_SIZE / WRITE_SIZE (mixed96, mixed precision)", "",
           "Two counter runs, one counter each, then scaled by the counts of a plain copy "
           "kernel of known size ($REPO: the repository root, $OUT: an output directory):", ""]
    out += ["    " + x for x in cmds]
    out += ["", f"Copy calibration (k_convert<float,float>, {c['block_bytes']:,} bytes read and "
                f"written): FETCH_SIZE {c['copy_fetch_kib']:.0f} KiB -> scale {c['scale_fetch']:.4f}; "
                f"WRITE_SIZE {c['copy_write_kib']:.0f} KiB -> scale {c['scale_write']:.4f}.", "",
            "| group | kernel | FETCH KiB | WRITE KiB | HBM bytes/launch | algorithmic | ratio |",
            "|---|---|---:|---:|---:|---:|---:|"]
    for g, r in res["groups"].items():
        out.append(f"| {g} | `{r['kernel']}` | {r['fetch_kib_per_dispatch']:.0f} | "
                   f"{r['write_kib_per_dispatch']:.0f} | {r['bytes_per_launch']:,} | "
                   f"{r['algorithmic_bytes']:,} | {r['ratio_to_algorithmic']} |")
    out += ["", "All kernels (scaled HBM MB per dispatch):", "", "| kernel | dispatches | MB |",
            "|---|---:|---:|"]
    for k, r in sorted(res["kernels"].items(), key=lambda kv: -kv[1]["hbm_bytes"]):
        out.append(f"| `{short(k)}` | {r['dispatches']} | {r['hbm_bytes'] / 1e6:.1f} |")
    return "\n".join(out) + "\n"


def sources_line():
    names = ["grid_kernels.hip", "dense_kernels.hip", "nonlocal_kernels.hip", "engine.hip"]
    return "Sources: " + ", ".join(f"{n} {source_sha(n)}" for n in names
                                   if os.path.exists(os.path.join(HERE, "csrc", n))) + "."


def stats_markdown(stats_csv, title, cmds, top=24):
    rows = list(csv.DictReader(open(stats_csv)))
    out = [f"# rocprofv3 kernel statistics: {title}", "",
           "Command ($REPO: the repository root, $OUT: an output directory):", ""]
    out += ["    " + x for x in cmds]
    out += ["", sources_line(), "",
            "| kernel | calls | avg us | min us | max us | total % |", "|---|---:|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                   f"{float(r['Percentage']):.2f} |")
    return "\n".join(out) + "\n"


def main():
    if "--stats" in sys.argv:
        ap = argparse.ArgumentParser()
        ap.add_argument("--stats")
        ap.add_argument("--md", required=True)
        ap.add_argument("--title", default="")
        ap.add_argument("--cmd", action="append", default=[])
        a = ap.parse_args()
        open(a.md, "w").write(stats_markdown(a.stats, a.title, a.cmd))
        return
    if "--mfma" in sys.argv:
        ap = argparse.ArgumentParser()
        ap.add_argument("--mfma", nargs=2, metavar=("COUNTER_CSV", "TRACE_CSV"))
        ap.add_argument("--md")
        ap.add_argument("--title", default="")
        ap.add_argument("--cmd", action="append", default=[])
        a = ap.parse_args()
        res = mfma_summary(*a.mfma)
        if a.md:
            open(a.md, "w").write(mfma_markdown(res, a.title, a.cmd).rstrip("\n") + "\n\n"
                                  + sources_line() + "\n")
        else:
            json.dump(res, sys.stdout, indent=1)
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("fetch")
    ap.add_argument("write")
    ap.add_argument("block", type=float)
    ap.add_argument("--json")
    ap.add_argument("--md")
    ap.add_argument("--norb", type=int, default=128)
    ap.add_argument("--n", type=int, default=96)
    a = ap.parse_args()
    res = summarise(a.fetch, a.write, a.block, a.norb, a.n)
    cmds = [
        "cd /tmp && TMPDIR=/tmp rocprofv3 --pmc FETCH_SIZE --output-format csv -d $OUT/fetch -o run -- python3 $REPO/bench.py --steps 3 --warmup 1 --no-converge --no-cpu-baseline --calibrate-copy --no-extras",
        "cd /tmp && TMPDIR=/tmp rocprofv3 --pmc WRITE_SIZE --output-format csv -d $OUT/write -o run -- python3 $REPO/bench.py --steps 3 --warmup 1 --no-converge --no-cpu-baseline --calibrate-copy --no-extras",
        f"python -m paper_1510_07230_amd.counters $OUT/fetch/run_counter_collection.csv $OUT/write/run_counter_collection.csv {int(a.block)} --json profiles/traffic_mixed96.json --md profiles/traffic_mixed96.md",
    ]
    if a.json:
        rec = {"_commands": cmds, "calibration": res["calibration"], "groups": res["groups"]}
        json.dump(rec, open(a.json, "w"), indent=1)
    if a.md:
        open(a.md, "w").write(markdown(res, cmds))
    if not a.json and not a.md:
        json.dump(res, sys.stdout, indent=1)


if __name__ == "__main__":
    main()
