"""Summarise rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs of bench.py.

Usage: python -m paper_1510_07230_amd.counters FETCH_CSV WRITE_CSV BLOCK_BYTES
BLOCK_BYTES is the size of the plain copy (k_convert<float,float>) that the
--calibrate-copy run performs: it reads and writes BLOCK_BYTES once, which
scales the counters to bytes.  Prints per-kernel KiB per dispatch, the scale
factors and the scaled HBM bytes per launch.
"""
import csv
import json
import sys
from collections import defaultdict


def per_kernel(path):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[r["Kernel_Name"]].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def main():
    fetch = per_kernel(sys.argv[1])
    write = per_kernel(sys.argv[2])
    block = float(sys.argv[3])
    copy = [k for k in fetch if "k_convert<float, float>" in k][0]
    sf = block / (fetch[copy][0] * 1024.0)
    sw = block / (write[copy][0] * 1024.0)
    out = {"copy_kernel": copy, "copy_fetch_kib": fetch[copy][0], "copy_write_kib": write[copy][0],
           "scale_fetch": sf, "scale_write": sw, "kernels": {}}
    for k in sorted(fetch, key=lambda k: -fetch[k][0]):
        f = fetch[k][0]
        w = write.get(k, (0.0, 0))[0]
        out["kernels"][k] = {"fetch_kib": f, "write_kib": w, "dispatches": fetch[k][1],
                             "hbm_bytes": f * 1024 * sf + w * 1024 * sw}
    json.dump(out, sys.stdout, indent=1)


if __name__ == "__main__":
    main()
