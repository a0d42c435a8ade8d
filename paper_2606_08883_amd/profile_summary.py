"""Summaries of rocprofv3 CSV output for the committed profiles.

  python -m paper_2606_08883_amd.profile_summary stats DIR APPLIES
      the kernel table of a ``--kernel-trace --stats`` run (run_kernel_stats.csv):
      calls, mean and total duration, share, and microseconds per application
      for kernels launched at least APPLIES times ("-" for the others: set-up
      kernels, or once-per-solve or once-per-cycle ones);
  python -m paper_2606_08883_amd.profile_summary traffic KERNEL WORKLOAD PRECISION \\
          FETCH_DIR WRITE_DIR COPY_FETCH_DIR COPY_WRITE_DIR BENCH_JSON
      HBM bytes per launch from two ``--pmc`` runs (FETCH_SIZE, then
      WRITE_SIZE, KiB per dispatch), each scaled by what the same counter reads
      for a 1 GiB device-to-device copy (``bench.py --copy-calibration 1024``),
      set against the algorithmic bytes per phase that the bench JSON line
      (BENCH_JSON, the ``--apply-only`` run's output) reports; ends with the
      key lines bench.py reads back (kernel, workload, precision, source hash,
      traffic_bytes_per_launch of KERNEL).
"""
from __future__ import annotations

import collections
import csv
import glob
import hashlib
import json
import os
import sys

CSRC = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
HASHED = ("kernels.hip", "device.h", "coarse.h", "setup_jobs.h")
PHASE_OF = {"k_local": "local", "k_reconstruct": "reconstruct", "k_residual": "residual",
            "k_patch": "patch"}


def kernel_source_hash() -> str:
    """First 16 hex digits of the sha256 of the 2-D kernel sources."""
    h = hashlib.sha256()
    for f in HASHED:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").replace("mrcm::", "").replace("void ", "")
    p = n.find("(")
    return n[:p] if p > 0 else n


def _csv(d: str, suffix: str) -> list:
    path = glob.glob(os.path.join(d, "**", f"*{suffix}"), recursive=True)
    if not path:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return list(csv.DictReader(open(path[0])))


def stats(d: str, applies: int) -> None:
    rows = _csv(d, "kernel_stats.csv")
    print(f"{'kernel':56s} {'calls':>6s} {'avg us':>9s} {'total ms':>9s} {'%':>6s} {'us/apply':>9s}")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        n, c = short(r["Name"]), int(r["Calls"])
        avg, tot = float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e6
        per = f"{tot * 1e3 / applies:9.2f}" if c >= applies else f"{'-':>9s}"
        print(f"{n[:56]:56s} {c:6d} {avg:9.2f} {tot:9.2f} {float(r['Percentage']):6.2f} {per}")


def counters(d: str) -> dict:
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in _csv(d, "counter_collection.csv"):
        k = short(r["Kernel_Name"])
        agg[k][0] += 1
        agg[k][1] += float(r["Counter_Value"])
    return agg


def traffic(kernel, workload, precision, dfetch, dwrite, cfetch, cwrite, bench_json) -> None:
    cf, cw = counters(cfetch), counters(cwrite)
    copy_k = [k for k in cf if "copyBuffer" in k][0]
    fetch_copy = cf[copy_k][1] / cf[copy_k][0]
    write_copy = cw[copy_k][1] / cw[copy_k][0]
    kib = 1024 * 1024  # the 1 GiB copy
    sf, sw = kib / fetch_copy, kib / write_copy
    lf, lw = counters(dfetch), counters(dwrite)
    with open(bench_json) as fh:
        line = [ln for ln in fh if ln.startswith("{")][-1]
    phases = json.loads(line)["phases"]
    print("Calibration: 1 GiB device-to-device copies (1048576 KiB read and written):")
    print(f"  runtime copy: FETCH_SIZE {fetch_copy:.1f} KiB, WRITE_SIZE {write_copy:.1f} KiB")
    print(f"scale factors: FETCH_SIZE {sf:.4f}, WRITE_SIZE {sw:.4f}\n")
    print(f"{'kernel':48s} {'launches':>8s} {'FETCH KiB':>12s} {'WRITE KiB':>12s} "
          f"{'scaled MB/launch':>17s}")
    target, ratios = None, []
    for k in sorted(lf, key=lambda k: -lf[k][1]):
        n, fe = lf[k]
        wr = lw.get(k, [1, 0.0])[1]
        per = (fe / n * sf + wr / n * sw) * 1024
        print(f"{k[:48]:48s} {n:8d} {fe / n:12.1f} {wr / n:12.1f} {per / 1e6:17.2f}")
        base = k.split("<")[0]
        if base == kernel:
            target = int(per)
        if base in PHASE_OF and PHASE_OF[base] in phases:
            alg = phases[PHASE_OF[base]]["algorithmic_bytes"]
            ratios.append((base, per, alg))
    print("\nCounted traffic over algorithmic bytes per launch (the bench's per-phase\n"
          "formulas: every factor word and vector read once):")
    for base, per, alg in ratios:
        print(f"  {base:14s} {per / 1e6:8.1f} MB / {alg / 1e6:8.1f} MB = {per / alg:.2f}")
    print(f"\nkernel: {kernel}\nworkload: {workload}\nprecision: {precision}")
    print(f"source_sha256_16: {kernel_source_hash()}\ntraffic_bytes_per_launch: {target}")


def main(argv: list) -> int:
    if len(argv) >= 4 and argv[1] == "stats":
        stats(argv[2], int(argv[3]))
        return 0
    if len(argv) >= 10 and argv[1] == "traffic":
        traffic(argv[2], argv[3], argv[4], *argv[5:10])
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv))
