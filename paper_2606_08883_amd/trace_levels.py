"""Per-level durations of the interface solve from a rocprofv3 kernel trace.

Usage: ``python -m paper_2606_08883_amd.trace_levels DIR [APPS]`` where DIR
holds the ``*_kernel_trace.csv`` of a ``rocprofv3 --kernel-trace
--output-format csv`` run.  Dispatches are ordered by start time; each
maximal run of interface kernels (``k_coarse_rhs``, ``k_coarse_fwd``,
``k_coarse_bwd``, ``k_coarse_resid``, ``k_coarse_add``) is one interface
solve, and the last APPS solves (default 4) are printed launch by launch:
kernel, workgroups, threads per workgroup and the duration of each solve's
launch in microseconds, then the per-launch mean and the solve total.
"""
from __future__ import annotations

import csv
import glob
import sys


def solves(trace_dir: str) -> list:
    path = glob.glob(f"{trace_dir}/**/*kernel_trace.csv", recursive=True)
    if not path:
        raise FileNotFoundError(f"no kernel_trace.csv under {trace_dir}")
    rows = sorted(csv.DictReader(open(path[0])), key=lambda r: int(r["Start_Timestamp"]))
    out, cur = [], []
    for r in rows:
        name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0].split("::")[-1]
        if name.startswith("k_coarse"):
            wg = int(r["Workgroup_Size_X"])
            cur.append((name, int(r["Grid_Size_X"]) // max(wg, 1), wg,
                        (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
        elif cur:
            out.append(cur)
            cur = []
    if cur:
        out.append(cur)
    return out


def main(argv: list) -> int:
    if len(argv) < 2 or argv[1].startswith("-") or (len(argv) > 2 and not argv[2].isdigit()):
        print(__doc__.strip())
        return 0 if len(argv) > 1 and argv[1] in ("-h", "--help") else 2
    apps = int(argv[2]) if len(argv) > 2 else 4
    try:
        sv = solves(argv[1])
    except FileNotFoundError as e:
        print(e, file=sys.stderr)
        return 1
    if not sv:
        print(f"no interface solve in the trace under {argv[1]}", file=sys.stderr)
        return 1
    last = sv[-apps:]
    n = min(len(a) for a in last)
    print(f"interface solves in the trace: {len(sv)}; the last {len(last)}, launch by launch (us)")
    total = 0.0
    for i in range(n):
        name, wgs, wg = last[0][i][:3]
        times = [a[i][3] for a in last]
        mean = sum(times) / len(times)
        total += mean
        print(f"{i:3d} {name:15s} workgroups {wgs:6d} x {wg:3d}  "
              + " ".join(f"{t:7.2f}" for t in times) + f"   mean {mean:7.2f}")
    print(f"solve total (sum of launch means): {total:.1f} us")
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv))
