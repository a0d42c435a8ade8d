"""Calibration of the oracle's readings against the paper's iteration counts
(Section 4.1, Tables 2 and 3).  Test infrastructure like the rest of
oracle/: it runs the oracle only.

The paper's two analytic problems (256 x 256 cells, pressure given on the
left and right sides, no flow on the others, GMRES(10) tested at each cycle
end against the absolute tolerance 1e-8) are solved with T built under the
base reading (interface degree d = 1, alpha = 10, Robin length L = H, patch
overlap delta = 2, restricted additive Schwarz) and under variants that
change one of these at a time:

  d0, d2        Legendre degree 0 or 2 of the multiplier spaces;
  alpha1/100    alpha = 1 or 100 in beta = alpha L / K_H;
  Lh            Robin length L = h instead of H;
  delta1/4      patch overlap of 1 or 4 cells;
  msm           multiplicative Schwarz smoothing instead of RAS.

For every variant and table it prints the restart cycles of each setting
(Table 1's notation: MRCM, lh, lh,kS) per partition, the paper's count in
brackets, and the summed absolute difference over the oversampled settings.

Usage:  python -m oracle.calibrate_tables [--parts 4 8] [--variants base d0 ...]
                                          [--tables 2 3] [--jobs N]
"""
import argparse
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from oracle.discretization import rhs as assemble_rhs
from oracle.gmres import gmres
from oracle.mrcm import MRCM
from paper_2606_08883_amd import workloads as wl

N = 256
GOLDEN = os.path.join(os.path.dirname(__file__), os.pardir, "tests", "golden",
                      "paper_tables_2_3.txt")
PARTS = (2, 4, 8, 16)
SETTINGS = {"MRCM": (0, 0), "2h": (2, 0), "4h": (4, 0), "2h,2S": (2, 2), "2h,4S": (2, 4),
            "4h,2S": (4, 2), "4h,4S": (4, 4)}
BASE = {"degree": 1, "alpha": 10.0, "beta_len": "H", "overlap": 2, "schwarz": "additive"}
VARIANTS = {
    "base": {},
    "d0": {"degree": 0},
    "d2": {"degree": 2},
    "alpha1": {"alpha": 1.0},
    "alpha100": {"alpha": 100.0},
    "Lh": {"beta_len": "h"},
    "delta1": {"overlap": 1},
    "delta4": {"overlap": 4},
    "msm": {"schwarz": "multiplicative"},
}


def paper_counts() -> dict:
    """(table, setting) -> {partition: cycles} as printed in Tables 2-3."""
    out = {}
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            tab, name, *counts = line.split()
            out[(int(tab), name)] = dict(zip(PARTS, (int(c) for c in counts)))
    return out


def problem(table: int):
    """K, boundary types and b of Table 2 (constant K) or Table 3 (variable
    K), with the exact solution's trace as the Dirichlet data."""
    Kf, ff, pf = wl.manufactured("const" if table == 2 else "var")
    x, y = wl.cell_centres(N, N)
    yc = (np.arange(N) + 0.5) / N
    bc = (1, 1, 0, 0)
    g = {0: pf(np.zeros(N), yc), 1: pf(np.ones(N), yc)}
    K = Kf(x, y)
    return K, bc, assemble_rhs(K, N, N, bc, ff(x, y), g, 1.0 / N)


def cycles(job) -> tuple:
    """Restart cycles of one (variant, table, partition, setting)."""
    variant, table, parts, name = job
    opts = dict(BASE, **VARIANTS[variant])
    K, bc, b = problem(table)
    l, k = SETTINGS[name]
    s = N // parts
    mr = MRCM(K, N, N, bc, s, s, l, opts["alpha"], opts["beta_len"], k, opts["overlap"],
              opts["degree"], schwarz=opts["schwarz"])
    res = gmres(lambda v: mr.A @ v, mr.apply, b, restart=10, maxit=300,
                check_every_step=False, atol=1e-8)
    return job, (res.restarts if res.converged else None)


def _one_thread():
    """Pool initialiser: one BLAS thread per worker process."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--parts", type=int, nargs="+", default=[4, 8])
    ap.add_argument("--variants", nargs="+", default=list(VARIANTS))
    ap.add_argument("--tables", type=int, nargs="+", default=[2, 3])
    ap.add_argument("--jobs", type=int, default=min(8, os.cpu_count() or 1))
    args = ap.parse_args()
    gold = paper_counts()
    jobs = [(v, t, p, s) for v in args.variants for t in args.tables for p in args.parts
            for s in SETTINGS]
    with ProcessPoolExecutor(args.jobs, initializer=_one_thread) as ex:
        got = dict(ex.map(cycles, jobs))
    head = " | ".join(f"{p}x{p}" for p in args.parts)
    for v in args.variants:
        for t in args.tables:
            diff = 0
            print(f"\nvariant {v}, Table {t}: cycles (paper)   [{head}]")
            for s in SETTINGS:
                cells = []
                for p in args.parts:
                    c = got[(v, t, p, s)]
                    ref = gold[(t, s)][p]
                    cells.append(f"{c if c is not None else '300+':>4} ({ref})")
                    if s != "MRCM":
                        diff += abs((c if c is not None else 30) - ref)
                print(f"  {s:7s} " + " | ".join(cells))
            print(f"  sum |cycles - paper| over the oversampled settings: {diff}")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
