"""Benchmark: GMRES + MRCM-OS solves per second on one MI355X.

A step is one solve of A p = b to a true FP64 relative residual of 1e-8 with
right-preconditioned GMRES(10) and the MRCM-OS operator, the operator's
factorisations resident in HBM (setup excluded from the timed region and
reported separately).  Every step runs the whole hot path: local Robin
solves with trace moments, interface solve, reconstruction, smoothing
residual and patch solves, output projection, the fine operator, Gram-Schmidt
and the solution update.

Prints one JSON line (rank 0).  Besides the contract keys it carries the
roofline of the dominant kernel (measured live with HIP events on the
library's stream), the oracle timed on the host cores on a bounded sample,
cell-DOF/s, p50/p99 latency of the timed solves and setup-inclusive
throughput.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
CSRC = os.path.join(ROOT, "paper_2606_08883_amd", "csrc")


def kernel_source_hash() -> str:
    """First 16 hex digits of the sha256 of the kernel sources."""
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "setup_jobs.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, workload: str, precision: int):
    """HBM bytes per launch of a kernel from the committed PMC summary
    (FETCH_SIZE and WRITE_SIZE scaled by a copy of known size), or None when
    no summary covers this kernel, workload and precision or the kernel
    sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith(" "):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if (kv.get("kernel") != kernel or kv.get("workload") != workload
            or kv.get("precision") != str(precision)
            or kv.get("source_sha256_16") != kernel_source_hash()):
        return None
    return int(kv["traffic_bytes_per_launch"])


def words(precision: int) -> tuple:
    """(work-vector word, factor storage word) in bytes of a precision mode."""
    return (4 if precision == 1 else 8), (8 if precision == 0 else 4)


DTYPES = {0: "f64", 1: "f32", 2: "f32-storage/f64-arith"}
PRECISION_NAMES = {0: "fp64", 1: "fp32 local/smoothing apply, fp64 interface + krylov",
                   2: "fp32 factor storage with fp64 arithmetic, fp64 interface + krylov"}


def box_cols(max_bx: int) -> int:
    """Column width of a box launch (the library's launch widths)."""
    for c in (16, 20, 24, 32, 36, 40, 48):
        if max_bx <= c:
            return c
    return 64


def algorithmic_bytes(cfg, maps, tw: int, sw: int) -> dict:
    """Algorithmic bytes of one launch of the local and patch kernels
    (tw: bytes of a work-vector word, sw: bytes of a stored factor word).

    The factor of a box bx cells wide and by rows is stored as by half
    blocks of rows x bx words (rows = cols / 2 + 1, cols the launch's column
    width) plus by x bx couplings; the algorithmic count reads them once.
    Local solve of subdomain i on its oversampled box (ox x oy cells, owned
    bx x by): factor and couplings, r read on the box (8 B/cell, FP64), p
    written on the owned cells (tw/cell), the four trace weights of every
    face of Gamma_i read (32 B per face) and two moments per dof written
    (16 B per dof).
    Patch solve of patch i (px x py cells, owned bx x by): factor and
    couplings, the residual read on the patch (tw/cell), p read and written
    on the owned cells (2 tw/cell).
    """
    b = maps["boxes"]
    bx = (b[:, 1] - b[:, 0]).astype(np.int64)
    by = (b[:, 3] - b[:, 2]).astype(np.int64)
    o = maps["oboxes"]
    ox = (o[:, 1] - o[:, 0]).astype(np.int64)
    oy = (o[:, 3] - o[:, 2]).astype(np.int64)
    lrows = box_cols(int(ox.max())) // 2 + 1
    local = int(np.sum(oy * ox * lrows * sw + oy * ox * sw + oy * ox * 8 + by * bx * tw))
    dofs = maps["dof_table"]
    faces = 0
    for i in range(len(b)):
        sides = set(dofs[dofs[:, 0] == i][:, 1].tolist()) if len(dofs) else set()
        faces += sum(int(by[i]) if s <= 1 else int(bx[i]) for s in sides)
    local += faces * 32 + len(dofs) * 16
    p = maps["pboxes"]
    px = (p[:, 1] - p[:, 0]).astype(np.int64)
    py = (p[:, 3] - p[:, 2]).astype(np.int64)
    prows = box_cols(int(px.max())) // 2 + 1
    patch = int(np.sum(py * px * prows * sw + py * px * sw + py * px * tw + 2 * bx * by * tw))
    return {"local": local, "patch": patch}


def interface_solve(ctx, phases) -> dict:
    """The interface solve (right-hand side, forward and backward levels),
    reported beside the roofline: its levels are latency-bound (each a
    dependent launch reading a few MB), so its effective bandwidth, the
    factor bytes per apply over its time per apply, sits far below the HBM
    peak."""
    ms = phases["coarse"][0] / max(1, phases["coarse"][1])
    nbytes = ctx.query("coarse_bytes")
    return {"bound": "latency", "launches_per_apply": int(ctx.query("coarse_launches")) + 1,
            "factor_bytes_per_apply": nbytes, "ms_per_apply": ms,
            "effective_GB_s": nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None}


def cpu_baseline(workload_name: str, gpu_iterations: int, budget_s: float = 25.0) -> dict:
    """Time the oracle (as it stands) on the host: its setup for the same
    workload, then GMRES inner steps until the budget is spent; the solve
    time is the mean inner-step time times the iterations of one solve."""
    code = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, %r)
from oracle.mrcm import MRCM
from oracle.gmres import gmres
from paper_2606_08883_amd.configs import WORKLOADS
w = WORKLOADS[%r]
K = w.permeability()
t0 = time.perf_counter()
mr = MRCM(K, **w.oracle_args())
t_setup = time.perf_counter() - t0
b = w.rhs()
steps = 0
t0 = time.perf_counter()
while True:
    res = gmres(lambda x: mr.A @ x, mr.apply, b, rtol=1e-8, restart=10, maxit=2)
    steps += res.iterations
    if time.perf_counter() - t0 > %f:
        break
t_step = (time.perf_counter() - t0) / steps
print(json.dumps({"setup_s": t_setup, "step_s": t_step, "steps": steps}))
""" % (ROOT, workload_name, budget_s)
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                         timeout=900)
    if out.returncode != 0:
        raise RuntimeError(out.stderr[-2000:])
    d = json.loads(out.stdout.strip().splitlines()[-1])
    solve_s = d["step_s"] * gpu_iterations
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle setup ({d['setup_s']:.1f} s, excluded) then {d['steps']} GMRES "
                       f"inner steps (T apply + A apply + MGS) of the same workload in "
                       f"{budget_s:.0f} s; solve time = mean step time "
                       f"({d['step_s'] * 1e3:.1f} ms) x {gpu_iterations} steps per solve")}


def rhs_of(w, ctx, dev):
    """b of a workload on the device: the corner sources of the no-flow
    workloads, or the library's assembly (mrcm_rhs) of the Dirichlet
    left/right data."""
    import torch
    if not any(w.bc):
        return torch.tensor(w.rhs(), dtype=torch.float64, device=dev)
    f, g = w.boundary_data()
    b = torch.empty(w.cells, dtype=torch.float64, device=dev)
    ctx.rhs(torch.tensor(f, dtype=torch.float64, device=dev),
            torch.tensor(g, dtype=torch.float64, device=dev), 1.0 / w.nx, b)
    return b


def apply_only(args, w, ctx, b, setup_s) -> int:
    """Applications of T per second on the workload (no GMRES)."""
    import torch

    from paper_2606_08883_amd import binding as B
    z = torch.empty_like(b)
    r = b.clone()
    for _ in range(args.warmup):
        ctx.apply(r, z)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.apply(r, z)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ctx.timing(True)
    for _ in range(args.steps):
        ctx.apply(r, z)
    torch.cuda.synchronize()
    phases = ctx.timing_read()
    ctx.timing(False)
    maps = B.maps(w.binding_config())
    abytes = algorithmic_bytes(w, maps, *words(w.precision))
    dom = max(("local", "patch"), key=lambda k: phases[k][0])
    avg_ms = phases[dom][0] / max(1, phases[dom][1])
    achieved = abytes[dom] / (avg_ms * 1e-3) / 1e9
    out = {"metric": "MRCM-OS preconditioner applications/s", "value": args.steps / elapsed,
           "unit": "applies/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "dtype": DTYPES[w.precision], "data": "synthetic",
           "config": {"workload": w.name, "cells": w.cells, "subdomains": int(maps["boxes"].shape[0])},
           "setup_s": setup_s,
           "autotune": {"ms": ctx.query("tune_ms"), "changes": ctx.query("tune_changes")},
           "device_gb": ctx.query("device_bytes") / 1e9,
           "coarse_min_pivot_ratio": ctx.query("coarse_pivot"),
           "phase_ms_per_launch": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in phases.items()},
           "algorithmic_bytes_per_launch": abytes,
           "roofline": {"bound": "hbm", "kernel": f"k_{dom}", "achieved": achieved,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                        "traffic": recorded_traffic(f"k_{dom}", f"{w.name}{w.nx}",
                                                    w.precision),
                        "traffic_unit": "bytes per launch", "avg_launch_ms": avg_ms},
           "interface_solve": interface_solve(ctx, phases)}
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def serve(args) -> int:
    """Serving run: capacity from a closed-loop burst, then a Poisson stream at
    0.8 of it; request latency from arrival to answer (setup included)."""
    from paper_2606_08883_amd import serving as S

    params = None if args.precision is None else dict(precision=args.precision)
    prec = S.SERVE_PARAMS["precision"] if args.precision is None else args.precision
    fp = (lambda r: S.footprint_of(r, params))
    # a set-up takes the host cores divided among the set-ups in progress
    B = S.gpu_solver(params, keep=False)
    warm = S.make_payload(S.Request(0, 128, 2.0, 999, 1999, 2, 0.0))
    S.Server(B, max_active=1).run([warm], realtime=False)
    burst = [S.make_payload(r) for r in S.make_requests(max(4, args.requests // 2), rate=None,
                                                          seed=5)]
    print(f"bench: serving burst of {len(burst)} requests", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    res = S.Server(B, max_active=args.max_active, footprint=fp).run(burst, realtime=False)
    cap = len(res) / (time.perf_counter() - t0)
    rate = 0.8 * cap
    reqs = [S.make_payload(r) for r in S.make_requests(args.requests, rate=rate, seed=4)]
    print(f"bench: capacity {cap:.2f} requests/s; Poisson stream of {len(reqs)} at "
          f"{rate:.2f}/s", file=sys.stderr, flush=True)
    server = S.Server(B, max_active=args.max_active, footprint=fp)
    t0 = time.perf_counter()
    res = server.run(reqs)
    wall = time.perf_counter() - t0
    sm = S.summary(res, wall)
    if not sm["all_converged"]:
        raise RuntimeError("a served request did not converge")
    sizes = sorted({r.n for r in reqs})
    out = {"metric": "GMRES+MRCM-OS solves/s & cell-DOF/s at rel.res 1e-8; p50/p99 solve latency",
           "value": sm["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": len(reqs),
           "warmup": 1, "ms_per_step": 1e3 * wall / len(reqs), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": DTYPES[prec], "data": "synthetic",
           "config": {"workload": f"serving: {len(reqs)} requests, grids {sizes} (uniform), "
                                  f"log-normal sigma U[1,3] corr. 16, 8 injector/producer "
                                  f"pairs each, Poisson arrivals at 0.8 x closed-loop capacity "
                                  f"({rate:.2f}/s), {args.max_active} slots",
                      "parallelism": "single GPU, requests in flight on separate streams"},
           "cell_dof_per_s": sm["cell_dof_per_s"], "latency_ms": sm["latency_ms"],
           "requests_per_s": sm["requests_per_s"], "capacity_requests_per_s": cap,
           "setup_s_mean": sm["setup_s_mean"], "solve_s_mean": sm["solve_s_mean"],
           "iterations_per_solve": sm["iterations_mean"], "peak_active": server.peak_active,
           "peak_footprint_gb": server.peak_bytes / 1e9}
    print(json.dumps(out), flush=True)
    return 0


def multi_rhs(args, w, ctx) -> dict:
    """Throughput of one gmres call on nrhs injector/producer right-hand sides
    (seeded cell pairs) on the same context, one at a time and with several in
    flight: lanes (streams) x width (right-hand sides sharing one
    multi-column application of T per step).  Each right-hand side's solution
    is the same bit for bit in every arrangement (checked here)."""
    import torch

    from paper_2606_08883_amd import workloads as wl

    b = torch.tensor(wl.random_pairs(w.nx, w.ny, args.nrhs, 2024), dtype=torch.float64,
                     device="cuda:0").contiguous()
    out = {"nrhs": args.nrhs, "rhs": "injector/producer cell pairs, seed 2024"}
    ref = None
    for lanes, width in ((1, 1), (4, 1), (1, 8), (2, 4)):
        ctx.set_lanes(lanes)
        ctx.set_batch(width)
        p = torch.zeros_like(b)
        ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)  # warm-up: lanes, graphs
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            st = ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        if ref is None:
            ref = p.clone()
        elif not torch.equal(ref, p):
            raise RuntimeError("lanes or batch width changed a solution")
        out[f"lanes_{lanes}_width_{width}"] = {
            "solves_per_s": args.nrhs / dt, "ms_per_call": 1e3 * dt,
            "iterations_per_solve": st.iterations / args.nrhs}
        print(f"bench: {args.nrhs} rhs on {lanes} lane(s) of width {width}: "
              f"{args.nrhs / dt:.1f} solves/s", file=sys.stderr, flush=True)
    ctx.set_lanes(4)
    ctx.set_batch(4)
    return out


INCLUSION_ROWS = [("MRCM", 0, 0), ("2h", 2, 0), ("4h", 4, 0), ("2h,2S", 2, 2), ("2h,4S", 2, 4),
                  ("4h,2S", 4, 2), ("4h,4S", 4, 4)]


def inclusions(args) -> int:
    """GMRES(10) on the thin-inclusion fields (the stand-ins for the paper's
    inclusion experiments): every row of the paper's tables (oversampling 0,
    2 or 4 cells, 0, 2 or 4 smoothing sweeps) under 4 x 4 and 8 x 8
    partitions, FP64, relative tolerance 1e-8.  Prints one JSON line with
    the inner steps, restart cycles and final true residual of each run."""
    import torch

    from paper_2606_08883_amd import binding as B
    from paper_2606_08883_amd.configs import WORKLOADS

    dev = torch.device("cuda:0")
    results = []
    for kind in ("high", "low", "both"):
        w0 = WORKLOADS[f"incl-{kind}"]
        K = torch.tensor(w0.permeability(), dtype=torch.float64, device=dev)
        f, g = w0.boundary_data()
        ft = torch.tensor(f, dtype=torch.float64, device=dev)
        gt = torch.tensor(g, dtype=torch.float64, device=dev)
        for s in (40, 20):
            for name, l, k in INCLUSION_ROWS:
                w = w0.with_(s=s, oversample=l, sweeps=k)
                print(f"bench: inclusions {kind} {160 // s}x{160 // s} {name}", file=sys.stderr,
                      flush=True)
                ctx = B.Context(w.binding_config(), K)
                b = torch.empty(w.cells, dtype=torch.float64, device=dev)
                ctx.rhs(ft, gt, 1.0 / w.nx, b)
                p = torch.zeros_like(b)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st = ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=300, raise_on_noconv=False)
                torch.cuda.synchronize()
                results.append({"field": kind, "partition": f"{160 // s}x{160 // s}", "row": name,
                                "iterations": st.iterations, "cycles": st.cycles,
                                "converged": bool(st.converged), "final_relres": st.final_relres,
                                "solve_ms": 1e3 * (time.perf_counter() - t0)})
                ctx.close()
    print(json.dumps({"metric": "GMRES(10) inner steps and restart cycles to rel.res 1e-8",
                      "data": "synthetic thin-inclusion fields, 160x160, Dirichlet left/right",
                      "dtype": "f64", "results": results}), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched",
                    choices=["small", "channel", "batched", "large"])
    ap.add_argument("--precision", type=int, default=None, help="0 FP64 apply, 1 FP32 apply, 2 FP32-stored factors with FP64 arithmetic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--nrhs", type=int, default=8,
                    help="right-hand sides of the extra multi-RHS measurement (0: skip)")
    ap.add_argument("--apply-only", action="store_true",
                    help="time preconditioner applications T r instead of solves")
    ap.add_argument("--serve", action="store_true",
                    help="serving workload: a Poisson stream of requests of mixed grid sizes "
                         "(128^2 .. 1024^2), each with its own log-normal field and 8 "
                         "injector/producer right-hand sides, served with continuous batching")
    ap.add_argument("--inclusions", action="store_true",
                    help="GMRES steps and cycles on the thin-inclusion fields for every "
                         "oversampling / smoothing row of the paper's inclusion tables")
    ap.add_argument("--requests", type=int, default=512, help="requests of the serving run")
    ap.add_argument("--max-active", type=int, default=8, help="serving slots")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB, as a runtime copy and "
                         "as an elementwise kernel (known-size kernels that scale the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the solver runs on a single device, with no "
              "multi-GPU mode; run it with --gpus 1", file=sys.stderr)
        return 2

    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(max(1, args.steps)):
            dst.copy_(src)
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8,
                          "copies": max(1, args.steps)}), flush=True)
        return 0

    if args.serve:
        return serve(args)
    if args.inclusions:
        return inclusions(args)

    from paper_2606_08883_amd import binding as B
    from paper_2606_08883_amd.configs import WORKLOADS

    w = WORKLOADS[args.workload]
    if args.precision is not None:
        w = w.with_(precision=args.precision)
    dev = torch.device("cuda:0")
    K = torch.tensor(w.permeability(), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    print(f"bench: workload {w.name} {w.nx}x{w.ny} precision {w.precision}", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    ctx = B.Context(w.binding_config(), K)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    b = rhs_of(w, ctx, dev)
    p = torch.zeros_like(b)
    print(f"bench: setup {setup_s:.2f} s", file=sys.stderr, flush=True)
    if args.apply_only:
        return apply_only(args, w, ctx, b, setup_s)
    for _ in range(args.warmup):
        st = ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
    torch.cuda.synchronize()
    lat = []
    its = []
    relres = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        t1 = time.perf_counter()
        st = ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
        lat.append(time.perf_counter() - t1)
        its.append(st.iterations)
        relres.append(st.final_relres)
        if not st.converged:
            raise RuntimeError("GMRES did not converge")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # Kernel durations: the same solves again with HIP events recorded around
    # every phase on the library's stream (eager launches; kernels are the
    # same as in the captured graphs of the timed region).
    ctx.timing(True)
    for _ in range(args.steps):
        ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
    torch.cuda.synchronize()
    phases = ctx.timing_read()
    ctx.timing(False)
    multi = multi_rhs(args, w, ctx) if args.nrhs > 0 else None
    n = w.cells
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps / elapsed
    maps = B.maps(w.binding_config())
    abytes = algorithmic_bytes(w, maps, *words(w.precision))
    # dominant kernel = the phase with the largest accumulated device time
    dom = max(("local", "patch"), key=lambda k: phases[k][0])
    avg_ms = phases[dom][0] / max(1, phases[dom][1])
    achieved = abytes[dom] / (avg_ms * 1e-3) / 1e9
    apply_ms = sum(v[0] for v in phases.values()) / max(1, phases["local"][1])
    out = {
        "metric": "GMRES+MRCM-OS solves/s & cell-DOF/s at rel.res 1e-8; p50/p99 solve latency",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[w.precision],
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.nx}x{w.ny} cells, {maps['boxes'].shape[0]} "
                               f"subdomains of {w.s}x{w.s}, oversampling {w.oversample}, "
                               f"{w.sweeps} smoothing sweep(s), overlap {w.overlap}, "
                               f"alpha {w.alpha}, field {w.field}, no-flow, corner sources",
                   "cells": n, "precision": PRECISION_NAMES[w.precision],
                   "rtol": 1e-8, "restart": 10, "parallelism": "single GPU"},
        "cell_dof_per_s": value * n,
        "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                       "p99": float(np.percentile(lat, 99) * 1e3)},
        "iterations_per_solve": float(np.mean(its)),
        "final_relres_max": float(np.max(relres)),
        "setup_s": setup_s,
        "autotune": {"ms": ctx.query("tune_ms"), "changes": ctx.query("tune_changes")},
        "solves_per_s_incl_setup": 1.0 / (setup_s + elapsed / args.steps),
        "apply_ms": apply_ms,
        "phase_ms_per_launch": {k: (v[0] / v[1] if v[1] else 0.0) for k, v in phases.items()},
        "roofline": {"bound": "hbm", "kernel": f"k_{dom}", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(f"k_{dom}", f"{w.name}{w.nx}", w.precision),
                     "traffic_unit": "bytes per launch",
                     "algorithmic_bytes_per_launch": abytes[dom],
                     "avg_launch_ms": avg_ms},
        "interface_solve": interface_solve(ctx, phases),
    }
    if multi:
        out["multi_rhs"] = multi
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w.name, int(round(np.mean(its))))
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
