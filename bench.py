"""Benchmark: GMRES + MRCM-OS solves per second on one MI355X.

A step is one solve of A p = b to a true FP64 relative residual of 1e-8 with
right-preconditioned GMRES(10) and the MRCM-OS operator, the operator's
factorisations resident in HBM (setup excluded from the timed region and
reported separately).  Every step runs the whole hot path: local solves on
the oversampled boxes with trace moments, interface solve, reconstruction,
smoothing residual and patch solves, output, the fine operator, Gram-Schmidt
and the solution update.

The default workload is the largest single-GPU configuration: 4096 x 4096
cells, the channel / log-normal mixture of contrast 1e8, 32 x 32 subdomains
grown by 4 cells, two smoothing sweeps, pressure 1 on the left side and 0 on
the right.  Prints one JSON line.  Besides the contract keys it carries:
  roofline         the dominant phase of the preconditioner apply (largest
                   device time), algorithmic bytes over its HIP-event
                   duration on the library's stream;
  phases           the same for every phase of the apply;
  precisions       solves/s of the same workload with FP64, FP32 and
                   FP32-stored factors;
  batched_1024     the 1024 x 1024 log-normal workload (4096 subdomains);
  serving          a short Poisson stream of mixed-size requests (p50/p99);
  cube_3d          the 3-D workload (96^3 cells, seven-point stencil): solves/s,
                   phases and the roofline entry of its dominant phase;
  cpu_baseline     the oracle timed on the host cores on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
CSRC = os.path.join(ROOT, "paper_2606_08883_amd", "csrc")
METRIC = "GMRES+MRCM-OS solves/s & cell-DOF/s at rel.res 1e-8; p50/p99 solve latency"


def kernel_source_hash() -> str:
    """First 16 hex digits of the sha256 of the kernel sources."""
    from paper_2606_08883_amd.profile_summary import kernel_source_hash as h
    return h()


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


def algorithmic_bytes(w, maps, ctx) -> dict:
    """Algorithmic bytes of one instance of every phase of the apply (tw:
    bytes of a work-vector word, sw: of a stored factor word).

    The factor of a box bx cells wide and by rows is stored as by half blocks
    of rows x bx words (rows = cols / 2 + 1, cols the launch's column width)
    plus by x bx couplings; the algorithmic count reads them once.
      local       per subdomain, on its oversampled box (ox x oy, owned
                  bx x by): factor and couplings, r read on the box (8 B/cell),
                  p written on the owned cells (tw), the four trace weights of
                  every face of Gamma_i (32 B) and two moments per dof (16 B);
      coarse      the interface solve: its factor matrices once per sweep and
                  the refinement residuals (mrcm_query's count);
      reconstruct the MBFs (sw per entry), the interface solution (8 B per
                  dof) and p read and written (2 tw per cell);
      residual    tx and ty (tw per face), r (8 B) and p (tw) read, rho
                  written (tw), per cell;
      patch       per patch (px x py, owned bx x by): factor and couplings, the
                  residual on the patch (tw), p read and written on the owned
                  cells (2 tw);
      finalize    p read (tw, twice with the zero-mean projection) and z
                  written (8 B) per cell.
    """
    tw, sw = words(w.precision)
    n = w.nx * w.ny
    b = maps["boxes"]
    bx = (b[:, 1] - b[:, 0]).astype(np.int64)
    by = (b[:, 3] - b[:, 2]).astype(np.int64)
    o = maps["oboxes"]
    ox = (o[:, 1] - o[:, 0]).astype(np.int64)
    oy = (o[:, 3] - o[:, 2]).astype(np.int64)
    lrows = box_cols(int(ox.max())) // 2 + 1
    local = int(np.sum(oy * ox * lrows * sw + oy * ox * sw + oy * ox * 8 + by * bx * tw))
    dofs = maps["dof_table"]
    nc = len(dofs)
    faces = 0
    if nc:
        sides = np.unique(dofs[:, :2], axis=0)
        lens = np.where(sides[:, 1] <= 1, by[sides[:, 0]], bx[sides[:, 0]])
        faces = int(lens.sum())
    local += faces * 32 + nc * 16
    per_sub = np.bincount(dofs[:, 0], minlength=len(b)) if nc else np.zeros(len(b), np.int64)
    recon = int(np.sum(per_sub * bx * by) * sw + nc * 8 + 2 * n * tw)
    p = maps["pboxes"]
    px = (p[:, 1] - p[:, 0]).astype(np.int64)
    py = (p[:, 3] - p[:, 2]).astype(np.int64)
    prows = box_cols(int(px.max())) // 2 + 1
    patch = int(np.sum(py * px * prows * sw + py * px * sw + py * px * tw + 2 * bx * by * tw))
    faces_all = w.ny * (w.nx + 1) + (w.ny + 1) * w.nx
    residual = faces_all * tw + n * (8 + 2 * tw)
    finalize = n * ((2 if not any(w.bc) else 1) * tw + 8)
    return {"local": local, "coarse": int(ctx.query("coarse_bytes")), "reconstruct": recon,
            "residual": residual, "patch": patch, "finalize": finalize}


PHASE_KERNELS = {"local": "k_local", "coarse": "interface solve (k_coarse_rhs, k_coarse_fwd "
                 "and k_coarse_bwd per level, k_coarse_resid and k_coarse_add per refinement)",
                 "reconstruct": "k_reconstruct", "residual": "k_residual", "patch": "k_patch",
                 "finalize": "k_sum + k_finalize"}


def phase_table(w, maps, ctx, phases) -> dict:
    """Per phase: device ms per instance (HIP events on the library's
    stream), algorithmic bytes per instance, achieved GB/s and fraction of
    the HBM peak."""
    ab = algorithmic_bytes(w, maps, ctx)
    out = {}
    napply = max(1, phases["local"][1])
    for k, (ms, cnt) in phases.items():
        if cnt == 0:
            continue
        avg = ms / cnt
        gbs = ab[k] / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
        out[k] = {"kernel": PHASE_KERNELS[k], "ms": avg, "per_apply": cnt / napply,
                  "algorithmic_bytes": ab[k], "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS}
    return out


def roofline_of(table: dict, w) -> dict:
    """The roofline entry of the phase with the largest device time per
    apply."""
    dom = max(table, key=lambda k: table[k]["ms"] * table[k]["per_apply"])
    t = table[dom]
    kernel = "k_" + dom if dom not in ("coarse", "finalize") else t["kernel"]
    return {"bound": "hbm", "kernel": kernel, "phase": dom, "achieved": t["GB_s"],
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": t["frac"],
            "traffic": recorded_traffic(kernel, f"{w.name}{w.nx}", w.precision),
            "traffic_unit": "bytes per launch",
            "algorithmic_bytes_per_launch": t["algorithmic_bytes"], "avg_launch_ms": t["ms"]}


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


def timed_solves(ctx, b, steps: int, warmup: int) -> dict:
    """`warmup` untimed solves, then `steps` timed ones between device
    synchronisations; per-solve latency, iterations and true residuals."""
    import torch
    p = torch.zeros_like(b)
    for _ in range(warmup):
        ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
    torch.cuda.synchronize()
    lat, its, rel = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        t1 = time.perf_counter()
        st = ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
        lat.append(time.perf_counter() - t1)
        its.append(st.iterations)
        rel.append(st.final_relres)
        if not st.converged:
            raise RuntimeError("GMRES did not converge")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return {"elapsed": elapsed, "value": steps / elapsed, "ms": 1e3 * elapsed / steps,
            "p50": float(np.percentile(lat, 50) * 1e3), "p99": float(np.percentile(lat, 99) * 1e3),
            "iterations": float(np.mean(its)), "relres_max": float(np.max(rel))}


def phase_timing(ctx, b, steps: int) -> dict:
    """The same solves again with HIP events around every phase of every
    apply, on the library's stream (eager launches; the kernels are those of
    the captured graphs of the timed region)."""
    import torch
    p = torch.zeros_like(b)
    ctx.timing(True)
    for _ in range(steps):
        ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
    torch.cuda.synchronize()
    phases = ctx.timing_read()
    ctx.timing(False)
    return phases


def workload_line(w) -> str:
    bcs = "Dirichlet left/right" if any(w.bc) else "no-flow, corner sources"
    return (f"{w.name}: {w.nx}x{w.ny} cells, subdomains of {w.s}x{w.s}, oversampling "
            f"{w.oversample}, {w.sweeps} smoothing sweep(s), overlap {w.overlap}, alpha {w.alpha}, "
            f"field {w.field}, {bcs}")


def precisions(w, K, steps: int) -> dict:
    """Solves/s of the same workload in every precision mode (setup, one
    warm-up solve, `steps` timed solves)."""
    import torch

    from paper_2606_08883_amd import binding as B
    out = {}
    for prec in (0, 1, 2):
        wp = w.with_(precision=prec)
        ctx = B.Context(wp.binding_config(), K)
        b = rhs_of(wp, ctx, K.device)
        try:
            r = timed_solves(ctx, b, steps, 1)
            out[DTYPES[prec]] = {"solves_per_s": r["value"], "iterations": r["iterations"],
                                 "relres_max": r["relres_max"]}
        except RuntimeError as e:
            out[DTYPES[prec]] = {"error": str(e)}
        ctx.close()
        torch.cuda.synchronize()
        print(f"bench: precision {prec}: {out[DTYPES[prec]]}", file=sys.stderr, flush=True)
    return out


def batched_leg(steps: int) -> dict:
    """The 1024 x 1024 log-normal workload (4096 subdomains): solves/s in
    every precision mode."""
    import torch

    from paper_2606_08883_amd import binding as B
    from paper_2606_08883_amd.configs import WORKLOADS
    w = WORKLOADS["batched"]
    dev = torch.device("cuda:0")
    K = torch.tensor(w.permeability(), dtype=torch.float64, device=dev)
    out = {"workload": workload_line(w)}
    for prec in (2, 1, 0):
        wp = w.with_(precision=prec)
        ctx = B.Context(wp.binding_config(), K)
        b = rhs_of(wp, ctx, dev)
        r = timed_solves(ctx, b, steps, 2)
        out[DTYPES[prec]] = {"solves_per_s": r["value"], "cell_dof_per_s": r["value"] * w.cells,
                             "latency_ms": {"p50": r["p50"], "p99": r["p99"]},
                             "iterations": r["iterations"]}
        ctx.close()
        print(f"bench: batched precision {prec}: {r['value']:.1f} solves/s", file=sys.stderr,
              flush=True)
    return out


def closed_loop_capacity(solver, burst, max_active: int, footprint, reps: int = 3) -> float:
    """Requests/s of a burst served closed-loop (all arrived at once): the
    median of `reps` runs, since one run moves with the host's load."""
    from paper_2606_08883_amd import serving as S
    caps = []
    for _ in range(reps):
        t0 = time.perf_counter()
        res = S.Server(solver, max_active=max_active, footprint=footprint).run(burst,
                                                                               realtime=False)
        caps.append(len(res) / (time.perf_counter() - t0))
    return float(np.median(caps))


def serving_leg(requests: int, max_active: int) -> dict:
    """A short Poisson stream of mixed-size requests (each with its own
    field and 8 right-hand sides) at 0.8 of the closed-loop capacity."""
    from paper_2606_08883_amd import serving as S
    solver = S.GpuBackend(None, keep=False)
    S.Server(solver, max_active=1).run([S.make_payload(S.Request(0, 128, 2.0, 999, 1999, 2, 0.0))],
                                       realtime=False)
    burst = [S.make_payload(r) for r in S.make_requests(max(4, requests // 2), rate=None, seed=5)]
    cap = closed_loop_capacity(solver, burst, max_active, S.footprint_of)
    rate = 0.8 * cap
    reqs = [S.make_payload(r) for r in S.make_requests(requests, rate=rate, seed=4)]
    server = S.Server(solver, max_active=max_active, footprint=S.footprint_of)
    t0 = time.perf_counter()
    res = server.run(reqs)
    wall = time.perf_counter() - t0
    sm = S.summary(res, wall)
    return {"requests": requests, "grids": sorted({r.n for r in reqs}),
            "arrival_rate_per_s": rate, "solves_per_s": sm["solves_per_s"],
            "latency_ms": sm["latency_ms"], "all_converged": sm["all_converged"],
            "setup_s_mean": sm["setup_s_mean"], "solve_s_mean": sm["solve_s_mean"],
            "peak_active": server.peak_active, "ticks": server.ticks,
            "driver": "one batched GMRES advanced in ticks (gmres_batch_tick), set-ups on "
                      "worker threads"}


def boxes3(w, grow: int) -> np.ndarray:
    """Subdomain boxes of a 3-D workload grown by `grow` cells and clipped to
    the grid, rows (x0, x1, y0, y1, z0, z1); layers of w.s cells per axis,
    the last one ragged."""
    dims = (w.nx, w.ny, w.nz)
    m = [-(-d // w.s) for d in dims]
    out = []
    for L in range(m[2]):
        for J in range(m[1]):
            for I in range(m[0]):
                b = []
                for a, q in enumerate((I, J, L)):
                    b += [max(0, q * w.s - grow), min(dims[a], (q + 1) * w.s + grow)]
                out.append(b)
    return np.array(out, dtype=np.int64)


def algorithmic_bytes3(w, coarse_bytes: float) -> dict:
    """Algorithmic bytes of one instance of every phase of the 3-D apply
    (FP64 throughout).  A box of bx x by x bz cells (plane P = bx by) stores
    bz symmetric P x P plane blocks by their P / 2 + 1 cyclic diagonals and
    bz x P couplings; the count reads them once.
      local       per subdomain on its oversampled box: factor and couplings,
                  r on the box, p written on the owned cells; per trace face
                  its two box-local cells (8 B) and four weights (32 B); per
                  interface dof its 32 B table entry and two moments (16 B);
      coarse      the interface solve: the factor matrices of its dissection
                  once per sweep and the refinement residuals (mrcm3d_query's
                  count);
      reconstruct the MBFs (N_i words per owned cell), the interface solution
                  and p read and written;
      residual    tx, ty, tz once, r and p read, rho written;
      patch       per patch: factor and couplings, rho on the patch, p read
                  and written on the owned cells;
      finalize    p read twice (zero-mean projection) and z written."""
    n = w.cells
    own = boxes3(w, 0)
    dims = (w.nx, w.ny, w.nz)

    def ext(b):
        return (b[:, 1] - b[:, 0]), (b[:, 3] - b[:, 2]), (b[:, 5] - b[:, 4])

    def factor(b):
        bx, by, bz = ext(b)
        P = bx * by
        return int(np.sum(bz * (P // 2 + 1) * P * 8 + bz * P * 8))

    ox, oy, oz = ext(own)
    cells_own = ox * oy * oz
    ob = boxes3(w, w.oversample)
    obx, oby, obz = ext(ob)
    tang = {0: (oy, oz), 1: (ox, oz), 2: (ox, oy)}
    faces, ndof = 0, np.zeros(len(own), dtype=np.int64)
    for a in range(3):
        t0, t1 = tang[a]
        nb = np.minimum(w.degree + 1, t0) * np.minimum(w.degree + 1, t1)
        for lo in (True, False):
            inner = own[:, 2 * a] > 0 if lo else own[:, 2 * a + 1] < dims[a]
            faces += int(np.sum((t0 * t1)[inner]))
            ndof += np.where(inner, nb, 0)
    nc = int(ndof.sum())
    local = factor(ob) + int(np.sum(obx * oby * obz)) * 8 + n * 8 + faces * 40 + nc * 48
    coarse = int(coarse_bytes)
    recon = int(np.sum(ndof * cells_own)) * 8 + nc * 8 + 16 * n
    faces_all = (w.nx + 1) * w.ny * w.nz + w.nx * (w.ny + 1) * w.nz + w.nx * w.ny * (w.nz + 1)
    residual = faces_all * 8 + 24 * n
    pb = boxes3(w, w.overlap)
    px, py, pz = ext(pb)
    patch = factor(pb) + int(np.sum(px * py * pz)) * 8 + 16 * n
    finalize = n * ((2 if not any(w.bc) else 1) * 8 + 8)
    return {"local": local, "coarse": coarse, "reconstruct": recon, "residual": residual,
            "patch": patch, "finalize": finalize, "nc": nc}


PHASE_KERNELS3 = {"local": "k_local3", "coarse": "interface solve (k_coarse_rhs, k_coarse_fwd "
                  "and k_coarse_bwd per level, k_coarse_resid and k_coarse_add per refinement)",
                  "reconstruct": "k_reconstruct3", "residual": "k_op3 (residual form)",
                  "patch": "k_patch3", "finalize": "k_sum + k_finalize"}


def cube_leg(steps: int) -> dict:
    """The 3-D cube workload (96^3 cells, 1728 subdomains): solves/s, phase
    table and the roofline entry of its dominant phase in FP64, and the same
    with the plane blocks stored in FP32 (precision 2)."""
    import torch

    from paper_2606_08883_amd import binding as B
    from paper_2606_08883_amd.configs import WORKLOADS3
    w0 = WORKLOADS3["cube"]
    dev = torch.device("cuda:0")
    K = torch.tensor(w0.permeability(), dtype=torch.float64, device=dev)
    b = torch.tensor(w0.rhs(), dtype=torch.float64, device=dev)
    out = None
    for prec in (0, 2):
        w = w0.with_(precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx = B.Context3(w.binding_config(), K)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        r = timed_solves(ctx, b, steps, 2)
        phases = phase_timing(ctx, b, max(1, min(steps, 5)))
        ab = algorithmic_bytes3(w, ctx.query("coarse_bytes"))
        napply = max(1, phases["local"][1])
        table = {}
        for k, (ms, cnt) in phases.items():
            if cnt == 0:
                continue
            avg = ms / cnt
            gbs = ab[k] / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
            table[k] = {"kernel": PHASE_KERNELS3[k], "ms": avg, "per_apply": cnt / napply,
                        "algorithmic_bytes": ab[k], "GB_s": gbs, "frac": gbs / HBM_PEAK_GBS}
        assert int(ctx.query("coarse_dofs")) == ab["nc"]
        refine, levels = int(ctx.query("coarse_refine")), int(ctx.query("coarse_levels"))
        res = {"solves_per_s": r["value"], "cell_dof_per_s": r["value"] * w.cells,
               "latency_ms": {"p50": r["p50"], "p99": r["p99"]}, "iterations": r["iterations"],
               "final_relres_max": r["relres_max"], "setup_s": setup_s,
               "device_gb": ctx.query("device_bytes") / 1e9,
               "apply_ms": sum(v[0] for v in phases.values()) / napply, "phases": table}
        ctx.close()
        if prec == 0:
            dom = max(table, key=lambda k: table[k]["ms"] * table[k]["per_apply"])
            t = table[dom]
            out = {"workload": f"{w.name}: {w.nx}x{w.ny}x{w.nz} cells, subdomains of {w.s}^3, "
                               f"oversampling {w.oversample}, degree {w.degree}, {w.sweeps} "
                               f"smoothing sweep(s), overlap {w.overlap}, alpha {w.alpha}, "
                               f"log-normal sigma {w.sigma} correlation {w.ell}, no-flow, "
                               "corner sources",
                   "dtype": "f64", "interface_dofs": ab["nc"],
                   "interface_refinement_steps": refine, "interface_levels_per_sweep": levels,
                   **res,
                   "roofline": {"bound": "hbm", "kernel": t["kernel"], "phase": dom,
                                "achieved": t["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": t["frac"],
                                "algorithmic_bytes_per_launch": t["algorithmic_bytes"],
                                "avg_launch_ms": t["ms"]}}
        else:
            out["f32-storage/f64-arith"] = res
    return out


def cpu_baseline(w, gpu_iterations: float, window: int = 512) -> dict:
    """The oracle as it stands, on the host cores, on a bounded sample of the
    workload: the bottom-left window x window cells of the same field with
    the same method parameters and boundary set-up, solved whole (setup,
    then GMRES to 1e-8), once on one core and then as independent copies on
    every core the box gives this run (at most 16).  The solve time per
    GMRES step scales with the cell count (one box solve per subdomain and
    sweep), so the estimate for the workload is the sample's time per step
    times the cell ratio times the GPU's iterations per solve."""
    code = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, %r)
from oracle.discretization import direct_solve, rhs
from oracle.gmres import gmres
from oracle.mrcm import MRCM
from paper_2606_08883_amd.configs import WORKLOADS
w0 = WORKLOADS[%r]
n = %d
w = w0.with_(nx=n, ny=n)
K = w0.permeability().reshape(w0.ny, w0.nx)[:n, :n].ravel().copy()
t0 = time.perf_counter()
mr = MRCM(K, **w.oracle_args())
t_setup = time.perf_counter() - t0
if any(w.bc):
    f, g = w.boundary_data()
    b = rhs(K, n, n, w.bc, f, {0: g[:n], 1: g[n:2 * n]}, 1.0 / n)
else:
    b = w.rhs()
t0 = time.perf_counter()
res = gmres(lambda x: mr.A @ x, mr.apply, b, rtol=1e-8, restart=10, maxit=300)
t_solve = time.perf_counter() - t0
t0 = time.perf_counter()
direct_solve(mr.A, b, w.bc)
t_splu = time.perf_counter() - t0
print(json.dumps({"setup_s": t_setup, "solve_s": t_solve, "its": res.iterations,
                  "converged": res.converged, "splu_s": t_splu}))
""" % (ROOT, w.name, window)
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        env[k] = "1"

    def run(copies: int) -> list:
        procs = [subprocess.Popen([sys.executable, "-c", code], stdout=subprocess.PIPE,
                                  stderr=subprocess.PIPE, text=True, env=env)
                 for _ in range(copies)]
        out = []
        for pr in procs:
            so, se = pr.communicate(timeout=900)
            if pr.returncode != 0:
                raise RuntimeError(se[-2000:])
            out.append(json.loads(so.strip().splitlines()[-1]))
        return out

    one = run(1)[0]
    cores = max(1, min(os.cpu_count() or 1, 16))
    t0 = time.perf_counter()
    many = run(cores)
    wall = time.perf_counter() - t0
    scale = (w.nx * w.ny) / float(window * window)
    step_1 = one["solve_s"] / one["its"]
    solve_est_1 = step_1 * scale * gpu_iterations
    # all cores: the copies solve at once; their combined steps per second,
    # scaled the same way
    step_rate_all = sum(m["its"] / m["solve_s"] for m in many)
    solve_est_all = scale * gpu_iterations / step_rate_all
    try:
        model = [ln.split(":", 1)[1].strip() for ln in
                 subprocess.run(["lscpu"], capture_output=True, text=True).stdout.splitlines()
                 if ln.startswith("Model name")][0]
    except Exception:
        model = platform.processor() or "unknown"
    return {"value": 1.0 / solve_est_all, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "single_core_solves_per_s": 1.0 / solve_est_1,
            "splu_window_s": one["splu_s"],
            "splu_note": (f"scipy splu (SuperLU, COLAMD ordering) direct solve of the same "
                          f"{window}x{window} window on one core, for reference: "
                          f"{one['splu_s']:.2f} s; its fill grows faster than the cell count, "
                          f"so it is not scaled to the workload"),
            "cpu_model": model, "nproc": os.cpu_count(),
            "sample": (f"the oracle (NumPy/SciPy FP64, one thread per process) on the "
                       f"{window}x{window} bottom-left window of the same field and method "
                       f"parameters, solved whole: setup {one['setup_s']:.1f} s, GMRES "
                       f"{one['its']} steps in {one['solve_s']:.1f} s on one core; {cores} "
                       f"independent copies at once took {wall:.1f} s wall.  Solve time of the "
                       f"workload = time per step x cell ratio ({scale:.0f}) x the GPU's "
                       f"{gpu_iterations:.1f} steps per solve; value = all {cores} cores")}


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
    table = phase_table(w, maps, ctx, phases)
    out = {"metric": "MRCM-OS preconditioner applications/s", "value": args.steps / elapsed,
           "unit": "applies/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
           "dtype": DTYPES[w.precision], "data": "synthetic",
           "config": {"workload": workload_line(w), "cells": w.cells,
                      "subdomains": int(maps["boxes"].shape[0])},
           "setup_s": setup_s, "device_gb": ctx.query("device_bytes") / 1e9,
           "roofline": roofline_of(table, w), "phases": table}
    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


def serve(args) -> int:
    """Serving run: capacity from closed-loop bursts (median of three), then a Poisson stream at
    0.8 of it; request latency from arrival to answer (setup included)."""
    from paper_2606_08883_amd import serving as S

    params = None if args.precision is None else dict(precision=args.precision)
    prec = S.SERVE_PARAMS["precision"] if args.precision is None else args.precision
    fp = (lambda r: S.footprint_of(r, params))
    B = S.GpuBackend(params, keep=False)
    warm = S.make_payload(S.Request(0, 128, 2.0, 999, 1999, 2, 0.0))
    S.Server(B, max_active=1).run([warm], realtime=False)
    burst = [S.make_payload(r) for r in S.make_requests(max(4, args.requests // 2), rate=None,
                                                          seed=5)]
    print(f"bench: serving burst of {len(burst)} requests", file=sys.stderr, flush=True)
    cap = closed_loop_capacity(B, burst, args.max_active, fp)
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
    out = {"metric": METRIC, "value": sm["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": len(reqs), "warmup": 1, "ms_per_step": 1e3 * wall / len(reqs),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": DTYPES[prec], "data": "synthetic",
           "config": {"workload": f"serving: {len(reqs)} requests, grids {sizes} (uniform), "
                                  f"log-normal sigma U[1,3] corr. 16, 8 injector/producer "
                                  f"pairs each, Poisson arrivals at 0.8 x closed-loop capacity "
                                  f"({rate:.2f}/s), {args.max_active} slots",
                      "parallelism": "single GPU, the right-hand sides of all requests in "
                                     "flight advanced together in ticks of one batched GMRES"},
           "cell_dof_per_s": sm["cell_dof_per_s"], "latency_ms": sm["latency_ms"],
           "requests_per_s": sm["requests_per_s"], "capacity_requests_per_s": cap,
           "setup_s_mean": sm["setup_s_mean"], "solve_s_mean": sm["solve_s_mean"],
           "iterations_per_solve": sm["iterations_mean"], "peak_active": server.peak_active,
           "ticks": server.ticks,
           "peak_footprint_gb": server.peak_bytes / 1e9}
    print(json.dumps(out), flush=True)
    return 0


def mfma_ab(args) -> int:
    """8-column applications of T with the reconstruction on the vector FMA
    kernel (the default) and on the matrix cores (MRCM_MFMA_RECON=mfma, and
    bf16 in FP32 mode): apply time and reconstruct phase time per variant,
    1024^2 cells, subdomains of 16^2, log-normal sigma 2."""
    import os

    import torch

    from paper_2606_08883_amd import binding as B
    from paper_2606_08883_amd import workloads as wl
    dev = torch.device("cuda", 0)
    n, sub = 1024, 16
    K = torch.tensor(wl.lognormal_K(n, n, 2.0, 16.0, 5), dtype=torch.float64, device=dev)
    R = torch.tensor(np.stack([wl.random_vector(n * n, 10 + k, zero_mean=True) for k in range(8)]),
                     dtype=torch.float64, device=dev).contiguous()
    out = {}
    for prec in (2, 1, 0):
        for mode in ([None, "mfma", "bf16"] if prec == 1 else [None, "mfma"]):
            if mode:
                os.environ["MRCM_MFMA_RECON"] = mode
            else:
                os.environ.pop("MRCM_MFMA_RECON", None)
            ctx = B.Context(B.Config(n, n, (0, 0, 0, 0), sub, sub, 4, 10.0, 0, 1, 2, 1, prec), K)
            Z = torch.empty_like(R)
            for _ in range(args.warmup):
                ctx.apply(R, Z)
            torch.cuda.synchronize()
            ctx.timing(True)
            for _ in range(args.steps):
                ctx.apply(R, Z)
            torch.cuda.synchronize()
            ph = ctx.timing_read()
            ctx.timing(False)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ctx.apply(R, Z)
            torch.cuda.synchronize()
            key = f"{DTYPES[prec]} {mode or 'fma'}"
            out[key] = {"apply_ms": 1e3 * (time.perf_counter() - t0) / args.steps,
                        "reconstruct_ms": ph["reconstruct"][0] / max(1, ph["reconstruct"][1]),
                        "mfma_recon": ctx.query("mfma_recon")}
            print(f"bench: {key}: {out[key]}", file=sys.stderr, flush=True)
            ctx.close()
    os.environ.pop("MRCM_MFMA_RECON", None)
    print(json.dumps({"metric": "8-column applications of T, reconstruction FMA vs MFMA",
                      "config": {"workload": "1024x1024 cells, subdomains of 16x16, oversampling "
                                             "4, one sweep, log-normal sigma 2, 8 columns"},
                      "variants": out}), flush=True)
    return 0


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
        for s in (40, 20):
            for name, l, k in INCLUSION_ROWS:
                w = w0.with_(s=s, oversample=l, sweeps=k)
                print(f"bench: inclusions {kind} {160 // s}x{160 // s} {name}", file=sys.stderr,
                      flush=True)
                ctx = B.Context(w.binding_config(), K)
                b = rhs_of(w, ctx, dev)
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
    ap.add_argument("--workload", default="large",
                    choices=["small", "channel", "batched", "large"])
    ap.add_argument("--precision", type=int, default=None,
                    help="0 FP64 apply, 1 FP32 apply, 2 FP32-stored factors with FP64 arithmetic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the precision comparison, the 1024^2 workload and the serving leg")
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
    ap.add_argument("--cube", action="store_true",
                    help="only the 3-D cube workload (96^3 cells): one JSON line")
    ap.add_argument("--mfma-ab", action="store_true",
                    help="time 8-column applications with the reconstruction on the FMA kernel "
                         "and on the matrix cores")
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
    if args.mfma_ab:
        return mfma_ab(args)
    if args.cube:
        print(json.dumps(cube_leg(args.steps)), flush=True)
        return 0
    if args.inclusions:
        return inclusions(args)

    from paper_2606_08883_amd import binding as B
    from paper_2606_08883_amd.configs import WORKLOADS

    w = WORKLOADS[args.workload]
    if args.precision is not None:
        w = w.with_(precision=args.precision)
    dev = torch.device("cuda:0")
    print(f"bench: workload {w.name} {w.nx}x{w.ny} precision {w.precision}: field",
          file=sys.stderr, flush=True)
    K = torch.tensor(w.permeability(), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx = B.Context(w.binding_config(), K)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"bench: setup {setup_s:.2f} s", file=sys.stderr, flush=True)
    b = rhs_of(w, ctx, dev)
    if args.apply_only:
        return apply_only(args, w, ctx, b, setup_s)
    r = timed_solves(ctx, b, args.steps, args.warmup)
    print(f"bench: {r['value']:.2f} solves/s, {r['iterations']:.1f} iterations", file=sys.stderr,
          flush=True)
    phases = phase_timing(ctx, b, max(1, min(args.steps, 5)))
    maps = B.maps(w.binding_config())
    table = phase_table(w, maps, ctx, phases)
    apply_ms = sum(v[0] for v in phases.values()) / max(1, phases["local"][1])
    out = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[w.precision],
        "data": "synthetic",
        "config": {"workload": workload_line(w), "cells": w.cells,
                   "precision": PRECISION_NAMES[w.precision], "rtol": 1e-8, "restart": 10,
                   "parallelism": "single GPU"},
        "cell_dof_per_s": r["value"] * w.cells,
        "latency_ms": {"p50": r["p50"], "p99": r["p99"]},
        "iterations_per_solve": r["iterations"],
        "final_relres_max": r["relres_max"],
        "setup_s": setup_s,
        "setup_stages_s": {"host_preparation": ctx.query("setup_host_s"),
                           "device": ctx.query("setup_device_s"),
                           "interface": ctx.query("setup_coarse_s")},
        "solves_per_s_incl_setup": 1.0 / (setup_s + r["elapsed"] / args.steps),
        "device_gb": ctx.query("device_bytes") / 1e9,
        "interface_refinement_steps": ctx.query("coarse_refine"),
        "apply_ms": apply_ms,
        "roofline": roofline_of(table, w),
        "phases": table,
    }
    ctx.close()
    torch.cuda.synchronize()
    if not args.no_extras:
        print("bench: precision modes", file=sys.stderr, flush=True)
        out["precisions"] = precisions(w, K, max(2, args.steps // 4))
        del K
        torch.cuda.empty_cache()
        print("bench: 1024^2 workload", file=sys.stderr, flush=True)
        out["batched_1024"] = batched_leg(max(5, args.steps // 2))
        print("bench: serving leg", file=sys.stderr, flush=True)
        out["serving"] = serving_leg(32, 8)
        print("bench: 3-D cube workload", file=sys.stderr, flush=True)
        out["cube_3d"] = cube_leg(max(5, args.steps // 2))
    if not args.no_cpu_baseline:
        print("bench: timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, r["iterations"])
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
