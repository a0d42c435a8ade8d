"""Request loop for pressure solves of mixed grid sizes (continuous batching).

A request is one pressure problem: a square grid, its own log-normal
permeability field and nrhs right-hand sides (injector/producer pairs).  Its
answer is the nrhs pressure fields, each solved by right-preconditioned
GMRES(10) with MRCM-OS to the relative tolerance.

Requests arrive over time.  The server admits an arrived request as soon as
one of its slots is free and the request's device footprint (mrcm_footprint:
factorisations, basis functions, interface factor, Krylov space of its right-
hand sides) fits under the memory budget beside the requests in flight.  An
admitted request is set up on its own stream (its factorisations stay
resident in device memory while it is in flight) and solved while the others
are in flight, so their kernels overlap on the device; its slot and memory are
released when its answer is complete, and the next arrived request takes
them.  Nothing is shared between requests and every kernel's arithmetic and
reduction order is fixed, so each answer is bit-identical to the same request
solved alone.

The scheduling is host logic and takes the solve function as an argument (the
tests drive it with stand-ins on the CPU); `gpu_solver` is the solve function
of the library.
"""
from __future__ import annotations

import threading
import time
from concurrent.futures import FIRST_COMPLETED, ThreadPoolExecutor, wait
from dataclasses import dataclass, field

import numpy as np

from . import workloads as wl

# Method parameters of a served request: subdomains of 16 x 16 cells,
# oversampling 4, one smoothing sweep with overlap 2, alpha 10 with L = H,
# interface degree 1, factors stored in FP32 and applied in FP64.
SERVE_PARAMS = dict(s=16, oversample=4, alpha=10.0, beta_len=0, sweeps=1, overlap=2, degree=1,
                    precision=2)


@dataclass
class Request:
    rid: int
    n: int                 # grid of n x n cells, no-flow on every side
    sigma: float           # log-normal K: ln K = sigma * Gaussian field (correlation 16)
    field_seed: int
    rhs_seed: int
    nrhs: int
    arrival: float         # seconds after the start of the run
    K: np.ndarray | None = None   # host payload, filled by make_payload
    B: np.ndarray | None = None   # (nrhs, n * n)


@dataclass
class Result:
    rid: int
    n: int
    nrhs: int
    arrival: float
    admitted: float
    done: float
    iterations: int = 0
    converged: bool = False
    final_relres: float = 0.0
    setup_s: float = 0.0
    solve_s: float = 0.0
    footprint: int = 0
    p: np.ndarray | None = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def make_requests(count: int, sizes=(128, 256, 512, 1024), rate: float | None = None,
                  nrhs: int = 8, seed: int = 4) -> list:
    """Seeded request stream: sizes drawn uniformly from `sizes`, sigma ~
    U[1, 3], field seed 1000 + i, right-hand-side seed 2000 + i, Poisson
    arrivals at `rate` per second (all at time 0 when rate is None)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for i in range(count):
        if rate is not None:
            t += rng.exponential(1.0 / rate)
        n = int(rng.choice(sizes))
        sigma = float(rng.uniform(1.0, 3.0))
        out.append(Request(i, n, sigma, 1000 + i, 2000 + i, nrhs, t if rate else 0.0))
    return out


def make_payload(req: Request) -> Request:
    """The request's data as a client sends it: K and the right-hand sides."""
    req.K = wl.lognormal_K(req.n, req.n, req.sigma, 16.0, req.field_seed)
    req.B = wl.random_pairs(req.n, req.n, req.nrhs, req.rhs_seed)
    return req


def config_for(n: int, params: dict | None = None):
    from .binding import Config
    p = dict(SERVE_PARAMS, **(params or {}))
    return Config(n, n, (0, 0, 0, 0), p["s"], p["s"], p["oversample"], p["alpha"], p["beta_len"],
                  p["sweeps"], p["overlap"], p["degree"], p["precision"])


LANES, WIDTH = 4, 4  # lanes and right-hand sides per lane of a request (mrcm_set_lanes/_batch)


def footprint_of(req: Request, params: dict | None = None) -> int:
    from .binding import footprint
    return footprint(config_for(req.n, params), min(req.nrhs, LANES * WIDTH))


def host_cores() -> int:
    """Cores this process may use: OMP_NUM_THREADS when set, else all."""
    import os
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return max(1, os.cpu_count() or 1)


def gpu_solver(params: dict | None = None, rtol: float = 1e-8, restart: int = 10,
               maxit: int = 500, keep: bool = True, device: int = 0,
               setup_threads: int | None = None):
    """Solve function of the library: set up the request's context on its
    own stream, solve its right-hand sides, copy the answer to the host and
    release everything.  setup_threads: host threads of each set-up; None
    (the default) divides the host cores among the set-ups in progress when
    a set-up starts (all of them when it runs alone); 0 = all cores always."""
    import torch

    from .binding import Context, set_host_threads

    cores = host_cores()
    lock = threading.Lock()
    setups = [0]  # set-ups in progress

    def solve(req: Request) -> dict:
        with lock:
            setups[0] += 1
            share = max(1, cores // setups[0])
        set_host_threads(share if setup_threads is None else setup_threads)
        in_setup = True
        try:
            dev = torch.device("cuda", device)
            stream = torch.cuda.Stream(device=dev)
            with torch.cuda.stream(stream):
                K = torch.tensor(req.K, dtype=torch.float64, device=dev)
                B = torch.tensor(req.B, dtype=torch.float64, device=dev).contiguous()
                t0 = time.perf_counter()
                ctx = Context(config_for(req.n, params), K, stream=stream)
                ctx.set_lanes(LANES)
                ctx.set_batch(WIDTH)
                stream.synchronize()
                t1 = time.perf_counter()
                with lock:
                    setups[0] -= 1
                in_setup = False
                P = torch.zeros_like(B)
                st = ctx.gmres(B, P, rtol=rtol, restart=restart, maxit=maxit, stream=stream,
                               raise_on_noconv=False)
                stream.synchronize()
                t2 = time.perf_counter()
                p = P.cpu().numpy() if keep else None
                ctx.close()
        finally:
            if in_setup:
                with lock:
                    setups[0] -= 1
        return dict(iterations=st.iterations, converged=st.converged,
                    final_relres=st.final_relres, setup_s=t1 - t0, solve_s=t2 - t1, p=p)

    return solve


class Server:
    """Admission and continuous batching of requests (see the module text).

    max_active: requests in flight at once; mem_budget: bytes their
    footprints may total; footprint(req) -> bytes; solve(req) -> dict of
    Result fields."""

    def __init__(self, solve, max_active: int = 8, mem_budget: int = 200 << 30,
                 footprint=footprint_of):
        if max_active < 1:
            raise ValueError("max_active must be at least 1")
        self.solve = solve
        self.max_active = max_active
        self.mem_budget = mem_budget
        self.footprint = footprint
        self.peak_active = 0
        self.peak_bytes = 0
        self.events = []   # (time, "admit" | "done", rid), in order

    def run(self, requests, realtime: bool = True) -> list:
        """Serve the requests (arrival times relative to the call); returns
        their Results in request order.  With realtime False every request
        counts as arrived at once (closed loop)."""
        reqs = sorted(requests, key=lambda r: (r.arrival if realtime else 0.0, r.rid))
        for r in reqs:
            if self.footprint(r) > self.mem_budget:
                raise ValueError(f"request {r.rid} needs more memory than the whole budget")
        lock = threading.Lock()
        results = {}
        start = time.perf_counter()
        clock = lambda: time.perf_counter() - start  # noqa: E731
        pending = list(reqs)
        inflight = {}  # future -> (request, bytes)
        used = 0
        with ThreadPoolExecutor(max_workers=self.max_active) as pool:
            while pending or inflight:
                now = clock()
                # admit, in arrival order, what has arrived and fits
                while pending:
                    r = pending[0]
                    arrived = (r.arrival <= now) if realtime else True
                    need = self.footprint(r)
                    if not arrived or len(inflight) >= self.max_active or used + need > self.mem_budget:
                        break
                    pending.pop(0)
                    used += need
                    t_adm = clock()
                    with lock:
                        self.events.append((t_adm, "admit", r.rid))
                    fut = pool.submit(self._serve_one, r, t_adm, clock, results, lock)
                    inflight[fut] = (r, need)
                    self.peak_active = max(self.peak_active, len(inflight))
                    self.peak_bytes = max(self.peak_bytes, used)
                if not inflight:
                    # nothing running: sleep until the next arrival
                    time.sleep(max(0.0, pending[0].arrival - clock()) if realtime else 0.0)
                    continue
                timeout = None
                if pending and realtime and pending[0].arrival > clock():
                    timeout = pending[0].arrival - clock()
                done, _ = wait(list(inflight), timeout=timeout, return_when=FIRST_COMPLETED)
                for f in done:
                    r, need = inflight.pop(f)
                    used -= need
                    f.result()  # re-raise a failed solve here
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]

    def _serve_one(self, r: Request, t_adm: float, clock, results: dict, lock):
        out = self.solve(r)
        t_done = clock()
        res = Result(r.rid, r.n, r.nrhs, r.arrival, t_adm, t_done, footprint=self.footprint(r),
                     **out)
        with lock:
            self.events.append((t_done, "done", r.rid))
            results[r.rid] = res
        return res


def summary(results, wall: float) -> dict:
    """Throughput and latency of a finished run."""
    lat = np.array([r.latency for r in results])
    solves = sum(r.nrhs for r in results)
    return {"requests": len(results), "solves": solves, "wall_s": wall,
            "solves_per_s": solves / wall, "requests_per_s": len(results) / wall,
            "cell_dof_per_s": sum(r.nrhs * r.n * r.n for r in results) / wall,
            "latency_ms": {"p50": float(np.percentile(lat, 50) * 1e3),
                           "p99": float(np.percentile(lat, 99) * 1e3)},
            "setup_s_mean": float(np.mean([r.setup_s for r in results])),
            "solve_s_mean": float(np.mean([r.solve_s for r in results])),
            "all_converged": all(r.converged for r in results),
            "iterations_mean": float(np.mean([r.iterations / max(1, r.nrhs) for r in results]))}
