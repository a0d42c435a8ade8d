"""Request loop for pressure solves of mixed grid sizes (continuous batching).

A request is one pressure problem: a square grid, its own log-normal
permeability field and nrhs right-hand sides (injector/producer pairs).  Its
answer is the nrhs pressure fields, each solved by right-preconditioned
GMRES(10) with MRCM-OS to the relative tolerance.

Requests arrive over time.  The server admits an arrived request as soon as
one of its slots is free and the request's device footprint (mrcm_footprint:
factorisations, basis functions, interface factor, Krylov spaces of its
right-hand sides) fits under the memory budget beside the requests in flight.
An admitted request is set up by a worker thread on its own stream (its
factorisations stay resident in device memory while it is in flight); when
its set-up ends, its right-hand sides join the batched GMRES that the serving
thread advances in ticks: every tick runs one Arnoldi step of every right-hand
side in flight, of every request, with one launch per phase of T over all of
them (gmres_batch_tick).  A request's slot and memory are released when its
answer is complete, and the next arrived request takes them.  Every kernel's
arithmetic and reduction order is fixed per right-hand side, so each answer
is bit-identical to the same request solved alone (and to gmres_solve).

The scheduling is host logic and takes the backend as an argument (the tests
drive it with stand-ins on the CPU); `GpuBackend` is the library's.
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




def footprint_of(req: Request, params: dict | None = None) -> int:
    from .binding import footprint
    return footprint(config_for(req.n, params), req.nrhs)


def host_cores() -> int:
    """Cores this process may use: OMP_NUM_THREADS when set, else all."""
    import os
    try:
        return max(1, int(os.environ.get("OMP_NUM_THREADS", "")))
    except ValueError:
        return max(1, os.cpu_count() or 1)


class GpuBackend:
    """The library behind the server: a request is set up on its own stream
    by a worker thread (its factorisations stay resident while it is in
    flight), then its right-hand sides join one batched GMRES (gmres_batch_*)
    that the server ticks; its answer is copied to the host when all of them
    have finished, and its context is released on a background thread (a
    release frees device memory, which can wait for the device; on the
    serving thread it held up the ticks).  flush() waits for the releases.

    setup_threads: host threads of each set-up; None (the default) divides
    the host cores among the set-ups in progress when a set-up starts (all
    of them when it runs alone); 0 = all cores always."""

    def __init__(self, params: dict | None = None, rtol: float = 1e-8, restart: int = 10,
                 maxit: int = 500, keep: bool = True, device: int = 0,
                 setup_threads: int | None = None):
        self.params, self.rtol, self.restart, self.maxit = params, rtol, restart, maxit
        self.keep, self.device, self.setup_threads = keep, device, setup_threads
        self.cores = host_cores()
        self.lock = threading.Lock()
        self.setups = 0
        self.batch = None
        self.releaser = ThreadPoolExecutor(max_workers=1)
        self.releases = []

    def setup(self, req: Request) -> dict:
        import torch

        from .binding import Context, set_host_threads
        with self.lock:
            self.setups += 1
            share = max(1, self.cores // self.setups)
        set_host_threads(share if self.setup_threads is None else self.setup_threads)
        try:
            dev = torch.device("cuda", self.device)
            stream = torch.cuda.Stream(device=dev)
            with torch.cuda.stream(stream):
                K = torch.tensor(req.K, dtype=torch.float64, device=dev)
                B = torch.tensor(req.B, dtype=torch.float64, device=dev).contiguous()
                t0 = time.perf_counter()
                ctx = Context(config_for(req.n, self.params), K, stream=stream)
                P = torch.zeros_like(B)
                stream.synchronize()
                t1 = time.perf_counter()
        finally:
            with self.lock:
                self.setups -= 1
        return dict(ctx=ctx, B=B, P=P, K=K, stream=stream, setup_s=t1 - t0)

    def add(self, h: dict) -> None:
        from .binding import Batch
        if self.batch is None:
            self.batch = Batch(self.restart)
        h["tag"] = self.batch.add(h["ctx"], h["B"], h["P"], rtol=self.rtol, maxit=self.maxit,
                                  stream=h["stream"])
        h["t_add"] = time.perf_counter()

    def tick(self) -> int:
        return self.batch.tick() if self.batch is not None else 0

    def poll(self, h: dict):
        st = self.batch.poll(h["tag"])
        if st is None:
            return None
        t2 = time.perf_counter()
        self.batch.remove(h["tag"])  # returns once the batch's device work has ended
        p = h["P"].cpu().numpy() if self.keep else None
        self.releases.append(self.releaser.submit(h["ctx"].close))
        return dict(iterations=st.iterations, converged=st.converged,
                    final_relres=st.final_relres, setup_s=h["setup_s"],
                    solve_s=t2 - h["t_add"], p=p)

    def flush(self) -> None:
        """Wait until every finished request's context is released (re-raises
        a failed release)."""
        done, self.releases = self.releases, []
        for f in done:
            f.result()


class Server:
    """Admission and continuous batching of requests (see the module text).

    backend: setup(req) -> handle, run on worker threads; add(handle),
    tick() -> right-hand sides still running, poll(handle) -> None or a dict
    of Result fields (the request is then finished and its release begun),
    run on the serving thread; optionally flush(), called at the end of
    run(), which waits for the releases.  A finished request's footprint
    counts as free from the moment poll() returns its answer.  max_active:
    requests in flight at once (set up or solving); mem_budget: bytes their
    footprints may total; footprint(req) -> bytes; setup_workers: set-ups in
    progress at once."""

    def __init__(self, backend, max_active: int = 8, mem_budget: int = 200 << 30,
                 footprint=footprint_of, setup_workers: int = 4):
        if max_active < 1:
            raise ValueError("max_active must be at least 1")
        self.backend = backend
        self.max_active = max_active
        self.mem_budget = mem_budget
        self.footprint = footprint
        self.setup_workers = max(1, setup_workers)
        self.peak_active = 0
        self.peak_bytes = 0
        self.ticks = 0
        self.events = []   # (time, "admit" | "done", rid), in order

    def run(self, requests, realtime: bool = True) -> list:
        """Serve the requests (arrival times relative to the call); returns
        their Results in request order.  With realtime False every request
        counts as arrived at once (closed loop)."""
        reqs = sorted(requests, key=lambda r: (r.arrival if realtime else 0.0, r.rid))
        for r in reqs:
            if self.footprint(r) > self.mem_budget:
                raise ValueError(f"request {r.rid} needs more memory than the whole budget")
        results = {}
        start = time.perf_counter()
        clock = lambda: time.perf_counter() - start  # noqa: E731
        pending = list(reqs)
        setting_up = {}   # future -> (request, bytes, admitted)
        solving = []      # (request, bytes, admitted, handle)
        used = 0
        with ThreadPoolExecutor(max_workers=self.setup_workers) as pool:
            while pending or setting_up or solving:
                now = clock()
                # admit, in arrival order, what has arrived and fits
                while pending:
                    r = pending[0]
                    arrived = (r.arrival <= now) if realtime else True
                    need = self.footprint(r)
                    inflight = len(setting_up) + len(solving)
                    if not arrived or inflight >= self.max_active or used + need > self.mem_budget:
                        break
                    pending.pop(0)
                    used += need
                    t_adm = clock()
                    self.events.append((t_adm, "admit", r.rid))
                    setting_up[pool.submit(self.backend.setup, r)] = (r, need, t_adm)
                    self.peak_active = max(self.peak_active, len(setting_up) + len(solving))
                    self.peak_bytes = max(self.peak_bytes, used)
                # requests whose set-up ended join the batch
                for f in [f for f in setting_up if f.done()]:
                    r, need, t_adm = setting_up.pop(f)
                    h = f.result()  # re-raise a failed set-up here
                    self.backend.add(h)
                    solving.append((r, need, t_adm, h))
                if solving:
                    self.backend.tick()
                    self.ticks += 1
                    still = []
                    for r, need, t_adm, h in solving:
                        out = self.backend.poll(h)
                        if out is None:
                            still.append((r, need, t_adm, h))
                            continue
                        t_done = clock()
                        used -= need
                        self.events.append((t_done, "done", r.rid))
                        results[r.rid] = Result(r.rid, r.n, r.nrhs, r.arrival, t_adm, t_done,
                                                footprint=need, **out)
                    solving = still
                    continue
                # nothing to tick: wait for a set-up or the next arrival
                timeout = None
                if pending and realtime and pending[0].arrival > clock():
                    timeout = pending[0].arrival - clock()
                if setting_up:
                    wait(list(setting_up), timeout=timeout, return_when=FIRST_COMPLETED)
                elif timeout is not None:
                    time.sleep(timeout)
        flush = getattr(self.backend, "flush", None)
        if flush is not None:
            flush()
        return [results[r.rid] for r in sorted(requests, key=lambda r: r.rid)]


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
