"""GPU tests of the serving path and of the batch and allocator entry points.

* Requests of mixed grid sizes served together (their right-hand sides in
  one batched GMRES, advanced in shared ticks) give answers bit-identical to
  the same requests served one at a time, and every answer meets the
  tolerance on the true residual.
* A served request in FP64 (precision 0) matches the oracle's GMRES solution
  (iterations within +-1, solution within the FP64 gate); served 512^2 and
  1024^2 requests in the serving mode (FP32 factor storage, FP64 arithmetic)
  equal gmres_solve bit for bit, the 512^2 one also matches the oracle's
  iterations (+-1 per right-hand side) and, driven to 1e-10, the direct
  solve within 1e-7; the 1024^2 answers meet the tolerance on the oracle's
  own A.
* mrcm_apply_many over contexts of several sizes, boundary types and
  precision modes (one launch per phase over all their columns) equals
  mrcm_apply on each, bit for bit.
* The batched GMRES (gmres_batch_*) over contexts of several families, with
  right-hand sides joining while others run, equals gmres_solve bit for bit.
* Contexts set up with a caller allocator (torch's caching allocator through
  mrcm_set_allocator) allocate through it and compute the same T r.
* gmres_solve advancing several right-hand sides at once (lanes, and
  several slots per lane sharing multi-column applications of T) gives the
  solutions and iteration counts of one lane, bit for bit, and of each
  right-hand side solved on its own.
* In a fresh process whose first library call is a host-only one made
  before torch is imported, a request served from a worker thread still
  sets up and converges (the binding loads torch's runtimes first).
"""
import numpy as np
import pytest

from oracle.discretization import assemble, direct_solve
from oracle.gmres import gmres
from oracle.mrcm import MRCM
from paper_2606_08883_amd import binding as B
from paper_2606_08883_amd import serving as S
from paper_2606_08883_amd import workloads as wl
from tests._gates import t_gate

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    B.lib()
    return torch.device("cuda:0")


def _requests():
    reqs = [S.Request(0, 128, 1.5, 1000, 2000, 3, 0.0), S.Request(1, 256, 2.5, 1001, 2001, 3, 0.0),
            S.Request(2, 128, 3.0, 1002, 2002, 3, 0.0), S.Request(3, 256, 1.0, 1003, 2003, 3, 0.0)]
    return [S.make_payload(r) for r in reqs]


def test_mix_equals_alone(dev):
    print("serving: 4 requests alone, then together", flush=True)
    reqs = _requests()
    alone = S.Server(S.GpuBackend(), max_active=1).run(reqs, realtime=False)
    mix_server = S.Server(S.GpuBackend(), max_active=4)
    mix = mix_server.run(reqs, realtime=False)
    assert mix_server.peak_active >= 2
    for a, m, r in zip(alone, mix, reqs):
        A = assemble(r.K, r.n, r.n, (0, 0, 0, 0))
        rel = [np.linalg.norm(r.B[k] - A @ m.p[k]) / np.linalg.norm(r.B[k]) for k in range(r.nrhs)]
        print(f"  request {r.rid} ({r.n}^2): its {m.iterations}, max relres {max(rel):.2e}, "
              f"identical {np.array_equal(a.p, m.p)}", flush=True)
        assert m.converged and a.converged
        assert a.iterations == m.iterations
        assert np.array_equal(a.p, m.p)
        assert max(rel) <= 1e-8 * (1 + 1e-6)


def test_served_request_matches_oracle(dev):
    r = S.make_payload(S.Request(0, 128, 2.0, 1000, 2000, 2, 0.0))
    params = dict(precision=0)
    res = S.Server(S.GpuBackend(params), max_active=1).run([r], realtime=False)[0]
    p = dict(S.SERVE_PARAMS, **params)
    mr = MRCM(r.K, nx=r.n, ny=r.n, bc=(0, 0, 0, 0), sx=p["s"], sy=p["s"],
              oversample=p["oversample"], alpha=p["alpha"],
              beta_len="h" if p["beta_len"] else "H", sweeps=p["sweeps"], overlap=p["overlap"],
              degree=p["degree"])
    gate = t_gate(mr)
    its = 0
    for k in range(r.nrhs):
        ref = gmres(lambda x: mr.A @ x, mr.apply, r.B[k], rtol=1e-8, restart=10, maxit=500)
        err = np.linalg.norm(res.p[k] - ref.p) / np.linalg.norm(ref.p)
        print(f"  rhs {k}: oracle its {ref.iterations}, rel L2 {err:.2e} (gate {gate:.1e})",
              flush=True)
        assert err <= gate
        its += ref.iterations
    assert abs(res.iterations - its) <= r.nrhs


def _mixed_contexts(dev):
    """Contexts of several sizes, boundary types and precision modes: two
    families share the serving parameters, the others differ in box widths,
    sweeps or precision."""
    cfgs = [S.config_for(128), S.config_for(256), S.config_for(128, dict(precision=0)),
            B.Config(100, 76, (1, 1, 0, 0), 12, 12, 2, 10.0, 0, 2, 2, 1, 2),
            S.config_for(192, dict(precision=1)), S.config_for(64)]
    Ks = [wl.lognormal_K(c.nx, c.ny, 2.0, 16.0, 40 + i) for i, c in enumerate(cfgs)]
    ctxs = [B.Context(c, torch.tensor(K, dtype=torch.float64, device=dev)) for c, K in zip(cfgs, Ks)]
    return cfgs, ctxs


def _rhs(c, nrhs, seed, dev):
    noflow = not any(c.bc)
    return torch.tensor(np.stack([wl.random_vector(c.nx * c.ny, seed + 7 * k, zero_mean=noflow)
                                  for k in range(nrhs)]), dtype=torch.float64,
                        device=dev).contiguous()


def test_apply_many_equals_apply(dev):
    print("apply_many: six contexts, four families, 1..3 columns each", flush=True)
    cfgs, ctxs = _mixed_contexts(dev)
    rs = [_rhs(c, 1 + i % 3, 50 + i, dev) for i, c in enumerate(cfgs)]
    for rep in range(2):   # the second call reuses the column work spaces and tables
        zs = [torch.full_like(r, 3.0) for r in rs]
        B.apply_many(ctxs, rs, zs)
        torch.cuda.synchronize()
        for c, r, z in zip(ctxs, rs, zs):
            z1 = torch.empty_like(r)
            c.apply(r, z1)
            torch.cuda.synchronize()
            assert torch.equal(z, z1)
    with pytest.raises(B.MrcmError):
        B.apply_many([ctxs[0], ctxs[0]], [rs[0], rs[0]], [zs[0], zs[0]])
    for c in ctxs:
        c.close()


def test_batch_equals_gmres_solve(dev):
    print("batched GMRES: six contexts, right-hand sides joining while others run", flush=True)
    cfgs, ctxs = _mixed_contexts(dev)
    bs = [_rhs(c, 1 + (i + 1) % 3, 90 + i, dev) for i, c in enumerate(cfgs)]
    ps = [torch.full_like(b, 5.0) for b in bs]
    batch = B.Batch(10)
    tags = {}
    ticks = 0
    for i in range(len(ctxs)):   # one more context joins every third tick
        tags[i] = batch.add(ctxs[i], bs[i], ps[i], rtol=1e-8, maxit=400)
        for _ in range(3):
            batch.tick()
            ticks += 1
    while batch.tick() > 0:
        ticks += 1
    stats = {i: batch.poll(t) for i, t in tags.items()}
    print(f"  {ticks} ticks", flush=True)
    for i, c in enumerate(ctxs):
        st = stats[i]
        assert st is not None and st.converged
        c.set_lanes(1)
        p1 = torch.zeros_like(bs[i])
        s1 = c.gmres(bs[i], p1, rtol=1e-8, restart=10, maxit=400)
        torch.cuda.synchronize()
        print(f"  context {i} ({cfgs[i].nx}x{cfgs[i].ny}, precision {cfgs[i].precision}): "
              f"iterations {st.iterations} / {s1.iterations}, identical "
              f"{torch.equal(p1, ps[i])}", flush=True)
        assert (st.iterations, st.cycles) == (s1.iterations, s1.cycles)
        assert st.final_relres == s1.final_relres
        assert torch.equal(p1, ps[i])
        batch.remove(tags[i])
    with pytest.raises(B.MrcmError):
        batch.poll(tags[0])
    # a second round on the same contexts reuses the removed tags' buffers
    held = [c.query("device_bytes") for c in ctxs]
    again = {}
    for i in (0, 3, 4):
        ps[i].fill_(-2.0)
        again[i] = batch.add(ctxs[i], bs[i], ps[i], rtol=1e-8, maxit=400)
    while batch.tick() > 0:
        pass
    for i, t in again.items():
        st = batch.poll(t)
        p1 = torch.zeros_like(bs[i])
        s1 = ctxs[i].gmres(bs[i], p1, rtol=1e-8, restart=10, maxit=400)
        torch.cuda.synchronize()
        assert st.iterations == s1.iterations and torch.equal(p1, ps[i])
        batch.remove(t)
    assert [c.query("device_bytes") for c in ctxs] == held
    batch.close()
    for c in ctxs:
        c.close()


def test_served_large_requests_in_the_serving_mode(dev):
    """512^2 and 1024^2 requests (precision 2) served together."""
    reqs = [S.make_payload(S.Request(0, 512, 2.5, 1100, 2100, 2, 0.0)),
            S.make_payload(S.Request(1, 1024, 2.0, 1101, 2101, 2, 0.0))]
    print("serving: 512^2 and 1024^2 requests together, precision 2", flush=True)
    served = S.Server(S.GpuBackend(), max_active=2).run(reqs, realtime=False)
    for r, res in zip(reqs, served):
        ctx = B.Context(S.config_for(r.n), torch.tensor(r.K, dtype=torch.float64, device=dev))
        b = torch.tensor(r.B, dtype=torch.float64, device=dev).contiguous()
        p1 = torch.zeros_like(b)
        s1 = ctx.gmres(b, p1, rtol=1e-8, restart=10, maxit=500)
        torch.cuda.synchronize()
        A = assemble(r.K, r.n, r.n, (0, 0, 0, 0))
        rel = [np.linalg.norm(r.B[k] - A @ res.p[k]) / np.linalg.norm(r.B[k])
               for k in range(r.nrhs)]
        print(f"  {r.n}^2: iterations {res.iterations} / gmres_solve {s1.iterations}, "
              f"max relres (oracle A) {max(rel):.2e}", flush=True)
        assert res.converged and res.iterations == s1.iterations
        assert np.array_equal(res.p, p1.cpu().numpy())
        assert max(rel) <= 1e-8 * (1 + 1e-6)
        ctx.close()
    # 512^2 against the oracle: its GMRES counts, and the direct solve at 1e-10
    r = reqs[0]
    p = S.SERVE_PARAMS
    mr = MRCM(r.K, nx=r.n, ny=r.n, bc=(0, 0, 0, 0), sx=p["s"], sy=p["s"],
              oversample=p["oversample"], alpha=p["alpha"], beta_len="H", sweeps=p["sweeps"],
              overlap=p["overlap"], degree=p["degree"])
    its = []
    for k in range(r.nrhs):
        ref = gmres(lambda x: mr.A @ x, mr.apply, r.B[k], rtol=1e-8, restart=10, maxit=500)
        its.append(ref.iterations)
    print(f"  512^2 oracle iterations {its} (served total {served[0].iterations})", flush=True)
    assert abs(served[0].iterations - sum(its)) <= r.nrhs
    tight = S.Server(S.GpuBackend(rtol=1e-10, maxit=800), max_active=1).run([r],
                                                                             realtime=False)[0]
    assert tight.converged
    for k in range(r.nrhs):
        exact = direct_solve(mr.A, r.B[k], (0, 0, 0, 0))
        got = tight.p[k] - tight.p[k].mean()
        err = np.linalg.norm(got - exact) / np.linalg.norm(exact)
        print(f"  512^2 rhs {k} at 1e-10: rel L2 to the direct solve {err:.2e}", flush=True)
        assert err <= 1e-7


def test_caller_allocator(dev):
    cfg = S.config_for(128)
    K = torch.tensor(wl.lognormal_K(128, 128, 2.0, 16.0, 60), dtype=torch.float64, device=dev)
    r = torch.tensor(wl.random_vector(128 * 128, 61, zero_mean=True), dtype=torch.float64,
                     device=dev)
    ref_ctx = B.Context(cfg, K)
    z0 = torch.empty_like(r)
    ref_ctx.apply(r, z0)
    torch.cuda.synchronize()
    ref_ctx.close()
    calls = {"alloc": 0, "free": 0, "live": 0}
    sizes = {}
    ta, tf = B.torch_allocator(0)

    def alloc(nbytes, stream):
        calls["alloc"] += 1
        calls["live"] += nbytes
        ptr = ta(nbytes, stream)
        sizes[ptr] = nbytes
        return ptr

    def release(ptr, stream):
        calls["free"] += 1
        calls["live"] -= sizes.pop(ptr)
        tf(ptr, stream)

    B.set_allocator(alloc, release)
    try:
        ctx = B.Context(cfg, K)
        z1 = torch.empty_like(r)
        ctx.apply(r, z1)
        torch.cuda.synchronize()
        held = ctx.query("device_bytes")
        live = calls["live"]   # set-up temporaries are already released
        ctx.close()
    finally:
        B.set_allocator(None, None)
    print(f"  allocator calls {calls}, context bytes {held:.0f}", flush=True)
    assert calls["alloc"] > 0 and calls["alloc"] == calls["free"] and calls["live"] == 0
    assert live == held
    assert torch.equal(z0, z1)


def test_failing_allocator_reports_enomem(dev):
    """Failure injection: a caller allocator that returns NULL part-way
    through the set-up makes mrcm_setup fail with MRCM_ENOMEM, and every
    allocation it had made is returned."""
    cfg = S.config_for(128)
    K = torch.tensor(wl.lognormal_K(128, 128, 2.0, 16.0, 62), dtype=torch.float64, device=dev)
    ta, tf = B.torch_allocator(0)
    calls = {"alloc": 0, "ok": 0, "free": 0}

    def alloc(nbytes, stream):
        calls["alloc"] += 1
        if calls["alloc"] > 6:
            return None
        calls["ok"] += 1
        return ta(nbytes, stream)

    def release(ptr, stream):
        calls["free"] += 1
        tf(ptr, stream)

    B.set_allocator(alloc, release)
    try:
        with pytest.raises(B.MrcmError) as e:
            B.Context(cfg, K)
    finally:
        B.set_allocator(None, None)
    print(f"  allocator calls {calls}", flush=True)
    assert e.value.code == B.MRCM_ENOMEM
    assert calls["ok"] == 6 and calls["free"] == calls["ok"]
    ctx = B.Context(cfg, K)   # the library is usable afterwards
    ctx.close()


@pytest.mark.parametrize("precision,n,nrhs,lanes,width",
                         [(2, 256, 6, 4, 1), (0, 128, 3, 2, 1), (2, 256, 7, 1, 8), (2, 256, 9, 2, 4),
                          (1, 128, 5, 2, 2), (0, 128, 4, 1, 4)])
def test_lanes_equal_one_lane(dev, precision, n, nrhs, lanes, width):
    print(f"lanes: {n}^2 precision {precision}, {nrhs} rhs on 1 lane and on {lanes} lanes of "
          f"width {width}", flush=True)
    cfg = S.config_for(n, dict(precision=precision))
    K = torch.tensor(wl.lognormal_K(n, n, 2.0, 16.0, 70), dtype=torch.float64, device=dev)
    b = torch.tensor(wl.random_pairs(n, n, nrhs, 71), dtype=torch.float64, device=dev).contiguous()
    ctx = B.Context(cfg, K)
    ctx.set_lanes(1)
    p1 = torch.zeros_like(b)
    s1 = ctx.gmres(b, p1, rtol=1e-8, restart=10, maxit=500)
    ctx.set_lanes(lanes)
    ctx.set_batch(width)
    pl = torch.full_like(b, 7.0)   # the solve must overwrite what p holds
    sl = ctx.gmres(b, pl, rtol=1e-8, restart=10, maxit=500)
    torch.cuda.synchronize()
    print(f"  iterations {s1.iterations} / {sl.iterations}, cycles {s1.cycles} / {sl.cycles}",
          flush=True)
    assert s1.converged and sl.converged
    assert (s1.iterations, s1.cycles) == (sl.iterations, sl.cycles)
    assert s1.final_relres == sl.final_relres
    assert s1.est_history == sl.est_history and s1.true_history == sl.true_history
    assert torch.equal(p1, pl)
    its = 0
    for k in range(nrhs):
        pk = torch.zeros_like(b[k])
        sk = ctx.gmres(b[k].contiguous(), pk, rtol=1e-8, restart=10, maxit=500)
        its += sk.iterations
        assert torch.equal(pk, pl[k])
    assert its == sl.iterations
    with pytest.raises(B.MrcmError):
        ctx.set_lanes(0)
    with pytest.raises(B.MrcmError):
        ctx.set_batch(9)
    ctx.close()


def test_library_loaded_before_torch_serves_from_a_worker():
    import os
    import subprocess
    import sys
    code = (
        "import sys\n"
        "from paper_2606_08883_amd import serving as S\n"
        "assert 'torch' not in sys.modules\n"
        "from paper_2606_08883_amd.binding import footprint\n"
        "print('footprint', footprint(S.config_for(128), 2), flush=True)\n"
        "assert 'torch' in sys.modules\n"
        "solver = S.GpuBackend(None, keep=True)\n"
        "req = S.make_payload(S.Request(0, 128, 2.0, 999, 1999, 2, 0.0))\n"
        "r = S.Server(solver, max_active=1).run([req], realtime=False)[0]\n"
        "print('served', r.converged, r.final_relres, flush=True)\n"
        "assert r.converged and r.final_relres <= 1e-8\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], cwd=root, capture_output=True,
                         text=True, timeout=180)
    print(out.stdout, out.stderr[-2000:], flush=True)
    assert out.returncode == 0
