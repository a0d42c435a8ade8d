"""GPU parity of the 3-D path (include/mrcm3d.h) against the 3-D oracle.

* op_apply: the seven-point operator elementwise against the oracle's A.
* T: the device application against the oracle's T (oracle.mrcm3d) within
  the FP64 gate derived from Skeel's condition number of the interface
  matrix, and against the library's own host evaluation of the uploaded
  tables within the same gate (the two differ only in the order of the sums
  of the interface solve, whose forward error that gate bounds); run-to-run
  bit identity.
* GMRES(10): the same step count as the oracle's GMRES with the same T, the
  solution compared with the oracle's iterate at the same step, and the
  reported true residual checked with the oracle's A.
Grids: Dirichlet and all-no-flow sides, ragged subdomain layers, with and
without oversampling and smoothing, one subdomain covering the grid, and a
32^3 grid of 64 subdomains of 8^3 (12^3 oversampled boxes).
"""
import numpy as np
import pytest

from oracle import mrcm3d as M3
from oracle.gmres import gmres
from paper_2606_08883_amd import binding as B
from tests._gates import mixed_t_gate3, t_gate

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # nx, ny, nz, (sx, sy, sz), l, k, bc
    (12, 10, 8, (4, 5, 4), 0, 0, (1, 1, 0, 0, 0, 0)),
    (12, 10, 8, (4, 5, 4), 2, 1, (1, 1, 0, 0, 0, 0)),
    (12, 12, 12, (4, 4, 4), 2, 2, (0,) * 6),
    (14, 9, 13, (5, 3, 5), 1, 1, (0, 1, 1, 0, 0, 1)),
    (8, 8, 8, (8, 8, 8), 0, 1, (0,) * 6),
    (32, 32, 32, (8, 8, 8), 2, 1, (1, 1, 0, 0, 0, 0)),
]
IDS = [f"{c[0]}x{c[1]}x{c[2]}-s{c[3][0]}-l{c[4]}-k{c[5]}-{'D' if any(c[6]) else 'N'}" for c in CASES]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    B.lib()
    return torch.device("cuda:0")


def _field(n, seed, sigma=1.5):
    return np.exp(sigma * np.random.Generator(np.random.PCG64(seed)).standard_normal(n))


def _vec(n, seed, zero_mean):
    v = np.random.Generator(np.random.PCG64(seed)).standard_normal(n)
    return v - v.mean() if zero_mean else v


def _setup(case, dev, seed=3, precision=0):
    nx, ny, nz, s, l, k, bc = case
    n = nx * ny * nz
    K = _field(n, seed)
    cfg = B.Config3(nx, ny, nz, bc, *s, l, 10.0, 0, k, 2, 1, precision)
    ctx = B.Context3(cfg, torch.tensor(K, dtype=torch.float64, device=dev))
    mr = M3.MRCM3D(K, nx, ny, nz, bc, *s, l, 10.0, "H", k, 2, 1)
    return cfg, K, ctx, mr


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_op_and_apply_3d(dev, case):
    print(f"3-D op and T: {case}", flush=True)
    cfg, K, ctx, mr = _setup(case, dev)
    n = cfg.n
    noflow = not any(cfg.bc)
    x = _vec(n, 5, False)
    y = torch.empty(n, dtype=torch.float64, device=dev)
    ctx.op(torch.tensor(x, dtype=torch.float64, device=dev), y)
    torch.cuda.synchronize()
    ref = mr.A @ x
    assert np.abs(y.cpu().numpy() - ref).max() <= 1e-14 * np.abs(ref).max()
    r = _vec(n, 6, noflow)
    rd = torch.tensor(r, dtype=torch.float64, device=dev)
    z = torch.full_like(rd, np.nan)
    ctx.apply(rd, z)
    z2 = torch.full_like(rd, np.nan)
    ctx.apply(rd, z2)
    torch.cuda.synchronize()
    assert torch.equal(z, z2)
    zg = z.cpu().numpy()
    zo = mr.apply(r)
    zh, nc = B.test3d_host_apply(cfg, K, r)
    gate = t_gate(mr)
    err = np.linalg.norm(zg - zo) / np.linalg.norm(zo)
    errh = np.linalg.norm(zg - zh) / np.linalg.norm(zh)
    print(f"  nc {nc}; T rel L2 to the oracle {err:.2e} (gate {gate:.1e}), to the host "
          f"evaluation {errh:.2e}", flush=True)
    assert nc == mr.part.nc
    assert err <= gate
    assert errh <= gate
    ctx.close()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_gmres_3d(dev, case):
    print(f"3-D GMRES: {case}", flush=True)
    cfg, K, ctx, mr = _setup(case, dev)
    n = cfg.n
    b = _vec(n, 8, not any(cfg.bc))
    bd = torch.tensor(b, dtype=torch.float64, device=dev)
    p = torch.full_like(bd, 3.0)
    st = ctx.gmres(bd, p, rtol=1e-8, restart=10, maxit=300)
    torch.cuda.synchronize()
    ref = gmres(lambda v: mr.A @ v, mr.apply, b, rtol=1e-8, restart=10, maxit=300)
    at = gmres(lambda v: mr.A @ v, mr.apply, b, rtol=0.0, restart=10, maxit=st.iterations,
               atol=0.0)
    pg = p.cpu().numpy()
    err = np.linalg.norm(pg - at.p) / np.linalg.norm(at.p)
    rel = np.linalg.norm(b - mr.A @ pg) / np.linalg.norm(b)
    gate = t_gate(mr)
    print(f"  its gpu {st.iterations} oracle {ref.iterations}; p rel L2 at the same step "
          f"{err:.2e} (gate {gate:.1e}); relres (oracle A) {rel:.2e} reported "
          f"{st.final_relres:.2e}", flush=True)
    assert st.converged and ref.converged
    assert abs(st.iterations - ref.iterations) <= 1
    assert err <= gate
    assert rel <= 1e-8 * (1 + 1e-6)
    assert abs(rel - st.final_relres) <= 1e-3 * rel + 1e-15
    ctx.close()


def test_oversized_3d_box_rejected(dev):
    n = 20 * 20 * 8
    K = torch.ones(n, dtype=torch.float64, device=dev)
    with pytest.raises(B.MrcmError) as e:   # 20 x 20 planes exceed 256 cells
        B.Context3(B.Config3(20, 20, 8, (1,) * 6, 20, 20, 8, 0), K)
    assert e.value.code == B.MRCM_EINVAL


def test_cube_workload_on_the_device(dev):
    """The 96^3 cube workload (1728 subdomains of 8^3, 38016 interface dofs, a
    dissection with separators of up to 144 subdomains): T on the device
    against the library's host evaluation of the same tables (pinned to the
    oracle on the grids above), and GMRES to 1e-8 with the true residual
    recomputed by the device operator."""
    from paper_2606_08883_amd.configs import WORKLOADS3
    w = WORKLOADS3["cube"]
    cfg = w.binding_config()
    n = w.cells
    K = w.permeability()
    print(f"3-D cube workload {w.nx}x{w.ny}x{w.nz}", flush=True)
    ctx = B.Context3(cfg, torch.tensor(K, dtype=torch.float64, device=dev))
    r = _vec(n, 6, True)
    rd = torch.tensor(r, dtype=torch.float64, device=dev)
    z = torch.full_like(rd, np.nan)
    ctx.apply(rd, z)
    torch.cuda.synchronize()
    zh, nc = B.test3d_host_apply(cfg, K, r)
    errh = np.linalg.norm(z.cpu().numpy() - zh) / np.linalg.norm(zh)
    print(f"  nc {nc}; T rel L2 to the host evaluation {errh:.2e}; refinement steps "
          f"{ctx.query('coarse_refine'):.0f}", flush=True)
    assert nc == ctx.query("coarse_dofs") == 38016
    assert errh <= 1e-10
    b = torch.tensor(w.rhs(), dtype=torch.float64, device=dev)
    p = torch.zeros_like(b)
    st = ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=500)
    y = torch.empty_like(b)
    ctx.op(p, y)
    torch.cuda.synchronize()
    rel = (torch.linalg.norm(b - y) / torch.linalg.norm(b)).item()
    print(f"  GMRES {st.iterations} steps, relres {rel:.2e} (reported {st.final_relres:.2e})",
          flush=True)
    assert st.converged and rel <= 1e-8 * (1 + 1e-6)
    assert abs(rel - st.final_relres) <= 1e-3 * rel
    ctx.close()


MIXED = [CASES[1], CASES[2], CASES[3], CASES[5]]


@pytest.mark.parametrize("case", MIXED, ids=[IDS[CASES.index(c)] for c in MIXED])
def test_fp32_storage_3d(dev, case):
    """Precision 2 (plane blocks stored in FP32, FP64 arithmetic): the device T
    against the host evaluation of the same rounded tables and against the
    oracle's FP64 T within the recurrence bound; GMRES takes the oracle's step
    count within one and reaches 1e-8 by the oracle's A.

    Device and host differ only in the order of FP64 sums, within the FP64
    gate.  On all-no-flow grids the difference exceeds FP64 rounding (1.9e-12
    on 12^3): the rounded blocks leave the interface right-hand side
    inconsistent with the pinned system by about 1e-8, its response carries a
    large near-constant part that the final projection removes, and the two
    summation orders round that part differently (in FP64 mode, 2e-15)."""
    print(f"3-D FP32 storage: {case}", flush=True)
    cfg, K, ctx, mr = _setup(case, dev, precision=2)
    n = cfg.n
    r = _vec(n, 6, not any(cfg.bc))
    rd = torch.tensor(r, dtype=torch.float64, device=dev)
    z = torch.full_like(rd, np.nan)
    ctx.apply(rd, z)
    torch.cuda.synchronize()
    zg = z.cpu().numpy()
    zh, _ = B.test3d_host_apply(cfg, K, r)
    zo = mr.apply(r)
    errh = np.linalg.norm(zg - zh) / np.linalg.norm(zh)
    err = np.linalg.norm(zg - zo) / np.linalg.norm(zo)
    gate = mixed_t_gate3(mr)
    b = _vec(n, 8, not any(cfg.bc))
    bd = torch.tensor(b, dtype=torch.float64, device=dev)
    p = torch.zeros_like(bd)
    st = ctx.gmres(bd, p, rtol=1e-8, restart=10, maxit=300)
    torch.cuda.synchronize()
    ref = gmres(lambda v: mr.A @ v, mr.apply, b, rtol=1e-8, restart=10, maxit=300)
    rel = np.linalg.norm(b - mr.A @ p.cpu().numpy()) / np.linalg.norm(b)
    print(f"  T to the host evaluation {errh:.2e}, to the oracle {err:.2e} (gate {gate:.1e}); "
          f"its {st.iterations} (oracle {ref.iterations}); relres {rel:.2e}", flush=True)
    assert errh <= 1e-10
    assert err <= gate
    assert st.converged and abs(st.iterations - ref.iterations) <= 1
    assert rel <= 1e-8 * (1 + 1e-6)
    ctx.close()


def test_rhs_and_dirichlet_solve_3d(dev):
    """mrcm3d_rhs against the oracle's right-hand side (random source and face
    values on all six sides, of which the no-flow sides' are ignored), and
    the GMRES solution of A p = b driven to 1e-10 against the sparse direct
    solve (the plain definition of the converged result)."""
    case = CASES[3]   # 14 x 9 x 13, Dirichlet on E, S and T
    print(f"3-D right-hand side and Dirichlet solve: {case}", flush=True)
    cfg, K, ctx, mr = _setup(case, dev)
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    rng = np.random.Generator(np.random.PCG64(11))
    f = rng.standard_normal(cfg.n)
    shapes = [(nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)]
    sides = [rng.standard_normal(sh) for sh in shapes]
    h = 1.0 / nx
    b_ref = M3.rhs(K, nx, ny, nz, cfg.bc, f, {sd: sides[sd] for sd in range(6)}, h)
    T = lambda a: torch.tensor(np.ascontiguousarray(a).ravel(), dtype=torch.float64, device=dev)  # noqa: E731
    b = torch.empty(cfg.n, dtype=torch.float64, device=dev)
    ctx.rhs(T(f), T(np.concatenate([x.ravel() for x in sides])), h, b)
    b0 = torch.empty_like(b)
    ctx.rhs(None, None, h, b0)
    torch.cuda.synchronize()
    bg = b.cpu().numpy()
    assert np.abs(bg - b_ref).max() <= 1e-15 * np.abs(b_ref).max()
    assert not b0.abs().max().item()
    p = torch.zeros_like(b)
    st = ctx.gmres(b, p, rtol=1e-10, restart=10, maxit=300)
    torch.cuda.synchronize()
    p_ref = M3.direct_solve(mr.A, b_ref, cfg.bc)
    err = np.linalg.norm(p.cpu().numpy() - p_ref) / np.linalg.norm(p_ref)
    print(f"  GMRES {st.iterations} steps; solution against the direct solve {err:.2e}", flush=True)
    assert st.converged and err <= 1e-7
    ctx.close()


def test_caller_allocator_3d(dev):
    """3-D contexts set up while a caller allocator is installed
    (mrcm_set_allocator) take all their device memory from it, return every
    allocation at destroy and compute the same T r bit for bit; an allocator
    that returns NULL part-way through the set-up gives MRCM_ENOMEM with every
    allocation returned."""
    cfg, K, ctx0, mr = _setup(CASES[1], dev)
    Kd = torch.tensor(K, dtype=torch.float64, device=dev)
    r = torch.tensor(_vec(cfg.n, 6, False), dtype=torch.float64, device=dev)
    z0 = torch.empty_like(r)
    ctx0.apply(r, z0)
    torch.cuda.synchronize()
    ctx0.close()
    ta, tf = B.torch_allocator(0)
    calls = {"alloc": 0, "free": 0, "live": 0, "fail_after": None}
    sizes = {}

    def alloc(nbytes, stream):
        calls["alloc"] += 1
        if calls["fail_after"] is not None and calls["alloc"] > calls["fail_after"]:
            return None
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
        ctx = B.Context3(cfg, Kd)
        z1 = torch.empty_like(r)
        ctx.apply(r, z1)
        torch.cuda.synchronize()
        held, live = ctx.query("device_bytes"), calls["live"]
        ctx.close()
        done = dict(calls)
        calls.update(alloc=0, free=0, fail_after=5)
        with pytest.raises(B.MrcmError) as e:
            B.Context3(cfg, Kd)
    finally:
        B.set_allocator(None, None)
    print(f"  allocator calls {done}, context bytes {held:.0f}; failing run {calls}", flush=True)
    assert done["alloc"] > 0 and done["alloc"] == done["free"] and done["live"] == 0
    assert live == held
    assert torch.equal(z0, z1)
    assert e.value.code == B.MRCM_ENOMEM
    assert calls["free"] == 5 and calls["live"] == 0
