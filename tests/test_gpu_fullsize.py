"""GPU parity at the benchmark's full sizes, in the configurations bench.py times.

* 1024 x 1024 log-normal workload (4096 subdomains), precision modes 2 (the
  benchmark's) and 0: T r and the GMRES solution element by element against
  the oracle, iteration counts within +-1 (mode 0) / +2 (mode 2).  The
  interface system of this field has cond_1(C) ~ 4e10, so the FP64 gate is
  the forward-error bound cond(C) * 2^-53 (tests/_gates.py), not 1e-10.
* 4096 x 4096 mixture workload (16384 subdomains, contrast 1e8), precision
  mode 2: the oracle's MRCM setup takes minutes there, so the check uses
  what holds at any size: A x element by element against the oracle's sparse
  A, zero mean and run-to-run bit identity of T r, and the true residual
  the library reports for a GMRES cycle recomputed with the oracle's A.
"""
import numpy as np
import pytest

from oracle.gmres import gmres
from oracle.discretization import assemble
from oracle.mrcm import MRCM
from paper_2606_08883_amd import binding as B
from paper_2606_08883_amd import workloads as wl
from paper_2606_08883_amd.configs import WORKLOADS
from tests._gates import t_gate

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    B.lib()
    return torch.device("cuda:0")


def T(x, dev):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def residual_gate(A, p, b):
    """Bound on the difference of two FP64 evaluations of ||b - A p|| / ||b||
    that sum in different orders.  Each residual entry carries a rounding
    error of at most about 6 u (|A| |p| + |b|) (five products and sums).  The
    norms add the error of summing n squares: at most m u relative with m the
    longest chain of additions, here the library's grid-stride per-thread sum
    (n / (1024 * 256) terms), the in-block tree (8) and the sequential sum of
    up to 1024 block partials (numpy's pairwise sum is shorter), so the norm,
    a square root, moves by at most m u / 2 relative."""
    u = 2.0 ** -53
    n = b.size
    m = n // (1024 * 256) + 1 + 8 + 1024
    relres = np.linalg.norm(b - A @ p) / np.linalg.norm(b)
    entry = 6.0 * u * np.linalg.norm(abs(A) @ np.abs(p) + np.abs(b)) / np.linalg.norm(b)
    return entry + m * u * relres


@pytest.fixture(scope="module")
def batched_oracle():
    w = WORKLOADS["batched"]
    print(f"oracle setup {w.nx}x{w.ny}", flush=True)
    K = w.permeability()
    mr = MRCM(K, **w.oracle_args())
    b = w.rhs()
    r = wl.random_vector(w.cells, 11, zero_mean=True)
    print("oracle T r and GMRES", flush=True)
    Tr = mr.apply(r)
    ref = gmres(lambda x: mr.A @ x, mr.apply, b, rtol=1e-8, restart=10, maxit=300)
    gate = t_gate(mr)
    print(f"interface forward-error gate {gate:.2e}", flush=True)
    return w, K, mr, b, r, Tr, ref, gate


@pytest.mark.timeout(900)
@pytest.mark.parametrize("precision", [2, 0])
def test_batched_fullsize(dev, batched_oracle, precision):
    w, K, mr, b, r, Tr, ref, tg = batched_oracle
    w = w.with_(precision=precision)
    print(f"batched {w.nx}x{w.ny} precision {precision}", flush=True)
    ctx = B.Context(w.binding_config(), T(K, dev))
    z = torch.empty(w.cells, dtype=torch.float64, device=dev)
    ctx.apply(T(r, dev), z)
    errT = np.linalg.norm(z.cpu().numpy() - Tr) / np.linalg.norm(Tr)
    p = torch.zeros(w.cells, dtype=torch.float64, device=dev)
    st = ctx.gmres(T(b, dev), p, rtol=1e-8, restart=10, maxit=300)
    pg = p.cpu().numpy()
    err = np.linalg.norm(pg - ref.p) / np.linalg.norm(ref.p)
    relres = np.linalg.norm(b - mr.A @ pg) / np.linalg.norm(b)
    print(f"  T rel L2 {errT:.2e}; its gpu {st.iterations} oracle {ref.iterations}; "
          f"p rel L2 {err:.2e}; relres (oracle A) {relres:.2e} reported {st.final_relres:.2e}",
          flush=True)
    ctx.close()
    gate = residual_gate(mr.A, pg, b)
    print(f"  residual rounding bound {gate:.2e}", flush=True)
    assert st.converged and relres <= 1e-8 + gate
    assert abs(relres - st.final_relres) <= gate
    if precision == 0:
        # FP64: the interface system's forward-error bound (cond(C) * 2^-53)
        assert errT <= tg
        assert abs(st.iterations - ref.iterations) <= 1
        assert err <= tg
    else:
        # FP32-stored factors: T differs by the FP32 rounding of the factors;
        # the solutions agree to the tolerance both were driven to.
        assert errT <= 1e-4
        assert st.iterations <= ref.iterations + 2
        assert err <= 1e-6


@pytest.mark.timeout(900)
def test_large_fullsize_properties(dev):
    w = WORKLOADS["large"]
    print(f"large {w.nx}x{w.ny} precision {w.precision}: permeability", flush=True)
    K = w.permeability()
    A = assemble(K, w.nx, w.ny, w.bc)
    print("  setup", flush=True)
    ctx = B.Context(w.binding_config(), T(K, dev))
    x = wl.random_vector(w.cells, 12)
    y = torch.empty(w.cells, dtype=torch.float64, device=dev)
    ctx.op(T(x, dev), y)
    ref = A @ x
    errA = np.linalg.norm(y.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"  op_apply rel L2 {errA:.2e}", flush=True)
    assert errA <= 1e-13

    r = T(wl.random_vector(w.cells, 13, zero_mean=True), dev)
    z1 = torch.empty_like(r)
    z2 = torch.empty_like(r)
    ctx.apply(r, z1)
    ctx.apply(r, z2)
    zc = z1.cpu().numpy()
    mean_rel = abs(zc.mean()) / np.abs(zc).max()
    print(f"  T r: |mean| / max {mean_rel:.2e}; bit-identical repeat "
          f"{bool(torch.equal(z1, z2))}", flush=True)
    assert torch.equal(z1, z2)
    assert mean_rel <= 1e-12 and np.all(np.isfinite(zc))

    b = w.rhs()
    p = torch.zeros(w.cells, dtype=torch.float64, device=dev)
    st = ctx.gmres(T(b, dev), p, rtol=1e-8, restart=10, maxit=10, raise_on_noconv=False)
    pg = p.cpu().numpy()
    relres = np.linalg.norm(b - A @ pg) / np.linalg.norm(b)
    print(f"  one GMRES cycle: {st.iterations} its, relres (oracle A) {relres:.3e} "
          f"reported {st.final_relres:.3e}", flush=True)
    ctx.close()
    assert st.iterations == 10
    assert abs(relres - st.final_relres) <= residual_gate(A, pg, b)
    assert relres <= 1.0 + 1e-12  # GMRES never increases the residual from p_0 = 0
