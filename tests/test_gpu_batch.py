"""GPU tests of the multi-RHS applications of T.

mrcm_apply with nrhs > 1 runs the steps of T on 8, 4 or 2 columns per launch
(each factor quad, MBF entry and interface-matrix tile loaded once for all
columns).  Every per-column sum keeps the order of the one-column kernels, so
the result must equal nrhs separate one-column applications bit for bit, for
every precision mode, box width (subdomains of 16 to 40 cells, patches up to
44), boundary type and column count (including counts that split into
several launches).  The one-column path itself is checked against the oracle
in the parity tests.
"""
import numpy as np
import pytest

from paper_2606_08883_amd import binding as B
from paper_2606_08883_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # (nx, ny, bc, s, oversample, sweeps, precision)
    (128, 128, (0, 0, 0, 0), 16, 4, 1, 2),
    (128, 128, (0, 0, 0, 0), 16, 4, 1, 0),
    (128, 128, (0, 0, 0, 0), 16, 4, 1, 1),
    (150, 118, (1, 1, 0, 0), 20, 2, 2, 2),   # ragged tail, Dirichlet W/E, two sweeps
    (160, 96, (0, 0, 0, 0), 32, 4, 1, 2),    # 32-wide subdomains, 36-wide patches
    (200, 120, (1, 0, 0, 1), 40, 2, 1, 0),   # 40-wide subdomains, 44-wide patches, FP64
    (96, 64, (0, 0, 0, 0), 16, 0, 0, 2),     # no oversampling, no smoothing
]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    B.lib()
    return torch.device("cuda:0")


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-s{c[3]}-l{c[4]}-k{c[5]}-p{c[6]}"
                                             for c in CASES])
def test_multi_rhs_apply_equals_columns(dev, case):
    nx, ny, bc, s, ov, sweeps, prec = case
    cfg = B.Config(nx, ny, bc, s, s, ov, 10.0, 0, sweeps, 2, 1, prec)
    K = torch.tensor(wl.lognormal_K(nx, ny, 2.0, 8.0, 91), dtype=torch.float64, device=dev)
    ctx = B.Context(cfg, K)
    n = nx * ny
    for nrhs in (2, 3, 4, 7, 8, 11):
        print(f"  {case}: {nrhs} columns", flush=True)
        r = torch.tensor(np.stack([wl.random_vector(n, 100 + 13 * k, zero_mean=not any(bc))
                                   for k in range(nrhs)]), dtype=torch.float64,
                         device=dev).contiguous()
        z = torch.full_like(r, np.nan)
        ctx.apply(r, z)
        zc = torch.full_like(r, np.nan)
        for k in range(nrhs):
            ctx.apply(r[k].contiguous(), zc[k])
        torch.cuda.synchronize()
        assert torch.isfinite(z).all()
        assert torch.equal(z, zc), f"{nrhs} columns differ from one-column applications"
    ctx.close()


def test_multi_rhs_apply_timing_phases(dev):
    """Per-phase timing also covers the multi-RHS launches (one mark set per
    batch of columns)."""
    cfg = B.Config(128, 128, (0, 0, 0, 0), 16, 16, 4, 10.0, 0, 1, 2, 1, 2)
    K = torch.tensor(wl.lognormal_K(128, 128, 2.0, 8.0, 92), dtype=torch.float64, device=dev)
    ctx = B.Context(cfg, K)
    r = torch.tensor(np.stack([wl.random_vector(128 * 128, 200 + k, zero_mean=True)
                               for k in range(8)]), dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    ctx.timing(True)
    ctx.apply(r, z)
    torch.cuda.synchronize()
    ph = ctx.timing_read()
    ctx.timing(False)
    assert all(ph[name][1] == 1 for name in ("local", "coarse", "reconstruct", "residual",
                                             "patch", "finalize"))
    ctx.close()


def test_multi_rhs_apply_equals_columns_fullsize(dev):
    """At 1024^2 the leaf levels of the interface solve have thousands of
    chunks and run as one-wave workgroups that take their chunk whole; the
    multi-column kernels must still reproduce them bit for bit."""
    from paper_2606_08883_amd.configs import WORKLOADS
    w = WORKLOADS["batched"]
    K = torch.tensor(w.permeability(), dtype=torch.float64, device=dev)
    ctx = B.Context(w.binding_config(), K)
    n = w.nx * w.ny
    r = torch.tensor(np.stack([wl.random_vector(n, 400 + k, zero_mean=True) for k in range(3)]),
                     dtype=torch.float64, device=dev).contiguous()
    z = torch.full_like(r, np.nan)
    ctx.apply(r, z)
    zc = torch.full_like(r, np.nan)
    for k in range(3):
        ctx.apply(r[k].contiguous(), zc[k])
    torch.cuda.synchronize()
    assert torch.isfinite(z).all()
    assert torch.equal(z, zc)
    ctx.close()
