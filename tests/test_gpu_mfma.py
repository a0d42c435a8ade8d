"""GPU tests of the matrix-core reconstruction (MRCM_MFMA_RECON).

With MRCM_MFMA_RECON=mfma at set-up, the reconstruction p[Omega_i] += P_i x_i
(Section 2.1, the multiscale basis functions) of 8-column applications runs
as 16 x 16 MFMA tiles in the arithmetic type (FP64 in modes 0 and 2, FP32 in
mode 1); with MRCM_MFMA_RECON=bf16 (mode 1) its inputs are rounded to BF16
and accumulated in FP32.  The MFMA sums round differently from the FMA
chain, so the 8-column result is compared with one-column applications
within a rounding bound, and with the oracle's T within the gate of the
mode (FP64: the FP64 gate; modes 1 and 2: the mixed-precision gate of the
box factors; BF16: the BF16 rounding of P and x, 2^-8 relative, on the
coarse part).  GMRES with 8 right-hand sides per application still meets
the tolerance on the true residual, with iterations within one of the FMA
path per right-hand side (BF16: reported, at most twice).
"""
import os

import numpy as np
import pytest

from oracle.mrcm import MRCM
from paper_2606_08883_amd import binding as B
from paper_2606_08883_amd import workloads as wl
from tests._gates import mixed_t_gate, t_gate

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, S = 128, 16


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    B.lib()
    return torch.device("cuda:0")


def _context(dev, precision, mode):
    cfg = B.Config(N, N, (0, 0, 0, 0), S, S, 4, 10.0, 0, 1, 2, 1, precision)
    K = wl.lognormal_K(N, N, 2.0, 16.0, 120)
    old = os.environ.get("MRCM_MFMA_RECON")
    if mode:
        os.environ["MRCM_MFMA_RECON"] = mode
    else:
        os.environ.pop("MRCM_MFMA_RECON", None)
    try:
        ctx = B.Context(cfg, torch.tensor(K, dtype=torch.float64, device=dev))
    finally:
        if old is None:
            os.environ.pop("MRCM_MFMA_RECON", None)
        else:
            os.environ["MRCM_MFMA_RECON"] = old
    return cfg, K, ctx


@pytest.mark.parametrize("precision,mode", [(0, "mfma"), (2, "mfma"), (1, "mfma"), (1, "bf16")])
def test_mfma_reconstruction(dev, precision, mode):
    print(f"mfma: precision {precision}, {mode}", flush=True)
    cfg, K, ctx = _context(dev, precision, mode)
    assert ctx.query("mfma_recon") == (2 if mode == "bf16" else 1)
    n = N * N
    R = np.stack([wl.random_vector(n, 130 + k, zero_mean=True) for k in range(8)])
    r = torch.tensor(R, dtype=torch.float64, device=dev).contiguous()
    z8 = torch.full_like(r, np.nan)
    ctx.apply(r, z8)
    z1 = torch.full_like(r, np.nan)
    for k in range(8):
        ctx.apply(r[k].contiguous(), z1[k])
    torch.cuda.synchronize()
    assert torch.isfinite(z8).all()
    d = (torch.linalg.norm(z8 - z1) / torch.linalg.norm(z1)).item()
    mr = MRCM(K, N, N, (0, 0, 0, 0), S, S, 4, 10.0, "H", 1, 2, 1)
    ref = np.stack([mr.apply(R[k]) for k in range(8)])
    e8 = np.linalg.norm(z8.cpu().numpy() - ref) / np.linalg.norm(ref)
    e1 = np.linalg.norm(z1.cpu().numpy() - ref) / np.linalg.norm(ref)
    gate = t_gate(mr) if precision == 0 else mixed_t_gate(mr)
    bound = {0: 1e-13, 2: 1e-13, 1: 1e-5}[precision] if mode == "mfma" else 2.0 ** -8
    print(f"  8 columns vs one-column {d:.2e} (bound {bound:.1e}); oracle: 8 columns {e8:.2e}, "
          f"one column {e1:.2e} (gate {gate:.1e})", flush=True)
    assert d <= bound
    assert e8 <= (gate if mode == "mfma" else 2.0 ** -8)
    # GMRES with 8 right-hand sides per application
    b = torch.tensor(wl.random_pairs(N, N, 8, 140), dtype=torch.float64, device=dev).contiguous()
    ctx.set_lanes(1)
    ctx.set_batch(8)
    p8 = torch.zeros_like(b)
    s8 = ctx.gmres(b, p8, rtol=1e-8, restart=10, maxit=400)
    _, _, plain = _context(dev, precision, None)
    plain.set_lanes(1)
    plain.set_batch(8)
    p0 = torch.zeros_like(b)
    s0 = plain.gmres(b, p0, rtol=1e-8, restart=10, maxit=400)
    torch.cuda.synchronize()
    print(f"  GMRES 8 rhs: iterations {s8.iterations} (FMA path {s0.iterations}), "
          f"relres {s8.final_relres:.2e}", flush=True)
    assert s8.converged and s8.final_relres <= 1e-8
    if mode == "mfma":
        assert abs(s8.iterations - s0.iterations) <= 8
    else:
        assert s8.iterations <= 2 * s0.iterations
    ctx.close()
    plain.close()
