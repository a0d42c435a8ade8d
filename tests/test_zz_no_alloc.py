"""mrcm_apply_noalloc (the entry point for callers that cannot allocate)
against mrcm_apply, through the C ABI: two calls in a row on two contexts,
the second smaller, each column equal bit for bit to a one-column
mrcm_apply; a context too large for the static work space is rejected."""
import numpy as np
import pytest

from paper_2606_08883_amd import binding as B
from paper_2606_08883_amd import workloads as wl
from paper_2606_08883_amd.configs import WORKLOADS

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    B.lib()
    return torch.device("cuda:0")


def _check(ctx, w, nrhs, seed, dev):
    r = torch.tensor(wl.random_vector(nrhs * w.cells, seed).reshape(nrhs, -1),
                     dtype=torch.float64, device=dev)
    z = torch.full_like(r, np.nan)
    ctx.apply_noalloc(r, z)
    torch.cuda.synchronize()
    for k in range(nrhs):
        ref = torch.empty(w.cells, dtype=torch.float64, device=dev)
        ctx.apply(r[k].contiguous(), ref)
        torch.cuda.synchronize()
        assert torch.equal(z[k], ref), k


def test_noalloc_equals_apply_twice_then_smaller(dev):
    w1 = WORKLOADS["batched"].with_(nx=256, ny=256, precision=0)
    w2 = WORKLOADS["small"].with_(precision=2)
    print("apply_noalloc: 256^2 FP64, 3 columns; then 64^2 mode 2, 1 column", flush=True)
    c1 = B.Context(w1.binding_config(),
                   torch.tensor(wl.lognormal_K(256, 256, 3.0, 16.0, 3), device=dev))
    c2 = B.Context(w2.binding_config(), torch.tensor(w2.permeability(), device=dev))
    _check(c1, w1, 3, 41, dev)
    _check(c2, w2, 1, 42, dev)
    _check(c1, w1, 1, 43, dev)
    c1.close()
    c2.close()


def test_noalloc_rejects_a_context_beyond_the_static_array(dev):
    w = WORKLOADS["small"].with_(nx=4200, ny=4096, s=32, oversample=2, sweeps=0)
    print("apply_noalloc: 4200x4096 FP64 context (work space above 256 MiB)", flush=True)
    ctx = B.Context(w.binding_config(), torch.ones(w.cells, dtype=torch.float64, device=dev))
    r = torch.zeros(w.cells, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    with pytest.raises(B.MrcmError) as e:
        ctx.apply_noalloc(r, z)
    assert e.value.code == B.MRCM_EINVAL and "work space" in str(e.value)
    ctx.close()
