"""GPU tests of the set-up autotuner.

With MRCM_TUNE=1, mrcm_setup times the free workgroup shapes of the
one-column launches (threads per chunk of every interface level; lane groups
per workgroup of the local and patch solves) and keeps the fastest.  Every
shape computes the same results bit for bit, so:

* contexts set up with the defaults (no MRCM_TUNE), with the last option of
  every choice (MRCM_TUNE=alt) and with the timed choice (MRCM_TUNE=1) give
  the same T r and the same GMRES iterates and counts, bit for bit, in every
  precision mode;
* a second context of a shape tuned before in the process reuses the cached
  choice (no timing) and gives the same results;
* at the benchmark's 1024^2 shape (interface levels of thousands of chunks,
  one-wave workgroups by default) the other shape gives the same T r.
"""
import numpy as np
import pytest

from paper_2606_08883_amd import binding as B
from paper_2606_08883_amd import workloads as wl

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [
    # (nx, ny, bc, s, oversample, sweeps, precision)
    (144, 112, (0, 0, 0, 0), 16, 4, 1, 2),
    (144, 112, (0, 0, 0, 0), 16, 4, 1, 0),
    (136, 104, (1, 1, 0, 0), 20, 2, 2, 1),   # ragged tail, Dirichlet W/E, two sweeps
]


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    B.lib()
    return torch.device("cuda:0")


def _run(cfg, K, r, b):
    ctx = B.Context(cfg, K)
    z = torch.full_like(r, np.nan)
    ctx.apply(r, z)
    p = torch.zeros_like(b)
    st = ctx.gmres(b, p, rtol=1e-8, restart=10, maxit=300, raise_on_noconv=False)
    torch.cuda.synchronize()
    out = dict(z=z.clone(), p=p.clone(), its=st.iterations, relres=st.final_relres,
               tune_ms=ctx.query("tune_ms"), changes=ctx.query("tune_changes"))
    ctx.close()
    return out


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}-s{c[3]}-k{c[5]}-p{c[6]}"
                                             for c in CASES])
def test_every_shape_same_result(dev, monkeypatch, case):
    nx, ny, bc, s, ov, sweeps, prec = case
    cfg = B.Config(nx, ny, bc, s, s, ov, 10.0, 0, sweeps, 2, 1, prec)
    K = torch.tensor(wl.lognormal_K(nx, ny, 2.0, 8.0, 81), dtype=torch.float64, device=dev)
    noflow = not any(bc)
    r = torch.tensor(wl.random_vector(nx * ny, 82, zero_mean=noflow), dtype=torch.float64,
                     device=dev)
    b = torch.tensor(wl.random_vector(nx * ny, 83, zero_mean=noflow), dtype=torch.float64,
                     device=dev)
    runs = {}
    for key, mode in (("default", None), ("alt", "alt"), ("timed", "1"), ("cached", "1")):
        if mode is None:
            monkeypatch.delenv("MRCM_TUNE", raising=False)
        else:
            monkeypatch.setenv("MRCM_TUNE", mode)
        print(f"  {case}: MRCM_TUNE={mode}", flush=True)
        runs[key] = _run(cfg, K, r, b)
    ref = runs["default"]
    print(f"  iterations {ref['its']}, alt changes {runs['alt']['changes']:.0f}, timed changes "
          f"{runs['timed']['changes']:.0f} in {runs['timed']['tune_ms']:.1f} ms", flush=True)
    assert torch.isfinite(ref["z"]).all()
    assert ref["tune_ms"] == 0.0 and ref["changes"] == 0.0
    assert runs["alt"]["changes"] >= 1
    assert runs["cached"]["tune_ms"] == 0.0
    assert runs["cached"]["changes"] == 0.0   # counted by the set-up that timed
    for key in ("alt", "timed", "cached"):
        assert torch.equal(runs[key]["z"], ref["z"]), f"T r differs with MRCM_TUNE={key}"
        assert torch.equal(runs[key]["p"], ref["p"]), f"GMRES iterate differs ({key})"
        assert runs[key]["its"] == ref["its"]
        assert runs[key]["relres"] == ref["relres"]


def test_fullsize_other_shape_same_result(dev, monkeypatch):
    from paper_2606_08883_amd.configs import WORKLOADS
    w = WORKLOADS["batched"]
    K = torch.tensor(w.permeability(), dtype=torch.float64, device=dev)
    r = torch.tensor(wl.random_vector(w.nx * w.ny, 84, zero_mean=True), dtype=torch.float64,
                     device=dev)
    zs = {}
    for mode in ("0", "alt"):
        monkeypatch.setenv("MRCM_TUNE", mode)   # 0 (not 1 or alt): the defaults
        print(f"  {w.nx}x{w.ny}: MRCM_TUNE={mode}", flush=True)
        ctx = B.Context(w.binding_config(), K)
        z = torch.full_like(r, np.nan)
        ctx.apply(r, z)
        torch.cuda.synchronize()
        zs[mode] = (z, ctx.query("tune_changes"))
        ctx.close()
    assert zs["alt"][1] >= 1
    assert torch.isfinite(zs["0"][0]).all()
    assert torch.equal(zs["alt"][0], zs["0"][0])
