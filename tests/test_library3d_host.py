"""The 3-D library set-up on the host against the 3-D oracle (CPU).

mrcm3d_test_host_apply evaluates T from the exact tables mrcm3d_setup
uploads (plane-block factors of the oversampled boxes and patches, trace
tables, multiscale basis functions, the dense interface inverse with one
refinement step) in the order the device applies them; it must match the
oracle's T (oracle.mrcm3d) within the FP64 gate, on Dirichlet and all-no-flow
grids, with and without oversampling and smoothing, and on ragged grids.
Invalid configurations are rejected.
"""
import numpy as np
import pytest

from oracle import mrcm3d as M3
from paper_2606_08883_amd import binding as B
from tests._gates import mixed_t_gate3

CASES = [
    # nx, ny, nz, (sx, sy, sz), l, k, bc
    (12, 10, 8, (4, 5, 4), 0, 0, (1, 1, 0, 0, 0, 0)),
    (12, 10, 8, (4, 5, 4), 2, 1, (1, 1, 0, 0, 0, 0)),
    (12, 12, 12, (4, 4, 4), 2, 2, (0,) * 6),
    (14, 9, 13, (5, 3, 5), 1, 1, (0, 1, 1, 0, 0, 1)),   # ragged in x and z
    (8, 8, 8, (8, 8, 8), 0, 1, (0,) * 6),                # one subdomain: A^-1, pinned
]


def _field(n, seed):
    return np.exp(1.5 * np.random.Generator(np.random.PCG64(seed)).standard_normal(n))


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}-l{c[4]}-k{c[5]}" for c in CASES])
def test_host_apply_matches_oracle(case):
    nx, ny, nz, s, l, k, bc = case
    n = nx * ny * nz
    K = _field(n, 3)
    r = np.random.Generator(np.random.PCG64(7)).standard_normal(n)
    if not any(bc):
        r -= r.mean()
    mr = M3.MRCM3D(K, nx, ny, nz, bc, *s, l, 10.0, "H", k, 2, 1)
    z_ref = mr.apply(r)
    z, nc = B.test3d_host_apply(B.Config3(nx, ny, nz, bc, *s, l, 10.0, 0, k, 2, 1), K, r)
    assert nc == mr.part.nc
    assert np.linalg.norm(z - z_ref) <= 1e-10 * np.linalg.norm(z_ref)


def test_invalid_3d_configurations_rejected():
    n = 14 * 9 * 11
    K = _field(n, 4)
    r = np.zeros(n)
    with pytest.raises(B.MrcmError) as e:   # oversampling crosses into a thin last layer
        B.test3d_host_apply(B.Config3(14, 9, 11, (0, 1, 1, 0, 0, 1), 5, 4, 4, 1), K, r)
    assert e.value.code == B.MRCM_EINVAL
    K[5] = 0.0
    with pytest.raises(B.MrcmError) as e:
        B.test3d_host_apply(B.Config3(14, 9, 11, (1,) * 6, 7, 9, 11, 0), K, r)
    assert e.value.code == B.MRCM_EINVAL


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 2, 2), (3, 2, 2), (5, 4, 3), (6, 6, 6), (12, 1, 7)])
def test_dissection_tree_separates_regions(dims):
    """Every subdomain is eliminated by one node; a node's region (its own
    subdomains and its descendants') is a box; its border is exactly the set of
    face neighbours of the region outside it; the subdomains of different
    children are never face neighbours (the separator splits them); leaves hold
    at most eight subdomains and children sit one level below their parent."""
    mx, my, mz = dims
    m = mx * my * mz
    T = B.test3d_dissection(mx, my, mz)
    nn = len(T["parent"])
    assert np.all(T["elim"] >= 0) and np.all(T["elim"] < nn)
    assert np.sum(T["parent"] == -1) == 1 and T["parent"][-1] == -1   # post-order: root last
    coords = lambda s: (s % mx, (s // mx) % my, s // (mx * my))  # noqa: E731

    def nbrs(s):
        x, y, z = coords(s)
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            q = (x + d[0], y + d[1], z + d[2])
            if 0 <= q[0] < mx and 0 <= q[1] < my and 0 <= q[2] < mz:
                yield (q[2] * my + q[1]) * mx + q[0]

    region = [set() for _ in range(nn)]
    for s in range(m):
        t = T["elim"][s]
        while t >= 0:
            region[t].add(s)
            t = T["parent"][t]
    assert region[-1] == set(range(m))
    children = [[] for _ in range(nn)]
    for t in range(nn):
        if T["parent"][t] >= 0:
            assert T["parent"][t] > t
            assert T["depth"][t] == T["depth"][T["parent"][t]] + 1
            children[T["parent"][t]].append(t)
    for t in range(nn):
        cs = np.array([coords(s) for s in region[t]])
        assert len(region[t]) == np.prod(cs.max(0) - cs.min(0) + 1)   # a box
        border = {q for s in region[t] for q in nbrs(s)} - region[t]
        assert sorted(border) == list(T["border"][t])
        own = {s for s in range(m) if T["elim"][s] == t}
        if not children[t]:
            assert len(own) <= 8 and own == region[t]
        for a in children[t]:
            for b in children[t]:
                if a < b:
                    assert not any(q in region[b] for s in region[a] for q in nbrs(s))


@pytest.mark.parametrize("case", CASES[1:4], ids=[f"{c[0]}x{c[1]}x{c[2]}-l{c[4]}-k{c[5]}" for c in CASES[1:4]])
def test_host_apply_fp32_storage(case):
    """Precision 2 rounds the plane blocks to FP32 after the FP64 set-up: T
    moves off the FP64 operator by at most the recurrence bound
    (k + 1)(2 planes + P) 2^-24 and by more than FP64 rounding."""
    nx, ny, nz, s, l, k, bc = case
    n = nx * ny * nz
    K = _field(n, 3)
    r = np.random.Generator(np.random.PCG64(7)).standard_normal(n)
    if not any(bc):
        r -= r.mean()
    mr = M3.MRCM3D(K, nx, ny, nz, bc, *s, l, 10.0, "H", k, 2, 1)
    z_ref = mr.apply(r)
    z, _ = B.test3d_host_apply(B.Config3(nx, ny, nz, bc, *s, l, 10.0, 0, k, 2, 1, 2), K, r)
    err = np.linalg.norm(z - z_ref) / np.linalg.norm(z_ref)
    assert 1e-12 < err <= mixed_t_gate3(mr)


def test_fp32_arithmetic_not_offered_in_3d():
    n = 8 * 8 * 8
    with pytest.raises(B.MrcmError) as e:
        B.test3d_host_apply(B.Config3(8, 8, 8, (1,) * 6, 4, 4, 4, 0, 10.0, 0, 0, 2, 1, 1),
                            _field(n, 4), np.zeros(n))
    assert e.value.code == B.MRCM_EINVAL
