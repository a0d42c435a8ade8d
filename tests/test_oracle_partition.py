"""Pins of the decomposition maps (oracle.partition): closed-form counts and
invariants of Omega_i, hat-Omega_i, the smoothing patches, the interior edges
and the coarse dofs / rows (Section 2.1)."""
import numpy as np
import pytest

from oracle.partition import FULL, build_partition

CASES = [(64, 64, 16, 16, 2, 2, 1), (220, 60, 20, 20, 4, 2, 1), (52, 39, 12, 12, 2, 3, 0),
         (40, 24, 8, 8, 0, 2, 2), (16, 16, 16, 16, 0, 2, 1), (34, 17, 8, 5, 1, 1, 1),
         (22, 18, 7, 7, 0, 2, 2)]


@pytest.mark.parametrize("nx,ny,sx,sy,l,d,deg", CASES)
def test_counts_and_invariants(nx, ny, sx, sy, l, d, deg):
    P = build_partition(nx, ny, sx, sy, l, d, deg)
    mx, my = -(-nx // sx), -(-ny // sy)
    assert (P.mx, P.my, P.m) == (mx, my, mx * my)
    E = my * (mx - 1) + mx * (my - 1)
    assert len(P.edges) == E
    assert P.nc == 2 * sum(min(deg + 1, int(e[4])) for e in P.edges)
    assert P.nc == len(P.row_table) == int(P.dof_offset[-1])
    # ownership is a partition: every cell owned by the box containing it
    counts = np.bincount(P.owner, minlength=P.m)
    for i, (x0, x1, y0, y1) in enumerate(P.boxes):
        assert counts[i] == (x1 - x0) * (y1 - y0)
        assert np.all(P.owner.reshape(ny, nx)[y0:y1, x0:x1] == i)
    assert counts.sum() == nx * ny
    for B, g in ((P.oboxes, l), (P.pboxes, d)):
        for (x0, x1, y0, y1), (X0, X1, Y0, Y1) in zip(P.boxes, B):
            assert (X0, X1, Y0, Y1) == (max(0, x0 - g), min(nx, x1 + g), max(0, y0 - g),
                                        min(ny, y1 + g))
    # each subdomain: min(d+1, side faces) dofs per interior side
    for i in range(P.m):
        x0, x1, y0, y1 = P.boxes[i]
        lens = [(y1 - y0) if s in (0, 1) else (x1 - x0) for s in P.sides[i]]
        assert P.dof_offset[i + 1] - P.dof_offset[i] == sum(min(deg + 1, n) for n in lens)
    for (L, R, o, st, ln) in P.edges:
        bL, bR = P.boxes[L], P.boxes[R]
        if o == 0:
            assert R == L + 1 and bL[1] == bR[0] and (bL[2], bL[3]) == (bR[2], bR[3])
            assert (st, ln) == (bL[2], bL[3] - bL[2])
        else:
            assert R == L + P.mx and bL[3] == bR[2] and (bL[0], bL[1]) == (bR[0], bR[1])
            assert (st, ln) == (bL[0], bL[1] - bL[0])


def test_edge_order_vertical_first_row_major():
    P = build_partition(48, 32, 16, 16, 0, 2, 1)  # 3 x 2 subdomains
    assert [tuple(e[:3]) for e in P.edges] == [(0, 1, 0), (1, 2, 0), (3, 4, 0), (4, 5, 0),
                                               (0, 3, 1), (1, 4, 1), (2, 5, 1)]


def test_oversampling_must_not_reach_the_boundary_across_an_interior_side():
    with pytest.raises(ValueError):
        build_partition(50, 37, 12, 12, 3, 2, 1)  # last column 2 cells wide


def test_full_space_counts():
    P = build_partition(24, 16, 8, 8, 0, 2, FULL)
    assert P.nc == 2 * sum(int(e[4]) for e in P.edges)
