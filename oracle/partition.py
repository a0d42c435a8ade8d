"""Decomposition geometry and index maps.

Section 2.1 of the paper: the Cartesian mesh is split into non-overlapping
subdomains Omega_i; Gamma_i is the part of the boundary of Omega_i that is not
on the domain boundary; hat-Omega_i is Omega_i enlarged by an adjoining region
(oversampling by l cells, the "lh" of Table 1) and never leaves the domain.
The smoothing patches (Section 1, overlapping Schwarz; Section 2.1, smoothing
"for a predetermined number of iterations") are Omega_i enlarged by delta
cells and clipped at the domain boundary.

Conventions (all integer, reproduced bit for bit by the library):

* subdomain (I, J) has id i = J * mx + I and box [I sx, min(nx,(I+1) sx)) x
  [J sy, min(ny,(J+1) sy)); when sx does not divide nx the last column is
  narrower (same for rows);
* boxes are stored as (x0, x1, y0, y1), half-open;
* interior sides of a box are listed in the order W, E, S, N;
* interior edges: all vertical edges first, row-major by (J, left I); then all
  horizontal edges, row-major by (lower J, I).  Each edge stores
  (L, R, orientation, start, length): L is the left/lower subdomain, R the
  right/upper one, orientation 0 for vertical and 1 for horizontal, start the
  first cell coordinate along the edge and length its number of faces;
* coarse dofs: for each subdomain, for each interior side (W, E, S, N order),
  for each basis function q: (i, side, q);
* coarse rows: for each edge, the flux rows F_{e,q} for every q, then the
  pressure rows P_{e,q} for every q.

``degree`` >= 0 selects Legendre polynomials P_0..P_degree per side
(reading of the multiplier and test spaces), capped at the number of faces of
the side; ``degree`` = -1 selects the test-only FULL space (one indicator per
face).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

W, E, S, N = 0, 1, 2, 3
FULL = -1


def subdomain_boxes(nx: int, ny: int, sx: int, sy: int) -> np.ndarray:
    mx = -(-nx // sx)
    my = -(-ny // sy)
    boxes = np.zeros((mx * my, 4), dtype=np.int32)
    for J in range(my):
        for I in range(mx):
            i = J * mx + I
            boxes[i] = (I * sx, min(nx, (I + 1) * sx), J * sy, min(ny, (J + 1) * sy))
    return boxes


def grown_boxes(boxes: np.ndarray, g: int, nx: int, ny: int) -> np.ndarray:
    """Each box enlarged by g cells on every side, clipped at the domain."""
    out = np.empty_like(boxes)
    for i, (x0, x1, y0, y1) in enumerate(boxes):
        out[i] = (max(0, x0 - g), min(nx, x1 + g), max(0, y0 - g), min(ny, y1 + g))
    return out


def interior_sides(box, nx: int, ny: int) -> list[int]:
    x0, x1, y0, y1 = (int(v) for v in box)
    sides = []
    if x0 > 0:
        sides.append(W)
    if x1 < nx:
        sides.append(E)
    if y0 > 0:
        sides.append(S)
    if y1 < ny:
        sides.append(N)
    return sides


def side_length(box, side: int) -> int:
    x0, x1, y0, y1 = (int(v) for v in box)
    return (y1 - y0) if side in (W, E) else (x1 - x0)


def nbasis(degree: int, length: int) -> int:
    """Functions per side: P_0..P_degree, but never more than the side has
    faces (Legendre values at n distinct points have rank n)."""
    return length if degree == FULL else min(degree + 1, length)


@dataclass
class Partition:
    nx: int
    ny: int
    sx: int
    sy: int
    oversample: int
    overlap: int
    degree: int
    mx: int = 0
    my: int = 0
    boxes: np.ndarray = field(default=None)
    oboxes: np.ndarray = field(default=None)
    pboxes: np.ndarray = field(default=None)
    owner: np.ndarray = field(default=None)
    sides: list = field(default=None)
    edges: np.ndarray = field(default=None)
    dof_table: np.ndarray = field(default=None)
    dof_offset: np.ndarray = field(default=None)
    row_table: np.ndarray = field(default=None)

    @property
    def m(self) -> int:
        return self.mx * self.my

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def nc(self) -> int:
        return int(self.dof_offset[-1])


def build_partition(nx: int, ny: int, sx: int, sy: int, oversample: int, overlap: int,
                    degree: int = 1) -> Partition:
    if min(nx, ny, sx, sy) < 1 or oversample < 0 or overlap < 0 or degree < FULL:
        raise ValueError("invalid partition parameters")
    P = Partition(nx, ny, sx, sy, oversample, overlap, degree)
    P.mx = -(-nx // sx)
    P.my = -(-ny // sy)
    P.boxes = subdomain_boxes(nx, ny, sx, sy)
    P.oboxes = grown_boxes(P.boxes, oversample, nx, ny)
    P.pboxes = grown_boxes(P.boxes, overlap, nx, ny)
    owner = np.empty(nx * ny, dtype=np.int32)
    for i, (x0, x1, y0, y1) in enumerate(P.boxes):
        for iy in range(y0, y1):
            owner[iy * nx + x0: iy * nx + x1] = i
    P.owner = owner
    P.sides = [interior_sides(b, nx, ny) for b in P.boxes]
    # The Robin sides of the oversampled region must be exactly the interior
    # sides of the subdomain (an oversampled side that reaches the domain
    # boundary would change the number of multipliers).
    for i in range(P.m):
        if interior_sides(P.oboxes[i], nx, ny) != P.sides[i]:
            raise ValueError("oversampling reaches the domain boundary across an interior side")
        if degree == FULL and oversample != 0:
            raise ValueError("the FULL interface space is defined for oversample 0 only")
    edges = []
    for J in range(P.my):
        for I in range(P.mx - 1):
            L = J * P.mx + I
            y0, y1 = P.boxes[L][2], P.boxes[L][3]
            edges.append((L, L + 1, 0, y0, y1 - y0))
    for J in range(P.my - 1):
        for I in range(P.mx):
            L = J * P.mx + I
            x0, x1 = P.boxes[L][0], P.boxes[L][1]
            edges.append((L, L + P.mx, 1, x0, x1 - x0))
    P.edges = np.array(edges, dtype=np.int32).reshape(-1, 5)
    dofs = []
    offs = [0]
    for i in range(P.m):
        for s in P.sides[i]:
            for q in range(nbasis(degree, side_length(P.boxes[i], s))):
                dofs.append((i, s, q))
        offs.append(len(dofs))
    P.dof_table = np.array(dofs, dtype=np.int32).reshape(-1, 3)
    P.dof_offset = np.array(offs, dtype=np.int32)
    rows = []
    for e, (L, R, o, st, ln) in enumerate(P.edges):
        nb = nbasis(degree, int(ln))
        for kind in (0, 1):
            for q in range(nb):
                rows.append((e, kind, q))
    P.row_table = np.array(rows, dtype=np.int32).reshape(-1, 3)
    if len(rows) != len(dofs):
        raise AssertionError("coarse system is not square")
    return P


def side_faces(box, side: int, nx: int):
    """Faces of one side of a box in increasing coordinate.

    Returns a list of (inside cell, outside cell, face kind, face row, face col)
    where kind 0 is an x-face stored at tx[row, col] and kind 1 a y-face at
    ty[row, col].  Outside cell ids refer to the global grid (they may lie
    outside the domain only for boundary sides, which callers never ask for).
    """
    x0, x1, y0, y1 = (int(v) for v in box)
    out = []
    if side == W:
        for y in range(y0, y1):
            out.append((y * nx + x0, y * nx + x0 - 1, 0, y, x0))
    elif side == E:
        for y in range(y0, y1):
            out.append((y * nx + x1 - 1, y * nx + x1, 0, y, x1))
    elif side == S:
        for x in range(x0, x1):
            out.append((y0 * nx + x, (y0 - 1) * nx + x, 1, y0, x))
    else:
        for x in range(x0, x1):
            out.append(((y1 - 1) * nx + x, y1 * nx + x, 1, y1, x))
    return out


def edge_sides(orientation: int) -> tuple[int, int]:
    """Side of L and side of R that an edge lies on."""
    return (E, W) if orientation == 0 else (N, S)
