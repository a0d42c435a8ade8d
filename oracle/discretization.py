"""Fine-scale system A p = b on a Cartesian grid of square cells.

Section 3 of the paper discretises eqs. (1a)-(1d) with lowest-order
Raviart-Thomas velocity / piecewise-constant pressure and statically condenses
the velocity to reach an SPD pressure system A p = b.  Reading used here: the
velocity mass matrix is integrated with the trapezoidal (vertex) rule, which
makes it diagonal on rectangles, so condensation is local and gives the
cell-centred five-point two-point-flux stencil with harmonic-mean face
permeability.  ``oracle.brute.rt0_vertex_quadrature_system`` builds the mixed
system from the RT0 basis functions themselves and condenses it densely; the
test suite checks that both agree.

Square cells (side h) make A independent of h: a face of length h between
centres a distance h apart has transmissibility K_H (harmonic mean).  A
Dirichlet face has the half-cell transmissibility 2 K_c.  Only b carries h:
the cell source integrates to f h^2.

Sides: W=0 (x=0), E=1 (x=1), S=2 (y=0), N=3 (y=top).  ``bc[side]`` is 0 for
no-flow (u.n = 0) and 1 for Dirichlet (p = g).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

W, E, S, N = 0, 1, 2, 3


def face_transmissibilities(K: np.ndarray, nx: int, ny: int, bc) -> tuple[np.ndarray, np.ndarray]:
    """x-face and y-face transmissibilities, shapes (ny, nx+1) and (ny+1, nx).

    Interior face: harmonic mean 2 K_c K_c' / (K_c + K_c').  Boundary face:
    2 K_c when Dirichlet, 0 when no-flow.
    """
    K = np.asarray(K, dtype=np.float64).reshape(ny, nx)
    tx = np.zeros((ny, nx + 1))
    ty = np.zeros((ny + 1, nx))
    tx[:, 1:nx] = 2.0 * K[:, :-1] * K[:, 1:] / (K[:, :-1] + K[:, 1:])
    ty[1:ny, :] = 2.0 * K[:-1, :] * K[1:, :] / (K[:-1, :] + K[1:, :])
    if bc[W]:
        tx[:, 0] = 2.0 * K[:, 0]
    if bc[E]:
        tx[:, nx] = 2.0 * K[:, nx - 1]
    if bc[S]:
        ty[0, :] = 2.0 * K[0, :]
    if bc[N]:
        ty[ny, :] = 2.0 * K[ny - 1, :]
    return tx, ty


def assemble(K: np.ndarray, nx: int, ny: int, bc) -> sp.csr_matrix:
    """Global matrix A: A_cc = sum of the cell's face transmissibilities,
    A_cc' = -t_f for the interior face shared by c and c'."""
    tx, ty = face_transmissibilities(K, nx, ny, bc)
    n = nx * ny
    diag = np.zeros((ny, nx))
    diag += tx[:, :nx] + tx[:, 1:]
    diag += ty[:ny, :] + ty[1:, :]
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [diag.ravel()]
    ids = np.arange(n).reshape(ny, nx)
    # interior x-faces: between (ix-1, iy) and (ix, iy)
    a = ids[:, :-1].ravel()
    b = ids[:, 1:].ravel()
    t = tx[:, 1:nx].ravel()
    rows += [a, b]
    cols += [b, a]
    vals += [-t, -t]
    # interior y-faces: between (ix, iy-1) and (ix, iy)
    a = ids[:-1, :].ravel()
    b = ids[1:, :].ravel()
    t = ty[1:ny, :].ravel()
    rows += [a, b]
    cols += [b, a]
    vals += [-t, -t]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()


def rhs(K: np.ndarray, nx: int, ny: int, bc, f_cells: np.ndarray | None,
        g_sides: dict | None, h: float) -> np.ndarray:
    """b = f h^2 + 2 K_c g_f on every Dirichlet face.

    ``g_sides[side]`` holds the Dirichlet values at the face midpoints of that
    side in increasing coordinate order (length ny for W/E, nx for S/N).
    """
    K = np.asarray(K, dtype=np.float64).reshape(ny, nx)
    b = np.zeros((ny, nx))
    if f_cells is not None:
        b += np.asarray(f_cells, dtype=np.float64).reshape(ny, nx) * h * h
    g_sides = g_sides or {}
    if bc[W] and W in g_sides:
        b[:, 0] += 2.0 * K[:, 0] * g_sides[W]
    if bc[E] and E in g_sides:
        b[:, nx - 1] += 2.0 * K[:, nx - 1] * g_sides[E]
    if bc[S] and S in g_sides:
        b[0, :] += 2.0 * K[0, :] * g_sides[S]
    if bc[N] and N in g_sides:
        b[ny - 1, :] += 2.0 * K[ny - 1, :] * g_sides[N]
    return b.ravel()


def all_noflow(bc) -> bool:
    return not any(bc)


def direct_solve(A: sp.spmatrix, b: np.ndarray, bc) -> np.ndarray:
    """Sparse direct solve of A p = b.

    With no-flow on every side A is singular with null space span(1) and the
    pressure is fixed by its mean: pin p_0 = 0, solve the rest, then subtract
    the mean.
    """
    A = sp.csc_matrix(A)
    if all_noflow(bc):
        p = np.zeros(A.shape[0])
        if A.shape[0] > 1:
            p[1:] = spla.splu(A[1:, 1:].tocsc()).solve(b[1:])
        return p - p.mean()
    return spla.splu(A).solve(b)
