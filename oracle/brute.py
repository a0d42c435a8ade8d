"""Brute-force companions that pin the oracle on tiny grids (test-only).

* ``rt0_vertex_quadrature_system`` builds the mixed RT0 / P0 system of
  Section 3 from the basis functions themselves (vertex quadrature of the mass
  term, exact divergence) and condenses the velocity densely.
* ``monolithic_mrcm`` solves the MRCM-O equations (11)-(14) with all local
  pressures and all multiplier coefficients as unknowns of one sparse system,
  without multiscale basis functions (the multiplier of subdomain i is
  phi_{i,r} + sum_k x_{i,k} phi_{i,k}, phi_{i,r} the trace of its source-driven
  oversampled solution).
* ``dense_operator`` applies an operator to every unit vector.
* ``krylov_lstsq_residuals`` computes GMRES residuals from an explicit Krylov
  basis and a dense least-squares solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .partition import edge_sides


def rt0_vertex_quadrature_system(K, nx: int, ny: int, bc, h: float,
                                 f_cells=None, g_sides=None):
    """Condensed matrix and right-hand side of the lumped RT0 mixed system.

    Velocity dofs are total face fluxes with a global orientation (+x for
    x-faces, +y for y-faces).  In a cell [xa, xa+h] x [ya, ya+h] the basis of
    its west x-face is ((xa + h - x) / h^2, 0) and of its east x-face
    ((x - xa) / h^2, 0) (flux 1 through their face), likewise in y.  The mass
    term int K^-1 phi_a . phi_b is evaluated with the four-corner rule (weight
    h^2 / 4 each); int div phi = +1 on the cell the face leaves, -1 on the cell
    it enters.  No-flow boundary faces carry no dof.  The mixed equations
    M U - B^T p = -G, B U = F condense to (B M^-1 B^T) p = F + B M^-1 G.
    """
    K = np.asarray(K, dtype=np.float64).reshape(ny, nx)
    W_, E_, S_, N_ = 0, 1, 2, 3
    faces = []  # (kind, i, j): x-face at x=i*h for row j, or y-face at y=j*h for column i
    for j in range(ny):
        for i in range(nx + 1):
            if (i == 0 and not bc[W_]) or (i == nx and not bc[E_]):
                continue
            faces.append((0, i, j))
    for j in range(ny + 1):
        for i in range(nx):
            if (j == 0 and not bc[S_]) or (j == ny and not bc[N_]):
                continue
            faces.append((1, i, j))
    fid = {f: k for k, f in enumerate(faces)}
    nf = len(faces)
    n = nx * ny
    M = np.zeros((nf, nf))
    B = np.zeros((n, nf))
    corners = [(0.0, 0.0), (1.0, 0.0), (0.0, 1.0), (1.0, 1.0)]  # in units of h
    for cy in range(ny):
        for cx in range(nx):
            c = cy * nx + cx
            # local basis: (face key, component, velocity at local coords (s, t) in [0,1]^2)
            loc = []
            for (key, comp, fn) in (((0, cx, cy), 0, lambda s, t: (1.0 - s) / h),
                                    ((0, cx + 1, cy), 0, lambda s, t: s / h),
                                    ((1, cx, cy), 1, lambda s, t: (1.0 - t) / h),
                                    ((1, cx, cy + 1), 1, lambda s, t: t / h)):
                if key in fid:
                    loc.append((fid[key], comp, fn))
            for (a, ca, fa) in loc:
                for (b, cb, fb) in loc:
                    if ca != cb:
                        continue
                    val = 0.0
                    for (s, t) in corners:
                        val += (h * h / 4.0) * fa(s, t) * fb(s, t) / K[cy, cx]
                    M[a, b] += val
            for (key, sign) in (((0, cx, cy), -1.0), ((0, cx + 1, cy), 1.0),
                                ((1, cx, cy), -1.0), ((1, cx, cy + 1), 1.0)):
                if key in fid:
                    B[c, fid[key]] += sign
    G = np.zeros(nf)
    g_sides = g_sides or {}
    for (kind, i, j), k in fid.items():
        if kind == 0 and i == 0 and W_ in g_sides:
            G[k] = g_sides[W_][j] * (-1.0)
        if kind == 0 and i == nx and E_ in g_sides:
            G[k] = g_sides[E_][j] * (1.0)
        if kind == 1 and j == 0 and S_ in g_sides:
            G[k] = g_sides[S_][i] * (-1.0)
        if kind == 1 and j == ny and N_ in g_sides:
            G[k] = g_sides[N_][i] * (1.0)
    Minv = np.linalg.inv(M)
    A = B @ Minv @ B.T
    F = np.zeros(n) if f_cells is None else np.asarray(f_cells, dtype=np.float64).ravel() * h * h
    b = F + B @ Minv @ G
    return A, b


def monolithic_mrcm(mr, r: np.ndarray) -> np.ndarray:
    """Solve the MRCM-O system directly: unknowns are every local pressure of
    every subdomain followed by every multiplier coefficient x_{i,k}; the
    Robin data on Gamma_i is lambda_i = phi_{i,r} + sum_k x_{i,k} phi_{i,k};
    equations are the local Robin problems on Omega_i with source r, then the
    flux rows and pressure rows of every edge (with the same no-flow row
    replacement as the coarse system).  Face traces: U = rho (p_c - lambda),
    pi = lambda + b U."""
    P = mr.part
    lam0 = mr.source_multiplier(r)
    offs = [0]
    cellsets = []
    for i in range(P.m):
        cells = mr.box_cells(P.boxes[i])
        cellsets.append(cells)
        offs.append(offs[-1] + cells.size)
    nloc = offs[-1]
    nc = P.nc
    ntot = nloc + nc
    M = sp.lil_matrix((ntot, ntot))
    rhs = np.zeros(ntot)
    for i in range(P.m):
        Ai = mr.box_matrix(P.boxes[i], robin=True).tolil()
        if mr._is_whole_noflow(P.boxes[i]):
            Ai[0, :] = 0.0
            Ai[:, 0] = 0.0
            Ai[0, 0] = 1.0
        o = offs[i]
        Ai = Ai.tocoo()
        for a, b, v in zip(Ai.row, Ai.col, Ai.data):
            M[o + a, o + b] += v
        rhs[o:o + cellsets[i].size] = r[cellsets[i]]
        loc = {int(c): j for j, c in enumerate(cellsets[i])}
        for g in mr.gamma[i]:
            for c, rho, l0 in zip(g.inside, g.rho, lam0[i][g.side]):
                rhs[o + loc[int(c)]] += rho * l0
        if mr._is_whole_noflow(P.boxes[i]):
            rhs[o] = 0.0
        for k, phi_k in enumerate(mr.phi[i]):
            col = nloc + P.dof_offset[i] + k
            for g in mr.gamma[i]:
                for c, rho, ph in zip(g.inside, g.rho, phi_k[g.side]):
                    M[o + loc[int(c)], col] -= rho * ph
    for e, (L, R, ori, st, ln) in enumerate(P.edges):
        sL, sR = edge_sides(int(ori))
        from .mrcm import side_basis
        Bq = side_basis(int(ln), mr.degree)
        nb = Bq.shape[0]
        r0 = nloc + int(mr.row_offset[e])
        for (sub, sd, sign) in ((int(L), sL, 1.0), (int(R), sR, -1.0)):
            g = mr._gamma_of(sub, sd)
            loc = {int(c): j for j, c in enumerate(cellsets[sub])}
            for jf, c in enumerate(g.inside):
                pc_col = offs[sub] + loc[int(c)]
                l0 = lam0[sub][sd][jf]
                for q in range(nb):
                    w = Bq[q, jf]
                    M[r0 + q, pc_col] += w * g.rho[jf]
                    M[r0 + nb + q, pc_col] += sign * w * g.b[jf] * g.rho[jf]
                    # the known part phi_{i,r} of lambda moves to the right-hand side
                    rhs[r0 + q] -= -w * g.rho[jf] * l0
                    rhs[r0 + nb + q] -= sign * w * (l0 - g.b[jf] * g.rho[jf] * l0)
                    for k, phi_k in enumerate(mr.phi[sub]):
                        col = nloc + P.dof_offset[sub] + k
                        lam = phi_k[sd][jf]
                        M[r0 + q, col] += -w * g.rho[jf] * lam
                        M[r0 + nb + q, col] += sign * w * (lam - g.b[jf] * g.rho[jf] * lam)
    if mr.pin_row >= 0:
        row = nloc + mr.pin_row
        M[row, :] = 0.0
        pin_col = nloc + int(np.flatnonzero(mr.C[mr.pin_row, :].toarray().ravel())[0])
        M[row, pin_col] = 1.0
        rhs[row] = 0.0
    sol = spla.splu(sp.csc_matrix(M)).solve(rhs)
    p = np.zeros(mr.nx * mr.ny)
    for i in range(P.m):
        p[cellsets[i]] = sol[offs[i]:offs[i + 1]]
    return p


def dense_operator(apply, n: int) -> np.ndarray:
    out = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        out[:, j] = apply(e)
    return out


def krylov_lstsq_residuals(A: np.ndarray, T: np.ndarray, b: np.ndarray, steps: int):
    """Relative residual of min ||b - A T y|| over y in span{b, ATb, ...}."""
    AT = A @ T
    basis = [b / np.linalg.norm(b)]
    out = []
    for j in range(steps):
        Kj = np.array(basis).T
        # orthonormal columns via SVD of the monomial basis (a dense library step)
        U, s, _ = np.linalg.svd(Kj, full_matrices=False)
        Q = U[:, s > s[0] * 1e-13]
        y, *_ = np.linalg.lstsq(AT @ Q, b, rcond=None)
        out.append(np.linalg.norm(b - AT @ Q @ y) / np.linalg.norm(b))
        nxt = AT @ basis[-1]
        basis.append(nxt / np.linalg.norm(nxt))
    return out
