"""The MRCM-OS preconditioner T (oracle).

Paper passages followed:

* Section 2.1, eqs. (11)-(14): local Robin problems on Omega_i coupled by weak
  flux continuity (13) and weak pressure continuity (14) on the interfaces.
* Section 2.1, the Robin condition -beta_i u.n_i + p = g_R and
  beta_i = alpha H / K_H with K_H the harmonic mean of the neighbouring K.
* Section 2.1, the informed multiplier spaces Lambda^i_H spanned by
  phi_i^k = -beta_i u^k.n_i + pi^k on Gamma_i, with (u^k, p^k) the solution of
  the zero-source oversampled problem on hat-Omega_i whose Robin data on the
  part of its boundary inside the domain is lambda^k.
* Section 2.1, the four-step MRCM-OS algorithm: decomposition and oversampling
  size; multiplier spaces from the oversampled problems; solve (11)-(14) with
  multiscale basis functions; a fixed number of smoothing steps.
* Section 3, the modified MRCM-O used as preconditioner: homogeneous boundary
  conditions and source r (the current Krylov vector); T r is the resulting
  pressure.
* Section 2.1, oversampling builds every multiscale basis function on the
  extended region while the compatibility conditions stay on the
  non-overlapping interfaces.  Reading: this includes the source-driven basis
  function.  The local solution on Omega_i is the restriction of the solution
  on hat-Omega_i with source r and Robin data sum_k x_k lambda^k on the part of
  its boundary inside the domain; on Gamma_i its Robin trace is phi_{i,r} +
  sum_k x_k phi_i^k, where phi_{i,r} is the trace of the zero-data oversampled
  solution with source r.  Without oversampling (l = 0) this is the plain MRCM
  particular solution with zero multiplier.

Discrete readings (all plain statements of how a face-based quantity is
evaluated on the lumped RT0 / two-point-flux discretisation; see
``oracle.discretization``):

* Robin face f of a cell set, inside cell c: with b_f = beta_f / h =
  alpha * L_cells / K_H(f) (L_cells = subdomain side in cells for L = H, or 1
  for L = h), the total outward face flux for Robin data lambda_f is
  U_f = rho_f (p_c - lambda_f) with rho_f = 1 / (1 / (2 K_c) + b_f), and the
  face pressure is pi_f = lambda_f + b_f U_f.
* Face interior to a solve region: U_f = t_f (p_c - p_c') and the
  flux-continuous face pressure pi_f = (K_c p_c + K_c' p_c') / (K_c + K_c').
* Multiplier and test functions on a side with n faces: Legendre P_q at the
  face parameters xi_j = (2 j + 1) / n - 1, q = 0..degree (``degree`` = -1:
  one indicator per face, test-only).
* Smoothing: restricted additive Schwarz.  Each sweep computes the residual
  rho = r - A p, solves on every patch S_i (Omega_i grown by delta and clipped)
  with the principal submatrix A[S_i] (zero Dirichlet data at the neighbouring
  cell centres), and adds the solution restricted to Omega_i.
* The interface system is solved by sparse LU followed by iterative
  refinement whose residuals g - C x are formed in extended precision
  (numpy.longdouble), so the oracle's interface solution is accurate to
  about the FP64 rounding of the exact one even where C is ill-conditioned.
* No-flow on all sides: the coarse system has a one-dimensional null space
  (a uniform pressure shift) and its constant-mode flux rows sum to the total
  source; the flux row F_{e0,0} of the first edge is replaced by a unit row on
  the dof (L(e0), side of L(e0) facing e0, q = 0), and T's output is projected
  to zero mean.  A local problem with neither Robin nor Dirichlet faces (one
  subdomain covering the grid) fixes its first cell to zero.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre

from .discretization import all_noflow, assemble, face_transmissibilities
from .partition import FULL, W, E, S, N, build_partition, edge_sides, nbasis, side_faces


def side_basis(n: int, degree: int) -> np.ndarray:
    """Side functions evaluated at the n face midpoints, shape (nbasis, n)."""
    if degree == FULL:
        return np.eye(n)
    nb = nbasis(degree, n)
    xi = (2.0 * np.arange(n) + 1.0) / n - 1.0
    return np.array([legendre.legval(xi, np.eye(nb)[q]) for q in range(nb)])


class BoxSolver:
    """Sparse direct solver of one local matrix (library LU as the step)."""

    def __init__(self, A: sp.spmatrix, pin: bool):
        A = sp.lil_matrix(A)
        if pin:
            A[0, :] = 0.0
            A[:, 0] = 0.0
            A[0, 0] = 1.0
        self.pin = pin
        self.lu = spla.splu(sp.csc_matrix(A))

    def solve(self, rhs: np.ndarray) -> np.ndarray:
        rhs = np.array(rhs, dtype=np.float64)
        if self.pin:
            rhs[0] = 0.0
        return self.lu.solve(rhs)


class SideFaces:
    """Faces of one side of a cell box, with the data the traces need."""

    def __init__(self, mr: "MRCM", box, side: int):
        faces = side_faces(box, side, mr.nx)
        self.side = side
        self.inside = np.array([f[0] for f in faces], dtype=np.int64)
        self.outside = np.array([f[1] for f in faces], dtype=np.int64)
        self.t = np.array([mr.tx[f[3], f[4]] if f[2] == 0 else mr.ty[f[3], f[4]] for f in faces])
        self.K_in = mr.K[self.inside]
        self.K_out = mr.K[self.outside]
        self.b = mr.alpha * mr.L_cells / self.t
        self.rho = 1.0 / (1.0 / (2.0 * self.K_in) + self.b)


class MRCM:
    """Setup and application of T for one permeability field."""

    def __init__(self, K, nx: int, ny: int, bc, sx: int, sy: int, oversample: int,
                 alpha: float, beta_len: str = "H", sweeps: int = 0, overlap: int = 2,
                 degree: int = 1, pin_edge: int = 0, schwarz: str = "additive"):
        self.K = np.asarray(K, dtype=np.float64).ravel()
        if self.K.size != nx * ny or not np.all(np.isfinite(self.K)) or np.any(self.K <= 0):
            raise ValueError("K must be finite and positive on every cell")
        self.nx, self.ny, self.bc = nx, ny, tuple(int(v) for v in bc)
        self.alpha = float(alpha)
        self.L_cells = float(max(sx, sy)) if beta_len == "H" else 1.0
        self.sweeps, self.overlap, self.degree = int(sweeps), int(overlap), int(degree)
        self.pin_edge = int(pin_edge)
        if schwarz not in ("additive", "multiplicative"):
            raise ValueError("schwarz must be 'additive' or 'multiplicative'")
        self.schwarz = schwarz
        self.part = build_partition(nx, ny, sx, sy, oversample, overlap, degree)
        self.tx, self.ty = face_transmissibilities(self.K, nx, ny, self.bc)
        self.A = assemble(self.K, nx, ny, self.bc)
        self.noflow = all_noflow(self.bc)
        self.ids = np.arange(nx * ny).reshape(ny, nx)
        P = self.part
        self.gamma = [[SideFaces(self, P.boxes[i], s) for s in P.sides[i]] for i in range(P.m)]
        self.local = [self._box_solver(P.boxes[i], robin=True) for i in range(P.m)]
        self.over = [self._box_solver(P.oboxes[i], robin=True) for i in range(P.m)]
        self.ocells = [self.box_cells(P.oboxes[i]) for i in range(P.m)]
        self.oloc = [{int(c): j for j, c in enumerate(oc)} for oc in self.ocells]
        self.phi = [self._informed_space(i) for i in range(P.m)]
        self.mbf = []
        self.mbf_U = []
        self.mbf_pi = []
        for i in range(P.m):
            Pi, Ui, pii = self._mbfs(i)
            self.mbf.append(Pi)
            self.mbf_U.append(Ui)
            self.mbf_pi.append(pii)
        self.patch = [self._box_solver(P.pboxes[i], robin=False) for i in range(P.m)] \
            if self.sweeps > 0 else []
        self._coarse_assemble()

    # ---- local operators -------------------------------------------------
    def box_cells(self, box) -> np.ndarray:
        x0, x1, y0, y1 = (int(v) for v in box)
        return self.ids[y0:y1, x0:x1].ravel()

    def box_matrix(self, box, robin: bool) -> sp.csc_matrix:
        """Local matrix on a cell box.  Faces inside the box couple as in A;
        faces on the domain boundary keep the global boundary condition
        (homogeneous data); faces leaving the box inside the domain carry the
        Robin conductance rho_f (robin=True) or keep t_f on the diagonal with
        zero data beyond (robin=False, i.e. the principal submatrix of A)."""
        x0, x1, y0, y1 = (int(v) for v in box)
        bx, by = x1 - x0, y1 - y0
        K = self.K.reshape(self.ny, self.nx)[y0:y1, x0:x1]
        tW = self.tx[y0:y1, x0:x1].copy()
        tE = self.tx[y0:y1, x0 + 1:x1 + 1].copy()
        tS = self.ty[y0:y1, x0:x1].copy()
        tN = self.ty[y0 + 1:y1 + 1, x0:x1].copy()
        diag = np.zeros((by, bx))
        if robin:
            def rho(Kc, t):
                return 1.0 / (1.0 / (2.0 * Kc) + self.alpha * self.L_cells / t)
            if x0 > 0:
                tW[:, 0] = rho(K[:, 0], tW[:, 0])
            if x1 < self.nx:
                tE[:, -1] = rho(K[:, -1], tE[:, -1])
            if y0 > 0:
                tS[0, :] = rho(K[0, :], tS[0, :])
            if y1 < self.ny:
                tN[-1, :] = rho(K[-1, :], tN[-1, :])
        diag += tW + tE + tS + tN
        loc = np.arange(bx * by).reshape(by, bx)
        rows = [loc.ravel()]
        cols = [loc.ravel()]
        vals = [diag.ravel()]
        a, b, t = loc[:, :-1].ravel(), loc[:, 1:].ravel(), tW[:, 1:].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
        a, b, t = loc[:-1, :].ravel(), loc[1:, :].ravel(), tS[1:, :].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
        return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(bx * by, bx * by))

    def _is_whole_noflow(self, box) -> bool:
        x0, x1, y0, y1 = (int(v) for v in box)
        return self.noflow and x0 == 0 and y0 == 0 and x1 == self.nx and y1 == self.ny

    def _box_solver(self, box, robin: bool) -> BoxSolver:
        return BoxSolver(self.box_matrix(box, robin), pin=self._is_whole_noflow(box))

    # ---- informed multiplier spaces (setup) ------------------------------
    def coarse_functions(self, i: int):
        """(side, q) pairs of subdomain i's coarse dofs in dof-table order."""
        P = self.part
        lo, hi = P.dof_offset[i], P.dof_offset[i + 1]
        return [(int(s), int(q)) for (_, s, q) in P.dof_table[lo:hi]]

    def oversampled_traces(self, i: int, ph: np.ndarray, lam=None):
        """Flux U and pressure pi of an oversampled solution ph (values on the
        cells of hat-Omega_i) across every face of Gamma_i, per side.

        With l = 0 the faces of Gamma_i are Robin faces of hat-Omega_i = Omega_i
        and ``lam`` (side -> Robin data on those faces, absent = 0) enters:
        U = rho (p_c - lambda), pi = lambda + b U.  With l > 0 the faces are
        inside hat-Omega_i: U = t (p_c - p_c') and the flux-continuous face
        pressure pi = (K_c p_c + K_c' p_c') / (K_c + K_c')."""
        oloc = self.oloc[i]
        out = {}
        for g in self.gamma[i]:
            pc = ph[[oloc[int(c)] for c in g.inside]]
            if self.part.oversample == 0:
                lam_f = lam[g.side] if lam is not None and g.side in lam else np.zeros(g.inside.size)
                U = g.rho * (pc - lam_f)
                pi = lam_f + g.b * U
            else:
                pn = ph[[oloc[int(c)] for c in g.outside]]
                U = g.t * (pc - pn)
                pi = (g.K_in * pc + g.K_out * pn) / (g.K_in + g.K_out)
            out[g.side] = (U, pi)
        return out

    def _informed_space(self, i: int):
        """phi_{i,k} on the faces of Gamma_i, one dict side -> values per k."""
        P = self.part
        obox = P.oboxes[i]
        oside = {s: SideFaces(self, obox, s) for s in P.sides[i]}
        phis = []
        for (s, q) in self.coarse_functions(i):
            sf = oside[s]
            lam = side_basis(sf.inside.size, self.degree)[q]
            rhs = np.zeros(self.ocells[i].size)
            np.add.at(rhs, [self.oloc[i][int(c)] for c in sf.inside], sf.rho * lam)
            ph = self.over[i].solve(rhs)
            tr = self.oversampled_traces(i, ph, {s: lam})
            phis.append({sd: pi - self._gamma_of(i, sd).b * U for sd, (U, pi) in tr.items()})
        return phis

    # ---- multiscale basis functions (setup) ------------------------------
    def _mbfs(self, i: int):
        cells = self.box_cells(self.part.boxes[i])
        loc = {int(c): j for j, c in enumerate(cells)}
        cols, Us, pis = [], [], []
        for phi_k in self.phi[i]:
            rhs = np.zeros(cells.size)
            for g in self.gamma[i]:
                np.add.at(rhs, [loc[int(c)] for c in g.inside], g.rho * phi_k[g.side])
            p = self.local[i].solve(rhs)
            U, pi = {}, {}
            for g in self.gamma[i]:
                pc = p[[loc[int(c)] for c in g.inside]]
                U[g.side] = g.rho * (pc - phi_k[g.side])
                pi[g.side] = phi_k[g.side] + g.b * U[g.side]
            cols.append(p)
            Us.append(U)
            pis.append(pi)
        Pi = np.array(cols).T if cols else np.zeros((cells.size, 0))
        return Pi, Us, pis

    # ---- coarse interface system (setup) ---------------------------------
    def _gamma_of(self, i: int, side: int) -> SideFaces:
        for g in self.gamma[i]:
            if g.side == side:
                return g
        raise KeyError(side)

    def _coarse_assemble(self):
        P = self.part
        nc = P.nc
        self.row_offset = np.zeros(len(P.edges) + 1, dtype=np.int64)
        for e, (L, R, o, st, ln) in enumerate(P.edges):
            nb = side_basis(int(ln), self.degree).shape[0]
            self.row_offset[e + 1] = self.row_offset[e] + 2 * nb
        C = sp.lil_matrix((nc, nc))
        for e, (L, R, o, st, ln) in enumerate(P.edges):
            sL, sR = edge_sides(int(o))
            B = side_basis(int(ln), self.degree)
            nb = B.shape[0]
            r0 = self.row_offset[e]
            for (sub, sd, sign) in ((int(L), sL, 1.0), (int(R), sR, -1.0)):
                for k in range(P.dof_offset[sub + 1] - P.dof_offset[sub]):
                    col = P.dof_offset[sub] + k
                    fU = B @ self.mbf_U[sub][k][sd]
                    fP = B @ self.mbf_pi[sub][k][sd]
                    for q in range(nb):
                        C[r0 + q, col] += fU[q]
                        C[r0 + nb + q, col] += sign * fP[q]
        self.pin_row = -1
        if self.noflow and len(P.edges) > 0:
            e0 = self.pin_edge
            L0, _, o0, _, _ = P.edges[e0]
            s0 = edge_sides(int(o0))[0]
            lo, hi = P.dof_offset[L0], P.dof_offset[L0 + 1]
            col = lo + [j for j, (s, q) in enumerate(self.coarse_functions(int(L0)))
                        if s == s0 and q == 0][0]
            self.pin_row = int(self.row_offset[e0])
            C[self.pin_row, :] = 0.0
            C[self.pin_row, col] = 1.0
        self.C = sp.csc_matrix(C)
        self.C_lu = spla.splu(self.C) if nc > 0 else None
        self.C_ext = sp.csr_matrix(self.C).astype(np.longdouble) if nc > 0 else None

    def coarse_solve(self, g: np.ndarray) -> np.ndarray:
        """x = C^-1 g: LU solve, then refinement steps x += C^-1 (g - C x) with
        the residual and the accumulated x in extended precision, until the
        correction stops changing x (at most ten steps)."""
        if self.part.nc == 0:
            return np.zeros(0)
        gl = np.asarray(g, dtype=np.longdouble)
        x = self.C_lu.solve(np.asarray(g, dtype=np.float64)).astype(np.longdouble)
        for _ in range(10):
            res = gl - self.C_ext @ x
            dx = self.C_lu.solve(np.asarray(res, dtype=np.float64))
            x = x + dx.astype(np.longdouble)
            if np.abs(dx).max() <= 1e-18 * float(np.abs(x).max()):
                break
        return np.asarray(x, dtype=np.float64)

    # ---- application of T (per Krylov step) ------------------------------
    def particular(self, r: np.ndarray):
        """Source-driven basis functions: the oversampled problem on hat-Omega_i
        with source r and zero Robin data, solved whole (values on the cells of
        hat-Omega_i).  Its restriction to Omega_i is the local particular
        solution p_{i,r}."""
        return [self.over[i].solve(r[self.ocells[i]]) for i in range(self.part.m)]

    def restrict(self, i: int, ph: np.ndarray) -> np.ndarray:
        """Values of an oversampled solution on the cells of Omega_i."""
        return ph[[self.oloc[i][int(c)] for c in self.box_cells(self.part.boxes[i])]]

    def source_multiplier(self, r: np.ndarray):
        """phi_{i,r}: the Robin trace -b U + pi on Gamma_i of the source-driven
        oversampled solution (zero for l = 0), per subdomain and side."""
        out = []
        for i, ph in enumerate(self.particular(r)):
            tr = self.oversampled_traces(i, ph)
            out.append({sd: pi - self._gamma_of(i, sd).b * U for sd, (U, pi) in tr.items()})
        return out

    def coarse_rhs(self, pover) -> np.ndarray:
        """g = minus the flux and pressure row functionals of the traces of the
        source-driven oversampled solutions."""
        P = self.part
        g = np.zeros(P.nc)
        traces = [self.oversampled_traces(i, pover[i]) for i in range(P.m)]
        for e, (L, R, o, st, ln) in enumerate(P.edges):
            sL, sR = edge_sides(int(o))
            B = side_basis(int(ln), self.degree)
            nb = B.shape[0]
            UL, piL = traces[int(L)][sL]
            UR, piR = traces[int(R)][sR]
            r0 = self.row_offset[e]
            g[r0:r0 + nb] = -(B @ (UL + UR))
            g[r0 + nb:r0 + 2 * nb] = -(B @ (piL - piR))
        if self.pin_row >= 0:
            g[self.pin_row] = 0.0
        return g

    def mrcm_solve(self, r: np.ndarray, return_coarse: bool = False):
        """MRCM-O solution with source r and homogeneous boundary data
        (optionally also the multiplier coefficients x)."""
        P = self.part
        pover = self.particular(r)
        p = np.zeros(self.nx * self.ny)
        x = self.coarse_solve(self.coarse_rhs(pover))
        for i in range(P.m):
            cells = self.box_cells(P.boxes[i])
            p[cells] = self.restrict(i, pover[i]) + self.mbf[i] @ x[P.dof_offset[i]:P.dof_offset[i + 1]]
        return (p, x) if return_coarse else p

    def smooth(self, r: np.ndarray, p: np.ndarray) -> np.ndarray:
        """Smoothing sweeps on A p = r (Section 2.1, the Schwarz-type
        smoothing step).  Additive (the default): one residual per sweep, every
        patch solved from it, each correction kept on the patch's own
        subdomain (restricted additive Schwarz).  Multiplicative (calibration
        only): patches in subdomain order, each solved from the residual left
        by the ones before it, its correction added on the whole patch."""
        P = self.part
        if self.schwarz == "multiplicative":
            for _ in range(self.sweeps):
                for i in range(P.m):
                    pcells = self.box_cells(P.pboxes[i])
                    rho = r - self.A @ p
                    p = p.copy()
                    p[pcells] += self.patch[i].solve(rho[pcells])
            return p
        for _ in range(self.sweeps):
            rho = r - self.A @ p
            corr = np.zeros_like(p)
            for i in range(P.m):
                pcells = self.box_cells(P.pboxes[i])
                e = self.patch[i].solve(rho[pcells])
                own = P.owner[pcells] == i
                corr[pcells[own]] = e[own]
            p = p + corr
        return p

    def apply(self, r: np.ndarray) -> np.ndarray:
        """z = T r."""
        r = np.asarray(r, dtype=np.float64)
        p = self.smooth(r, self.mrcm_solve(r))
        if self.noflow:
            p = p - p.mean()
        return p
