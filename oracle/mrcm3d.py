"""The MRCM-OS preconditioner T on a 3-D Cartesian grid (oracle).

Test infrastructure, like the rest of oracle/: a plain NumPy/SciPy FP64
statement of the method for d = 3, written from the same passages as the
2-D oracle (oracle.mrcm), with the model problem posed on d-dimensional
Cartesian elements (Section 2, eqs. (1a)-(1d), d = 2 or 3; Section 2.1 for
the decomposition, the Robin conditions, the informed multiplier spaces, the
multiscale basis functions and the four-step algorithm; Section 3 for the
preconditioner with source r and homogeneous data).

Readings for d = 3 (each the direct extension of the 2-D reading):

* Cubic cells of side h; lumped RT0 gives the seven-point two-point-flux
  stencil with harmonic-mean face permeability.  A face of area h^2 between
  centres h apart has transmissibility K_H h; the system is divided by h, so
  A does not depend on h (as in 2-D) and the cell source integrates to
  f h^2.  A Dirichlet face has 2 K_c, a no-flow face 0.
* Sides W, E (x), S, N (y), B, T (z) = 0..5; bc[side] 1 = Dirichlet, 0 =
  no flow.  Cell (ix, iy, iz) has index (iz ny + iy) nx + ix.
* Subdomain (I, J, L) has id (L my + J) mx + I; boxes are
  (x0, x1, y0, y1, z0, z1), half-open; the last layer in each direction is
  narrower when s does not divide n.  Oversampled boxes and smoothing patches
  grow every box by l and delta cells, clipped at the domain.
* The interfaces are the faces shared by neighbouring subdomains: all
  x-interfaces first, then y, then z, each ordered by (L, J, I) of its lower
  subdomain.  A side's faces are ordered by its two tangential coordinates
  (the lower axis fastest).
* Multiplier and test functions on a side with n0 x n1 faces: tensor
  Legendre products P_a(xi) P_b(eta), a < min(d + 1, n0), b < min(d + 1, n1)
  (a fastest), at the face-centre parameters xi_j = (2 j + 1) / n - 1; at
  most (d + 1)^2 per side.  ``degree`` = -1: one indicator per face
  (test-only).
* Robin coefficient b_f = alpha L_cells / K_H(f), L_cells = max(sx, sy, sz)
  for L = H or 1 for L = h; Robin face: U = rho (p_c - lambda), pi = lambda
  + b U with rho = 1 / (1 / (2 K_c) + b); face inside a solve region:
  U = t (p_c - p_c'), pi = (K_c p_c + K_c' p_c') / (K_c + K_c').
* Source-driven basis function on the oversampled box, interface system
  with flux and pressure rows, sparse LU with refinement in extended
  precision, restricted additive Schwarz smoothing, the no-flow pin and the
  zero-mean projection: as in oracle.mrcm.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from numpy.polynomial import legendre

FULL = -1
W, E, S, N, B, T = 0, 1, 2, 3, 4, 5


# ---- fine operator ---------------------------------------------------------
def face_transmissibilities(K, nx, ny, nz, bc):
    """x-, y- and z-face transmissibilities, shapes (nz, ny, nx + 1),
    (nz, ny + 1, nx) and (nz + 1, ny, nx): harmonic mean inside, 2 K_c on
    Dirichlet faces, 0 on no-flow faces."""
    K = np.asarray(K, dtype=np.float64).reshape(nz, ny, nx)
    tx = np.zeros((nz, ny, nx + 1))
    ty = np.zeros((nz, ny + 1, nx))
    tz = np.zeros((nz + 1, ny, nx))
    tx[:, :, 1:nx] = 2.0 * K[:, :, :-1] * K[:, :, 1:] / (K[:, :, :-1] + K[:, :, 1:])
    ty[:, 1:ny, :] = 2.0 * K[:, :-1, :] * K[:, 1:, :] / (K[:, :-1, :] + K[:, 1:, :])
    tz[1:nz, :, :] = 2.0 * K[:-1, :, :] * K[1:, :, :] / (K[:-1, :, :] + K[1:, :, :])
    if bc[W]:
        tx[:, :, 0] = 2.0 * K[:, :, 0]
    if bc[E]:
        tx[:, :, nx] = 2.0 * K[:, :, nx - 1]
    if bc[S]:
        ty[:, 0, :] = 2.0 * K[:, 0, :]
    if bc[N]:
        ty[:, ny, :] = 2.0 * K[:, ny - 1, :]
    if bc[B]:
        tz[0, :, :] = 2.0 * K[0, :, :]
    if bc[T]:
        tz[nz, :, :] = 2.0 * K[nz - 1, :, :]
    return tx, ty, tz


def _stencil_matrix(diag, couplings, shape):
    """Sparse symmetric matrix from a diagonal array and (a, b, t) couplings."""
    n = diag.size
    rows = [np.arange(n)]
    cols = [np.arange(n)]
    vals = [diag.ravel()]
    for a, b, t in couplings:
        rows += [a, b]
        cols += [b, a]
        vals += [-t, -t]
    return sp.csc_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def assemble(K, nx, ny, nz, bc) -> sp.csc_matrix:
    """A_cc = sum of the cell's six face transmissibilities; A_cc' = -t_f."""
    tx, ty, tz = face_transmissibilities(K, nx, ny, nz, bc)
    diag = tx[:, :, :nx] + tx[:, :, 1:] + ty[:, :ny, :] + ty[:, 1:, :] + tz[:nz] + tz[1:]
    ids = np.arange(nx * ny * nz).reshape(nz, ny, nx)
    cpl = [(ids[:, :, :-1].ravel(), ids[:, :, 1:].ravel(), tx[:, :, 1:nx].ravel()),
           (ids[:, :-1, :].ravel(), ids[:, 1:, :].ravel(), ty[:, 1:ny, :].ravel()),
           (ids[:-1].ravel(), ids[1:].ravel(), tz[1:nz].ravel())]
    return _stencil_matrix(diag, cpl, (nz, ny, nx))


def rhs(K, nx, ny, nz, bc, f_cells, g_sides, h):
    """b = f h^2 + 2 K_c g_f on every Dirichlet face; g_sides[side] holds the
    face-centre values of that side as an array over its two tangential
    coordinates in (slower, faster) = (z, y) for W/E, (z, x) for S/N and
    (y, x) for B/T."""
    K = np.asarray(K, dtype=np.float64).reshape(nz, ny, nx)
    b = np.zeros((nz, ny, nx))
    if f_cells is not None:
        b += np.asarray(f_cells, dtype=np.float64).reshape(nz, ny, nx) * h * h
    g = g_sides or {}
    sel = {W: (slice(None), slice(None), 0), E: (slice(None), slice(None), nx - 1),
           S: (slice(None), 0, slice(None)), N: (slice(None), ny - 1, slice(None)),
           B: (0, slice(None), slice(None)), T: (nz - 1, slice(None), slice(None))}
    for side, ix in sel.items():
        if bc[side] and side in g:
            b[ix] += 2.0 * K[ix] * g[side]
    return b.ravel()


def all_noflow(bc) -> bool:
    return not any(bc)


def direct_solve(A, b, bc):
    """Sparse direct solve; with no flow everywhere pin p_0 = 0 and subtract
    the mean (null space span(1))."""
    A = sp.csc_matrix(A)
    if all_noflow(bc):
        p = np.zeros(A.shape[0])
        if A.shape[0] > 1:
            p[1:] = spla.splu(A[1:, 1:].tocsc()).solve(b[1:])
        return p - p.mean()
    return spla.splu(A).solve(b)


# ---- decomposition -------------------------------------------------------------
def _axis(side):
    return side // 2


def _tangential(side):
    """The two tangential axes of a side, lower first."""
    return [a for a in range(3) if a != _axis(side)]


def subdomain_boxes(dims, sizes):
    m = [-(-d // s) for d, s in zip(dims, sizes)]
    boxes = []
    for L in range(m[2]):
        for J in range(m[1]):
            for I in range(m[0]):
                idx = (I, J, L)
                box = []
                for a in range(3):
                    box += [idx[a] * sizes[a], min(dims[a], (idx[a] + 1) * sizes[a])]
                boxes.append(box)
    return np.array(boxes, dtype=np.int64).reshape(-1, 6), m


def grown_boxes(boxes, g, dims):
    out = boxes.copy()
    for a in range(3):
        out[:, 2 * a] = np.maximum(0, boxes[:, 2 * a] - g)
        out[:, 2 * a + 1] = np.minimum(dims[a], boxes[:, 2 * a + 1] + g)
    return out


def interior_sides(box, dims):
    out = []
    for a in range(3):
        if box[2 * a] > 0:
            out.append(2 * a)
        if box[2 * a + 1] < dims[a]:
            out.append(2 * a + 1)
    return out


def side_extent(box, side):
    """Face counts of a side along its two tangential axes."""
    t0, t1 = _tangential(side)
    return int(box[2 * t0 + 1] - box[2 * t0]), int(box[2 * t1 + 1] - box[2 * t1])


def nbasis_1d(degree, length):
    return length if degree == FULL else min(degree + 1, length)


def side_basis(n0, n1, degree):
    """Side functions at the n0 x n1 face centres (lower tangential axis
    fastest), shape (nbasis, n0 n1)."""
    if degree == FULL:
        return np.eye(n0 * n1)
    b0, b1 = nbasis_1d(degree, n0), nbasis_1d(degree, n1)
    x0 = (2.0 * np.arange(n0) + 1.0) / n0 - 1.0
    x1 = (2.0 * np.arange(n1) + 1.0) / n1 - 1.0
    P0 = np.array([legendre.legval(x0, np.eye(b0)[a]) for a in range(b0)])
    P1 = np.array([legendre.legval(x1, np.eye(b1)[q]) for q in range(b1)])
    out = []
    for q in range(b1):
        for a in range(b0):
            out.append(np.outer(P1[q], P0[a]).ravel())
    return np.array(out)


class Partition:
    """Subdomains, oversampled boxes, patches, interfaces, coarse dofs."""

    def __init__(self, dims, sizes, oversample, overlap, degree):
        if min(dims) < 1 or min(sizes) < 1 or oversample < 0 or overlap < 0 or degree < FULL:
            raise ValueError("invalid partition parameters")
        self.dims, self.sizes = tuple(dims), tuple(sizes)
        self.oversample, self.overlap, self.degree = oversample, overlap, degree
        self.boxes, self.mdims = subdomain_boxes(dims, sizes)
        self.m = len(self.boxes)
        self.oboxes = grown_boxes(self.boxes, oversample, dims)
        self.pboxes = grown_boxes(self.boxes, overlap, dims)
        nx, ny, nz = dims
        owner = np.empty(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
        for i, b in enumerate(self.boxes):
            owner[b[4]:b[5], b[2]:b[3], b[0]:b[1]] = i
        self.owner = owner.ravel()
        self.sides = [interior_sides(b, dims) for b in self.boxes]
        for i in range(self.m):
            if interior_sides(self.oboxes[i], dims) != self.sides[i]:
                raise ValueError("oversampling reaches the domain boundary across an interior side")
            if degree == FULL and oversample != 0:
                raise ValueError("the FULL interface space is defined for oversample 0 only")
        mx, my, mz = self.mdims
        stride = (1, mx, mx * my)
        idx = lambda I, J, L: (L * my + J) * mx + I  # noqa: E731
        self.faces = []   # (L, R, axis)
        for a in range(3):
            for L in range(mz):
                for J in range(my):
                    for I in range(mx):
                        c = (I, J, L)
                        if c[a] + 1 < self.mdims[a]:
                            lo = idx(I, J, L)
                            self.faces.append((lo, lo + stride[a], a))
        dofs, offs = [], [0]
        for i in range(self.m):
            for s in self.sides[i]:
                n0, n1 = side_extent(self.boxes[i], s)
                nb = n0 * n1 if degree == FULL else \
                    nbasis_1d(degree, n0) * nbasis_1d(degree, n1)
                for q in range(nb):
                    dofs.append((i, s, q))
            offs.append(len(dofs))
        self.dof_table = np.array(dofs, dtype=np.int64).reshape(-1, 3)
        self.dof_offset = np.array(offs, dtype=np.int64)

    @property
    def nc(self):
        return int(self.dof_offset[-1])


def face_sides(axis):
    """Side of the lower and of the upper subdomain an interface lies on."""
    return 2 * axis + 1, 2 * axis


# ---- the preconditioner ------------------------------------------------------------
class BoxSolver:
    """Sparse direct solver of one local matrix (library LU as the step)."""

    def __init__(self, A, pin):
        A = sp.lil_matrix(A)
        if pin:
            A[0, :] = 0.0
            A[:, 0] = 0.0
            A[0, 0] = 1.0
        self.pin = pin
        self.lu = spla.splu(sp.csc_matrix(A))

    def solve(self, r):
        r = np.array(r, dtype=np.float64)
        if self.pin:
            r[0] = 0.0
        return self.lu.solve(r)


class SideFaces:
    """Faces of one side of a box: inside and outside cells, t, K, b, rho."""

    def __init__(self, mr, box, side):
        a = _axis(side)
        t0, t1 = _tangential(side)
        hi = side % 2 == 1
        rng = [np.arange(box[2 * k], box[2 * k + 1]) for k in range(3)]
        pos = box[2 * a + 1] - 1 if hi else box[2 * a]
        out = pos + 1 if hi else pos - 1
        fpos = box[2 * a + 1] if hi else box[2 * a]   # face index along the axis
        ins, outs, ts = [], [], []
        tarr = (mr.tx, mr.ty, mr.tz)[a]
        for c1 in rng[t1]:
            for c0 in rng[t0]:
                ci = [0, 0, 0]
                ci[t0], ci[t1], ci[a] = c0, c1, pos
                co = list(ci)
                co[a] = out
                fi = list(ci)
                fi[a] = fpos
                ins.append(mr.cell(*ci))
                outs.append(mr.cell(*co))
                ts.append(tarr[fi[2], fi[1], fi[0]])
        self.side = side
        self.n0, self.n1 = len(rng[t0]), len(rng[t1])
        self.inside = np.array(ins, dtype=np.int64)
        self.outside = np.array(outs, dtype=np.int64)
        self.t = np.array(ts)
        self.K_in = mr.K[self.inside]
        valid = (self.outside >= 0) & (self.outside < mr.n)
        self.K_out = np.where(valid, mr.K[np.clip(self.outside, 0, mr.n - 1)], 1.0)
        with np.errstate(divide="ignore"):
            self.b = mr.alpha * mr.L_cells / self.t
        self.rho = 1.0 / (1.0 / (2.0 * self.K_in) + self.b)


class MRCM3D:
    """Set-up and application of T for one 3-D permeability field."""

    def __init__(self, K, nx, ny, nz, bc, sx, sy, sz, oversample, alpha, beta_len="H",
                 sweeps=0, overlap=2, degree=1):
        self.K = np.asarray(K, dtype=np.float64).ravel()
        self.nx, self.ny, self.nz = nx, ny, nz
        self.n = nx * ny * nz
        if self.K.size != self.n or not np.all(np.isfinite(self.K)) or np.any(self.K <= 0):
            raise ValueError("K must be finite and positive on every cell")
        self.bc = tuple(int(v) for v in bc)
        self.alpha = float(alpha)
        self.L_cells = float(max(sx, sy, sz)) if beta_len == "H" else 1.0
        self.sweeps, self.overlap, self.degree = int(sweeps), int(overlap), int(degree)
        self.part = Partition((nx, ny, nz), (sx, sy, sz), oversample, overlap, degree)
        self.tx, self.ty, self.tz = face_transmissibilities(self.K, nx, ny, nz, self.bc)
        self.A = assemble(self.K, nx, ny, nz, self.bc)
        self.noflow = all_noflow(self.bc)
        P = self.part
        self.gamma = [[SideFaces(self, P.boxes[i], s) for s in P.sides[i]] for i in range(P.m)]
        self.local = [self._box_solver(P.boxes[i], True) for i in range(P.m)]
        self.over = [self._box_solver(P.oboxes[i], True) for i in range(P.m)]
        self.ocells = [self.box_cells(P.oboxes[i]) for i in range(P.m)]
        self.oloc = [{int(c): j for j, c in enumerate(oc)} for oc in self.ocells]
        self.phi = [self._informed_space(i) for i in range(P.m)]
        self.mbf, self.mbf_U, self.mbf_pi = [], [], []
        for i in range(P.m):
            Pi, Ui, pii = self._mbfs(i)
            self.mbf.append(Pi)
            self.mbf_U.append(Ui)
            self.mbf_pi.append(pii)
        self.patch = [self._box_solver(P.pboxes[i], False) for i in range(P.m)] \
            if self.sweeps > 0 else []
        self._coarse_assemble()

    # ---- cells and local operators ------------------------------------------
    def cell(self, ix, iy, iz):
        if not (0 <= ix < self.nx and 0 <= iy < self.ny and 0 <= iz < self.nz):
            return -1
        return (iz * self.ny + iy) * self.nx + ix

    def box_cells(self, box):
        ids = np.arange(self.n).reshape(self.nz, self.ny, self.nx)
        return ids[box[4]:box[5], box[2]:box[3], box[0]:box[1]].ravel()

    def box_matrix(self, box, robin):
        """Local matrix on a cell box: faces inside couple as in A, domain
        boundary faces keep the global condition, faces leaving the box
        inside the domain carry rho_f (robin) or t_f with zero data beyond
        (the principal submatrix of A)."""
        x0, x1, y0, y1, z0, z1 = (int(v) for v in box)
        K = self.K.reshape(self.nz, self.ny, self.nx)[z0:z1, y0:y1, x0:x1]
        tW = self.tx[z0:z1, y0:y1, x0:x1].copy()
        tE = self.tx[z0:z1, y0:y1, x0 + 1:x1 + 1].copy()
        tS = self.ty[z0:z1, y0:y1, x0:x1].copy()
        tN = self.ty[z0:z1, y0 + 1:y1 + 1, x0:x1].copy()
        tB = self.tz[z0:z1, y0:y1, x0:x1].copy()
        tT = self.tz[z0 + 1:z1 + 1, y0:y1, x0:x1].copy()
        if robin:
            def rho(Kc, t):
                return 1.0 / (1.0 / (2.0 * Kc) + self.alpha * self.L_cells / t)
            if x0 > 0:
                tW[:, :, 0] = rho(K[:, :, 0], tW[:, :, 0])
            if x1 < self.nx:
                tE[:, :, -1] = rho(K[:, :, -1], tE[:, :, -1])
            if y0 > 0:
                tS[:, 0, :] = rho(K[:, 0, :], tS[:, 0, :])
            if y1 < self.ny:
                tN[:, -1, :] = rho(K[:, -1, :], tN[:, -1, :])
            if z0 > 0:
                tB[0] = rho(K[0], tB[0])
            if z1 < self.nz:
                tT[-1] = rho(K[-1], tT[-1])
        diag = tW + tE + tS + tN + tB + tT
        loc = np.arange(diag.size).reshape(diag.shape)
        cpl = [(loc[:, :, :-1].ravel(), loc[:, :, 1:].ravel(), tW[:, :, 1:].ravel()),
               (loc[:, :-1, :].ravel(), loc[:, 1:, :].ravel(), tS[:, 1:, :].ravel()),
               (loc[:-1].ravel(), loc[1:].ravel(), tB[1:].ravel())]
        return _stencil_matrix(diag, cpl, diag.shape)

    def _box_solver(self, box, robin):
        whole = all(box[2 * a] == 0 and box[2 * a + 1] == (self.nx, self.ny, self.nz)[a]
                    for a in range(3))
        return BoxSolver(self.box_matrix(box, robin), pin=self.noflow and whole)

    # ---- informed multiplier spaces and MBFs (set-up) ----------------------------
    def coarse_functions(self, i):
        P = self.part
        return [(int(s), int(q)) for (_, s, q) in P.dof_table[P.dof_offset[i]:P.dof_offset[i + 1]]]

    def _gamma_of(self, i, side):
        for g in self.gamma[i]:
            if g.side == side:
                return g
        raise KeyError(side)

    def oversampled_traces(self, i, ph, lam=None):
        """Flux and face pressure of an oversampled solution across the faces
        of Gamma_i, per side (Robin faces when l = 0, interior faces else)."""
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

    def _informed_space(self, i):
        P = self.part
        oside = {s: SideFaces(self, P.oboxes[i], s) for s in P.sides[i]}
        phis = []
        for (s, q) in self.coarse_functions(i):
            sf = oside[s]
            lam = side_basis(sf.n0, sf.n1, self.degree)[q]
            rhs_ = np.zeros(self.ocells[i].size)
            np.add.at(rhs_, [self.oloc[i][int(c)] for c in sf.inside], sf.rho * lam)
            ph = self.over[i].solve(rhs_)
            tr = self.oversampled_traces(i, ph, {s: lam})
            phis.append({sd: pi - self._gamma_of(i, sd).b * U for sd, (U, pi) in tr.items()})
        return phis

    def _mbfs(self, i):
        cells = self.box_cells(self.part.boxes[i])
        loc = {int(c): j for j, c in enumerate(cells)}
        cols, Us, pis = [], [], []
        for phi_k in self.phi[i]:
            rhs_ = np.zeros(cells.size)
            for g in self.gamma[i]:
                np.add.at(rhs_, [loc[int(c)] for c in g.inside], g.rho * phi_k[g.side])
            p = self.local[i].solve(rhs_)
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

    # ---- interface system ------------------------------------------------------
    def _face_basis(self, f):
        L, R, a = self.part.faces[f]
        sL, _ = face_sides(a)
        n0, n1 = side_extent(self.part.boxes[L], sL)
        return side_basis(n0, n1, self.degree)

    def _coarse_assemble(self):
        P = self.part
        nc = P.nc
        self.row_offset = np.zeros(len(P.faces) + 1, dtype=np.int64)
        for f in range(len(P.faces)):
            self.row_offset[f + 1] = self.row_offset[f] + 2 * self._face_basis(f).shape[0]
        if self.row_offset[-1] != nc:
            raise AssertionError("coarse system is not square")
        C = sp.lil_matrix((nc, nc))
        for f, (L, R, a) in enumerate(P.faces):
            sL, sR = face_sides(a)
            Bf = self._face_basis(f)
            nb = Bf.shape[0]
            r0 = self.row_offset[f]
            for (sub, sd, sign) in ((L, sL, 1.0), (R, sR, -1.0)):
                for k in range(P.dof_offset[sub + 1] - P.dof_offset[sub]):
                    col = P.dof_offset[sub] + k
                    fU = Bf @ self.mbf_U[sub][k][sd]
                    fP = Bf @ self.mbf_pi[sub][k][sd]
                    for q in range(nb):
                        C[r0 + q, col] += fU[q]
                        C[r0 + nb + q, col] += sign * fP[q]
        self.pin_row = -1
        if self.noflow and len(P.faces) > 0:
            L0, _, a0 = P.faces[0]
            s0 = face_sides(a0)[0]
            col = P.dof_offset[L0] + [j for j, (s, q) in enumerate(self.coarse_functions(L0))
                                      if s == s0 and q == 0][0]
            self.pin_row = 0
            C[0, :] = 0.0
            C[0, col] = 1.0
        self.C = sp.csc_matrix(C)
        self.C_lu = spla.splu(self.C) if nc > 0 else None
        self.C_ext = sp.csr_matrix(self.C).astype(np.longdouble) if nc > 0 else None

    def coarse_solve(self, g):
        """LU solve, then refinement with extended-precision residuals."""
        if self.part.nc == 0:
            return np.zeros(0)
        gl = np.asarray(g, dtype=np.longdouble)
        x = self.C_lu.solve(np.asarray(g, dtype=np.float64)).astype(np.longdouble)
        for _ in range(10):
            dx = self.C_lu.solve(np.asarray(gl - self.C_ext @ x, dtype=np.float64))
            x = x + dx.astype(np.longdouble)
            if np.abs(dx).max() <= 1e-18 * float(np.abs(x).max()):
                break
        return np.asarray(x, dtype=np.float64)

    # ---- application of T --------------------------------------------------------
    def particular(self, r):
        return [self.over[i].solve(r[self.ocells[i]]) for i in range(self.part.m)]

    def restrict(self, i, ph):
        return ph[[self.oloc[i][int(c)] for c in self.box_cells(self.part.boxes[i])]]

    def coarse_rhs(self, pover):
        P = self.part
        g = np.zeros(P.nc)
        traces = [self.oversampled_traces(i, pover[i]) for i in range(P.m)]
        for f, (L, R, a) in enumerate(P.faces):
            sL, sR = face_sides(a)
            Bf = self._face_basis(f)
            nb = Bf.shape[0]
            UL, piL = traces[L][sL]
            UR, piR = traces[R][sR]
            r0 = self.row_offset[f]
            g[r0:r0 + nb] = -(Bf @ (UL + UR))
            g[r0 + nb:r0 + 2 * nb] = -(Bf @ (piL - piR))
        if self.pin_row >= 0:
            g[self.pin_row] = 0.0
        return g

    def mrcm_solve(self, r, return_coarse=False):
        P = self.part
        pover = self.particular(r)
        x = self.coarse_solve(self.coarse_rhs(pover))
        p = np.zeros(self.n)
        for i in range(P.m):
            p[self.box_cells(P.boxes[i])] = self.restrict(i, pover[i]) + \
                self.mbf[i] @ x[P.dof_offset[i]:P.dof_offset[i + 1]]
        return (p, x) if return_coarse else p

    def smooth(self, r, p):
        """Restricted additive Schwarz sweeps on A p = r."""
        P = self.part
        for _ in range(self.sweeps):
            rho = r - self.A @ p
            corr = np.zeros_like(p)
            for i in range(P.m):
                pc = self.box_cells(P.pboxes[i])
                e = self.patch[i].solve(rho[pc])
                own = P.owner[pc] == i
                corr[pc[own]] = e[own]
            p = p + corr
        return p

    def apply(self, r):
        """z = T r."""
        r = np.asarray(r, dtype=np.float64)
        p = self.smooth(r, self.mrcm_solve(r))
        if self.noflow:
            p = p - p.mean()
        return p
