"""Pins of the MRCM-OS operator T (oracle.mrcm), Sections 2.1 and 3.

* l = 0: the informed functions are the Robin data themselves (phi = lambda).
* l > 0: each multiscale basis function equals the oversampled solution
  restricted to Omega_i (the Robin data phi reproduces it exactly).
* FULL interface space with l = 0: weak continuity becomes face-wise flux and
  pressure continuity, so the MRCM solve is the exact fine solve A^-1 r.
* The MBF-reduced solve equals the monolithic solve of eqs. (11)-(14).
* The source-driven oversampled solution restricted to Omega_i solves the
  local Robin problem on Omega_i with source r and its own trace phi_{i,r} as
  Robin data (so every local solution of T satisfies (11)-(12) on Omega_i);
  with l = 0 that trace is zero.
* One subdomain covering the grid: T = A^-1 and GMRES converges in one step.
* Smoothing: an exact solution is a fixed point; a patch covering the whole
  grid gives A^-1 r in one sweep.
* Linearity, the zero-mean projection's independence from the replaced row,
  subdomain mass balance and the weak continuity equations themselves.
"""
import numpy as np
import pytest

from oracle.brute import monolithic_mrcm
from oracle.discretization import direct_solve
from oracle.gmres import gmres
from oracle.mrcm import MRCM, side_basis
from oracle.partition import FULL, edge_sides
from paper_2606_08883_amd import workloads as wl


def _setup(nx=24, ny=20, bc=(1, 1, 0, 0), s=8, l=0, k=0, d=1, alpha=10.0, blen="H", seed=3,
           sigma=2.0, **kw):
    K = wl.lognormal_K(nx, ny, sigma, 4.0, seed)
    return MRCM(K, nx, ny, bc, s, s, l, alpha, blen, k, 2, d, **kw)


def test_local_solves_match_dense_solve():
    mr = _setup()
    r = wl.random_vector(mr.nx * mr.ny, 1)
    for i in range(mr.part.m):
        cells = mr.box_cells(mr.part.boxes[i])
        Ad = mr.box_matrix(mr.part.boxes[i], True).toarray()
        assert np.all(np.linalg.eigvalsh(Ad) > 0)
        ref = np.linalg.solve(Ad, r[cells])
        assert np.linalg.norm(mr.local[i].solve(r[cells]) - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_informed_space_without_oversampling_is_the_data(d):
    mr = _setup(l=0, d=d)
    for i in range(mr.part.m):
        for k, (s, q) in enumerate(mr.coarse_functions(i)):
            for g in mr.gamma[i]:
                lam = side_basis(g.inside.size, d)[q] if g.side == s else np.zeros(g.inside.size)
                assert np.abs(mr.phi[i][k][g.side] - lam).max() <= 1e-13


@pytest.mark.parametrize("l", [1, 2, 3])
def test_basis_functions_reproduce_oversampled_solutions(l):
    mr = _setup(l=l, nx=30, ny=26, s=10)
    P = mr.part
    for i in (0, P.m // 2, P.m - 1):
        ob = P.oboxes[i]
        ocells = mr.box_cells(ob)
        A = mr.box_matrix(ob, True).toarray()
        cells = mr.box_cells(P.boxes[i])
        pos = [int(np.flatnonzero(ocells == c)[0]) for c in cells]
        from oracle.mrcm import SideFaces
        for k, (s, q) in enumerate(mr.coarse_functions(i)):
            sf = SideFaces(mr, ob, s)
            rhs = np.zeros(ocells.size)
            lam = side_basis(sf.inside.size, mr.degree)[q]
            for c, rho, lv in zip(sf.inside, sf.rho, lam):
                rhs[int(np.flatnonzero(ocells == c)[0])] += rho * lv
            ph = np.linalg.solve(A, rhs)
            assert np.linalg.norm(mr.mbf[i][:, k] - ph[pos]) <= 1e-11 * np.linalg.norm(ph[pos])


@pytest.mark.parametrize("l,bc", [(0, (1, 1, 0, 0)), (2, (1, 1, 0, 0)), (3, (0, 0, 0, 0)),
                                  (1, (1, 0, 1, 0))])
def test_source_driven_solution_solves_the_local_problem(l, bc):
    mr = _setup(l=l, nx=30, ny=26, s=10, bc=bc)
    P = mr.part
    r = wl.random_vector(mr.nx * mr.ny, 21)
    pover = mr.particular(r)
    lam0 = mr.source_multiplier(r)
    for i in range(P.m):
        cells = mr.box_cells(P.boxes[i])
        pos = {int(c): j for j, c in enumerate(cells)}
        rhs = r[cells].copy()
        for g in mr.gamma[i]:
            for c, rho, l0 in zip(g.inside, g.rho, lam0[i][g.side]):
                rhs[pos[int(c)]] += rho * l0
            if l == 0:
                assert np.abs(lam0[i][g.side]).max() == 0.0
        ref = np.linalg.solve(mr.box_matrix(P.boxes[i], True).toarray(), rhs)
        got = mr.restrict(i, pover[i])
        assert np.linalg.norm(got - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("bc", [(1, 1, 0, 0), (0, 0, 0, 0), (1, 0, 1, 0)])
def test_full_interface_space_gives_the_exact_solve(bc):
    mr = _setup(nx=20, ny=16, s=5, d=FULL, bc=bc)
    r = wl.random_vector(mr.nx * mr.ny, 4, zero_mean=not any(bc))
    p = mr.mrcm_solve(r)
    exact = direct_solve(mr.A, r, bc)
    if not any(bc):
        p = p - p.mean()
    assert np.linalg.norm(p - exact) <= 1e-10 * np.linalg.norm(exact)


@pytest.mark.parametrize("l,d,bc", [(0, 1, (1, 1, 0, 0)), (2, 1, (0, 0, 0, 0)),
                                    (3, 2, (1, 0, 0, 1)), (1, 0, (1, 1, 0, 0))])
def test_mbf_reduction_equals_monolithic_system(l, d, bc):
    mr = _setup(nx=25, ny=20, s=7, l=l, d=d, bc=bc)
    r = wl.random_vector(mr.nx * mr.ny, 8, zero_mean=not any(bc))
    p1 = mr.mrcm_solve(r)
    p2 = monolithic_mrcm(mr, r)
    assert np.linalg.norm(p1 - p2) <= 1e-11 * np.linalg.norm(p2)


@pytest.mark.parametrize("bc", [(1, 1, 0, 0), (0, 0, 0, 0)])
@pytest.mark.parametrize("k", [0, 2])
def test_one_subdomain_is_the_exact_inverse(bc, k):
    mr = _setup(nx=16, ny=12, s=16, l=0, k=k, bc=bc)
    assert mr.part.m == 1 and mr.part.nc == 0
    r = wl.random_vector(mr.nx * mr.ny, 2, zero_mean=not any(bc))
    exact = direct_solve(mr.A, r, bc)
    assert np.linalg.norm(mr.apply(r) - exact) <= 1e-10 * np.linalg.norm(exact)
    res = gmres(lambda x: mr.A @ x, mr.apply, r, rtol=1e-8)
    assert res.iterations == 1 and res.converged


def test_smoothing_fixed_point_and_whole_grid_patch():
    mr = _setup(k=2, l=2)
    r = wl.random_vector(mr.nx * mr.ny, 6)
    exact = direct_solve(mr.A, r, mr.bc)
    assert np.linalg.norm(mr.smooth(r, exact) - exact) <= 1e-12 * np.linalg.norm(exact)
    big = _setup(k=1, l=0, s=8)
    big.part.pboxes[:] = (0, big.nx, 0, big.ny)
    big.patch = [big._box_solver(big.part.pboxes[i], robin=False) for i in range(big.part.m)]
    one = big.smooth(r, np.zeros_like(r))
    assert np.linalg.norm(one - exact) <= 1e-12 * np.linalg.norm(exact)


def test_multiplicative_smoothing_is_the_product_of_patch_projections():
    """Multiplicative Schwarz (the calibration variant of the smoothing
    step): one sweep maps the error e = x - p to prod_i (I - R_i^T
    A_{S_i}^-1 R_i A) e, patches in subdomain order (the last factor
    applied first), written out densely here."""
    mr = _setup(k=1, l=2, schwarz="multiplicative")
    n = mr.nx * mr.ny
    r = wl.random_vector(n, 7)
    exact = direct_solve(mr.A, r, mr.bc)
    assert np.linalg.norm(mr.smooth(r, exact) - exact) <= 1e-12 * np.linalg.norm(exact)
    p0 = wl.random_vector(n, 8)
    A = mr.A.toarray()
    E = np.eye(n)
    for i in range(mr.part.m):
        cells = mr.box_cells(mr.part.pboxes[i])
        R = np.zeros((len(cells), n))
        R[np.arange(len(cells)), cells] = 1.0
        Pi = R.T @ np.linalg.solve(A[np.ix_(cells, cells)], R @ A)
        E = (np.eye(n) - Pi) @ E
    want = exact - E @ (exact - p0)
    got = mr.smooth(r, p0)
    assert np.linalg.norm(got - want) <= 1e-10 * np.linalg.norm(want)
    with pytest.raises(ValueError):
        _setup(schwarz="jacobi")


def test_calibration_script_runs_a_paper_case():
    """The calibration script's set-up of Table 2 gives the printed count
    within one cycle for a cheap case (8 x 8, 2h,2S, multiplicative)."""
    from oracle import calibrate_tables as ct
    job = ("msm", 2, 8, "2h,2S")
    got = ct.cycles(job)[1]
    assert got is not None and abs(got - ct.paper_counts()[(2, "2h,2S")][8]) <= 1


def test_principal_submatrix_patches():
    mr = _setup(k=1, l=2)
    for i in range(mr.part.m):
        cells = mr.box_cells(mr.part.pboxes[i])
        sub = mr.A[cells][:, cells].toarray()
        diff = np.abs(mr.box_matrix(mr.part.pboxes[i], False).toarray() - sub).max()
        assert diff <= 1e-14 * np.abs(sub).max()


@pytest.mark.parametrize("bc", [(1, 1, 0, 0), (0, 0, 0, 0)])
def test_linearity(bc):
    mr = _setup(l=2, k=1, bc=bc)
    n = mr.nx * mr.ny
    r1 = wl.random_vector(n, 1, zero_mean=not any(bc))
    r2 = wl.random_vector(n, 2, zero_mean=not any(bc))
    lhs = mr.apply(2.5 * r1 - 0.75 * r2)
    rhs_ = 2.5 * mr.apply(r1) - 0.75 * mr.apply(r2)
    assert np.linalg.norm(lhs - rhs_) <= 1e-12 * np.linalg.norm(rhs_)


def test_noflow_projection_independent_of_replaced_row():
    a = _setup(l=2, k=1, bc=(0, 0, 0, 0), pin_edge=0)
    b = _setup(l=2, k=1, bc=(0, 0, 0, 0), pin_edge=len(a.part.edges) - 1)
    assert a.pin_row != b.pin_row
    r = wl.random_vector(a.nx * a.ny, 5, zero_mean=True)
    za, zb = a.apply(r), b.apply(r)
    assert abs(za.mean()) < 1e-14 * np.abs(za).max()
    assert np.linalg.norm(za - zb) <= 1e-10 * np.linalg.norm(za)


@pytest.mark.parametrize("l", [0, 2])
def test_subdomain_mass_balance_and_weak_continuity(l):
    mr = _setup(l=l, d=1, bc=(1, 1, 0, 0))
    P = mr.part
    r = wl.random_vector(mr.nx * mr.ny, 12)
    p, x = mr.mrcm_solve(r, return_coarse=True)
    lam0 = mr.source_multiplier(r)
    U, PI = {}, {}
    for i in range(P.m):
        lam = {g.side: lam0[i][g.side].copy() for g in mr.gamma[i]}
        for k in range(P.dof_offset[i + 1] - P.dof_offset[i]):
            for g in mr.gamma[i]:
                lam[g.side] += x[P.dof_offset[i] + k] * mr.phi[i][k][g.side]
        net = 0.0
        for g in mr.gamma[i]:
            u = g.rho * (p[g.inside] - lam[g.side])
            U[(i, g.side)] = u
            PI[(i, g.side)] = lam[g.side] + g.b * u
            net += u.sum()
        cells = mr.box_cells(P.boxes[i])
        # no-flow top/bottom; Dirichlet faces carry flux 2 K p (homogeneous data)
        Kc = mr.K[cells]
        xs = cells % mr.nx
        dir_flux = sum(2 * Kc[xs == 0] * p[cells][xs == 0]) + \
            sum(2 * Kc[xs == mr.nx - 1] * p[cells][xs == mr.nx - 1])
        assert abs(net + dir_flux - r[cells].sum()) <= 1e-10 * np.abs(r[cells]).sum()
    for (L, R, o, st, ln) in P.edges:
        sL, sR = edge_sides(int(o))
        B = side_basis(int(ln), 1)
        flux = B @ (U[(L, sL)] + U[(R, sR)])
        pres = B @ (PI[(L, sL)] - PI[(R, sR)])
        scale = np.abs(U[(L, sL)]).sum() + np.abs(PI[(L, sL)]).sum() + 1e-300
        assert np.abs(flux).max() <= 1e-10 * scale and np.abs(pres).max() <= 1e-10 * scale


def test_ragged_grid_converges():
    mr = _setup(nx=37, ny=29, s=10, l=2, k=1, bc=(0, 0, 0, 0))
    b = wl.corner_sources(37, 29)
    res = gmres(lambda x: mr.A @ x, mr.apply, b, rtol=1e-8)
    exact = direct_solve(mr.A, b, mr.bc)
    assert res.converged
    assert np.linalg.norm(res.p - res.p.mean() - exact) <= 1e-6 * np.linalg.norm(exact)


def test_rejects_bad_permeability():
    with pytest.raises(ValueError):
        MRCM(np.r_[np.ones(15), 0.0], 4, 4, (1, 1, 0, 0), 2, 2, 0, 10.0)
    with pytest.raises(ValueError):
        MRCM(np.r_[np.ones(15), np.nan], 4, 4, (1, 1, 0, 0), 2, 2, 0, 10.0)


def test_refined_interface_solve_matches_exact_rational_solve():
    """The oracle's interface solve (LU + refinement with extended-precision
    residuals) against Gaussian elimination in exact rational arithmetic on
    the same FP64 matrix and right-hand side, for an interface system of a
    1e6-contrast channel field (condition number far above 1e8)."""
    from fractions import Fraction
    K = wl.channel_K(40, 20, 10.0, 3.0, 2)
    mr = MRCM(K, 40, 20, (1, 1, 0, 0), 10, 10, 2, 10.0, "H", 0, 2, 1)
    C = mr.C.toarray()
    n = C.shape[0]
    assert np.linalg.cond(C) > 1e8
    g = wl.random_vector(n, 31)
    M = [[Fraction(float(C[i, j])) for j in range(n)] + [Fraction(float(g[i]))] for i in range(n)]
    for c in range(n):
        piv = max(range(c, n), key=lambda r: abs(M[r][c]))
        M[c], M[piv] = M[piv], M[c]
        for r in range(c + 1, n):
            if M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [a - f * b for a, b in zip(M[r], M[c])]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        x[i] = (M[i][n] - sum(M[i][j] * x[j] for j in range(i + 1, n))) / M[i][i]
    exact = np.array([float(v) for v in x])
    got = mr.coarse_solve(g)
    assert np.linalg.norm(got - exact) <= 4e-16 * np.linalg.norm(exact)
