"""Pins of the fine system A p = b (oracle.discretization).

* The condensed matrix equals the one obtained by building the mixed RT0 / P0
  system from its basis functions (vertex quadrature) and eliminating the
  velocity densely (Section 3, static condensation of the RT0 system).
* Manufactured solutions of Section 4 (constant and variable K) converge at
  second order at cell centres, with the paper's Dirichlet left/right setup
  and with no-flow on all sides (both exact solutions have zero normal
  derivative on every side and zero mean).
"""
import math

import numpy as np
import pytest

from oracle.brute import rt0_vertex_quadrature_system
from oracle.discretization import assemble, direct_solve, rhs
from paper_2606_08883_amd import workloads as wl

BCS = [(0, 0, 0, 0), (1, 1, 0, 0), (1, 0, 1, 1), (1, 1, 1, 1)]


@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("shape", [(5, 4), (3, 3), (7, 2)])
def test_tpfa_equals_condensed_rt0(bc, shape):
    nx, ny = shape
    K = wl.lognormal_K(nx, ny, 1.5, 2.0, 11)
    h = 0.1
    f = wl.random_vector(nx * ny, 5)
    g = {0: np.linspace(1, 2, ny), 1: np.linspace(-1, 0.5, ny), 2: np.linspace(0, 3, nx),
         3: np.linspace(2, -2, nx)}
    A = assemble(K, nx, ny, bc).toarray()
    b = rhs(K, nx, ny, bc, f, g, h)
    Ab, bb = rt0_vertex_quadrature_system(K, nx, ny, bc, h, f, {s: g[s] for s in range(4) if bc[s]})
    assert np.abs(A - Ab).max() <= 1e-13 * np.abs(A).max()
    assert np.abs(b - bb).max() <= 1e-13 * max(1.0, np.abs(b).max())


def test_harmonic_transmissibility_by_hand():
    # two cells, K = 1 and 3: interior transmissibility 2*1*3/(1+3) = 1.5
    A = assemble(np.array([1.0, 3.0]), 2, 1, (1, 0, 0, 0)).toarray()
    assert A[0, 1] == -1.5 and A[1, 0] == -1.5
    assert A[0, 0] == 1.5 + 2.0 and A[1, 1] == 1.5


@pytest.mark.parametrize("bc", BCS)
def test_operator_invariants(bc):
    nx, ny = 9, 7
    K = wl.lognormal_K(nx, ny, 2.0, 3.0, 2)
    A = assemble(K, nx, ny, bc)
    assert abs(A - A.T).max() == 0.0
    ones = A @ np.ones(nx * ny)
    Kg = K.reshape(ny, nx)
    expect = np.zeros((ny, nx))
    if bc[0]:
        expect[:, 0] += 2 * Kg[:, 0]
    if bc[1]:
        expect[:, -1] += 2 * Kg[:, -1]
    if bc[2]:
        expect[0, :] += 2 * Kg[0, :]
    if bc[3]:
        expect[-1, :] += 2 * Kg[-1, :]
    assert np.abs(ones - expect.ravel()).max() <= 1e-13 * np.abs(A.diagonal()).max()
    w = np.linalg.eigvalsh(A.toarray())
    if any(bc):
        assert w.min() > 0
    else:
        assert abs(w[0]) < 1e-10 * w[-1] and w[1] > 0


@pytest.mark.parametrize("bc", [(0, 0, 0, 0), (1, 1, 0, 0)])
def test_direct_solve_vs_dense(bc):
    nx, ny = 12, 10
    K = wl.lognormal_K(nx, ny, 2.0, 3.0, 4)
    A = assemble(K, nx, ny, bc)
    b = wl.random_vector(nx * ny, 9, zero_mean=not any(bc))
    p = direct_solve(A, b, bc)
    if any(bc):
        ref = np.linalg.solve(A.toarray(), b)
    else:
        ref = np.linalg.lstsq(A.toarray(), b, rcond=None)[0]
        ref -= ref.mean()
    assert np.linalg.norm(p - ref) <= 1e-12 * np.linalg.norm(ref)
    assert np.linalg.norm(A @ p - b) <= 1e-12 * np.linalg.norm(b)


def _manufactured_error(case, nx, bc):
    h = 1.0 / nx
    Kf, ff, pf = wl.manufactured(case)
    X, Y = wl.cell_centres(nx, nx)
    K = Kf(X, Y)
    yc = (np.arange(nx) + 0.5) * h
    g = {}
    if bc[0]:
        g[0] = pf(np.zeros(nx), yc)
    if bc[1]:
        g[1] = pf(np.ones(nx), yc)
    b = rhs(K, nx, nx, bc, ff(X, Y), g, h)
    p = direct_solve(assemble(K, nx, nx, bc), b, bc)
    exact = pf(X, Y)
    if not any(bc):
        exact = exact - exact.mean()
    return np.sqrt(np.mean((p - exact) ** 2))


@pytest.mark.parametrize("case", ["const", "var"])
@pytest.mark.parametrize("bc", [(1, 1, 0, 0), (0, 0, 0, 0)])
def test_manufactured_second_order(case, bc):
    errs = [_manufactured_error(case, n, bc) for n in (16, 32, 64, 128)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(3)]
    assert all(1.8 <= o <= 2.2 for o in orders[1:]), (errs, orders)
    assert errs[-1] < 1e-3


def test_paper_dirichlet_data_of_the_variable_case_is_not_the_trace():
    # Section 4 gives cos(2 pi y) on both sides for both analytic cases; for
    # p = cos(pi x) cos(pi y) the traces are cos(pi y) and -cos(pi y).
    Kf, ff, pf = wl.manufactured("var")
    y = np.linspace(0, 1, 11)
    assert np.allclose(pf(np.zeros_like(y), y), np.cos(np.pi * y))
    assert np.allclose(pf(np.ones_like(y), y), -np.cos(np.pi * y))
    assert not np.allclose(pf(np.zeros_like(y), y), np.cos(2 * np.pi * y))
