"""Parity gates shared by the test modules.

FP64 gate: relative L2 1e-10.  When the oracle's interface matrix C is
ill-conditioned (the 1e6-contrast channel field: cond(C) ~ 1e9 - 1e12; the
sigma = 3 log-normal field at 1024 x 1024: cond_1(C) ~ 4e10), two FP64
implementations that factor C differently (the oracle: one sparse LU; the
library: row equilibration and a nested-dissection multifrontal LU) both
carry a forward error of up to about cond(C) * 2^-53 in the interface
solution, so they can differ by that much.  The gate is then that
first-order bound (never below 1e-10).  cond(C) is the 2-norm condition
number of the oracle's own C for small systems and the estimated 1-norm
condition number (scipy's onenormest on C and on C^-1 through its LU) for
large ones.
"""
import numpy as np
import scipy.sparse.linalg as spla

FP64_GATE = 1e-10
UNIT_ROUNDOFF = 2.0 ** -53
DENSE_COND_MAX = 4000


def interface_condition(mr) -> float:
    C = mr.C
    n = C.shape[0]
    if n <= DENSE_COND_MAX:
        return float(np.linalg.cond(C.toarray()))
    lu = spla.splu(C.tocsc())
    inv = spla.LinearOperator((n, n), matvec=lu.solve,
                              rmatvec=lambda x: lu.solve(x, trans="T"), dtype=float)
    return float(spla.onenormest(C) * spla.onenormest(inv))


def t_gate(mr) -> float:
    if mr.part.nc == 0:
        return FP64_GATE
    return max(FP64_GATE, interface_condition(mr) * UNIT_ROUNDOFF)
