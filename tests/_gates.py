"""Parity gates shared by the test modules.

FP64 gate: relative L2 1e-10.

Mixed precision (precision modes 1 and 2): solutions driven to relative
residual 1e-10 agree to MIXED_GATE = 1e-7.  T itself differs from the FP64
operator by the FP32 rounding of the box factors (mode 2: stored in FP32,
applied in FP64; mode 1: also applied in FP32): a box solve runs its block
recurrence down and back up the rows of the box, one product with a rounded
inverse block per row and direction, each of up to `cols` terms in FP32 in
mode 1, so its first-order relative error is at most about
(2 rows + cols) u32 (u32 = 2^-24); T chains the local solve and one patch
solve per smoothing sweep, so mixed_t_gate = (k + 1) (2 rows + cols) u32
with rows and cols the largest extents of the oversampled boxes and patches.
In 3-D (precision 2) a box recurrence runs over its z-planes and each product
has up to P = bx by terms (the plane), so mixed_t_gate3 = (k + 1)
(2 planes + P) u32 with the largest plane count and plane size.

The interface system C x = g of T is the one step whose conditioning can
exceed what 1e-10 allows (the 1e6-contrast channel field, the sigma = 3
log-normal field at 1024 x 1024).  The oracle solves it accurately (LU plus
refinement with extended-precision residuals), so the difference to the
library is the library's own forward error.  The library scales the rows of
C and factors it by LU with partial pivoting, a backward-stable solve whose
forward error is bounded to first order by cond_S(C) u, with Skeel's
condition number cond_S(C) = || |C^-1| |C| ||_inf (unchanged by any row
scaling, so it measures C and not the scale of its rows) and u = 2^-53.  The
gate for T and for FP64 solutions is that bound times the dimension factor
GATE_FACTOR (the rounding steps of a solve add up over its elimination
levels), and never below 1e-10.  cond_S is exact (dense) for small systems
and estimated with scipy's 1-norm estimator (onenormest of diag(v) C^-T,
v = |C| 1, whose 1-norm is || |C^-1| v ||_inf) for large ones.
"""
import numpy as np
import scipy.sparse.linalg as spla

FP64_GATE = 1e-10
MIXED_GATE = 1e-7
UNIT_ROUNDOFF = 2.0 ** -53
UNIT_ROUNDOFF_32 = 2.0 ** -24
GATE_FACTOR = 16.0
DENSE_COND_MAX = 4000


def skeel_condition(mr) -> float:
    C = mr.C
    n = C.shape[0]
    if n == 0:
        return 1.0
    v = np.asarray(abs(C).sum(axis=1)).ravel()
    if n <= DENSE_COND_MAX:
        Ci = np.linalg.inv(C.toarray())
        return float(np.max(np.abs(Ci) @ v))
    lu = spla.splu(C.tocsc())
    op = spla.LinearOperator((n, n), matvec=lambda x: v * lu.solve(np.ravel(x), trans="T"),
                             rmatvec=lambda y: lu.solve(v * np.ravel(y)), dtype=float)
    return float(spla.onenormest(op))


def t_gate(mr) -> float:
    if mr.part.nc == 0:
        return FP64_GATE
    return max(FP64_GATE, GATE_FACTOR * skeel_condition(mr) * UNIT_ROUNDOFF)


def mixed_t_gate(mr) -> float:
    P = mr.part
    boxes = list(P.oboxes) + (list(P.pboxes) if mr.sweeps > 0 else [])
    rows = max(int(b[3] - b[2]) for b in boxes)
    cols = max(int(b[1] - b[0]) for b in boxes)
    return (mr.sweeps + 1) * (2 * rows + cols) * UNIT_ROUNDOFF_32


def mixed_t_gate3(mr) -> float:
    P = mr.part
    boxes = list(P.oboxes) + (list(P.pboxes) if mr.sweeps > 0 else [])
    planes = max(int(b[5] - b[4]) for b in boxes)
    plane = max(int((b[1] - b[0]) * (b[3] - b[2])) for b in boxes)
    return (mr.sweeps + 1) * (2 * planes + plane) * UNIT_ROUNDOFF_32
