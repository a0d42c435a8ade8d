"""Parity gates shared by the test modules.

FP64 gate: relative L2 1e-10.  When the oracle's interface matrix C is
ill-conditioned (the 1e6-contrast channel field: cond(C) ~ 1e9 - 1e12), two
FP64 implementations that sum in different orders can differ by up to the
first-order forward-error bound cond(C) * 2^-53 of the interface solve; the
gate is then that bound (never below 1e-10).
"""
import numpy as np

FP64_GATE = 1e-10
UNIT_ROUNDOFF = 2.0 ** -53


def t_gate(mr) -> float:
    if mr.part.nc == 0:
        return FP64_GATE
    return max(FP64_GATE, float(np.linalg.cond(mr.C.toarray())) * UNIT_ROUNDOFF)
