"""Right-preconditioned restarted GMRES (the paper's Algorithm 1).

Each cycle starts from r_0 = b - A p_0, beta = ||r_0||, v_1 = r_0 / beta.
Inner step j: z_j = T v_j, w = A z_j, modified Gram-Schmidt against
v_1..v_j giving h_{i,j}, then h_{j+1,j} = ||w|| and v_{j+1} = w / h_{j+1,j}.
The least-squares problem min ||beta e_1 - H y|| is solved with Givens
rotations (r = hypot(a, b), c = a / r, s = b / r; the right-hand side becomes
(c g_j, -s g_j)), and p_m = p_0 + Z_m y_m with the stored z_j.

Readings: the estimated residual |g_{j+1}| is tested after every inner step
against rtol * ||b|| (relative tolerance, Section 4 reports ||b - A p||_2 with
tolerance 1e-8); the iteration count is the number of inner steps, i.e. of
applications of T; at the end of a cycle the true residual ||b - A p|| decides
whether to stop or restart; a zero h_{j+1,j} (happy breakdown) ends the cycle.
The Krylov dimension is 10 (Section 4).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresResult:
    p: np.ndarray
    iterations: int
    converged: bool
    restarts: int  # number of cycles started (one pass of Algorithm 1 each)
    est_history: list = field(default_factory=list)
    true_history: list = field(default_factory=list)
    final_relres: float = 0.0


def gmres(A_apply, T_apply, b: np.ndarray, rtol: float = 1e-8, restart: int = 10,
          maxit: int = 300, check_every_step: bool = True, atol: float | None = None
          ) -> GmresResult:
    """``check_every_step=False`` follows Algorithm 1 literally (every cycle
    runs all ``restart`` inner steps unless h_{j+1,j} = 0, and only the true
    residual at the end of a cycle is tested); ``atol`` replaces rtol * ||b||
    by an absolute tolerance."""
    b = np.asarray(b, dtype=np.float64)
    p = np.zeros_like(b)
    bnorm = float(np.linalg.norm(b))
    res = GmresResult(p=p, iterations=0, converged=False, restarts=0)
    if bnorm == 0.0:
        res.converged = True
        return res
    tol = rtol * bnorm if atol is None else float(atol)
    while True:
        r = b - A_apply(p)
        beta = float(np.linalg.norm(r))
        res.true_history.append(beta / bnorm)
        if beta <= tol:
            res.converged = True
            break
        if res.iterations >= maxit:
            break
        res.restarts += 1
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        jj = 0
        for j in range(restart):
            z = T_apply(V[j])
            Z.append(z)
            w = A_apply(z)
            res.iterations += 1
            for i in range(j + 1):
                H[i, j] = float(np.dot(w, V[i]))
                w = w - H[i, j] * V[i]
            hnext = float(np.linalg.norm(w))
            H[j + 1, j] = hnext
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            a, c = H[j, j], H[j + 1, j]
            rr = float(np.hypot(a, c))
            cs[j], sn[j] = a / rr, c / rr
            H[j, j] = rr
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            res.est_history.append(abs(g[j + 1]) / bnorm)
            jj = j + 1
            if hnext == 0.0 or res.iterations >= maxit:
                break
            if check_every_step and abs(g[j + 1]) <= tol:
                break
            V.append(w / hnext)
        y = np.zeros(jj)
        for i in range(jj - 1, -1, -1):
            y[i] = (g[i] - np.dot(H[i, i + 1:jj], y[i + 1:jj])) / H[i, i]
        for i in range(jj):
            p = p + y[i] * Z[i]
    res.p = p
    res.final_relres = res.true_history[-1]
    return res
