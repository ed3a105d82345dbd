"""Left-preconditioned restarted GMRES (oracle). Test infrastructure only.

Sec. 3.2 solves P^{-1} G dU = P^{-1} R with GMRES; the tolerance of Table 1 is
max(1e-12, 1e-8 |R~|). GMRES itself: Saad & Schultz (1986); the Arnoldi basis
is orthogonalised by classical Gram-Schmidt applied twice (Giraud, Langou,
Rozloznik 2005), the least-squares problem is reduced by Givens rotations and
the stopping test uses the preconditioned residual norm |g_{j+1}|.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresInfo:
    iterations: int = 0
    converged: bool = False
    residuals: list = field(default_factory=list)   # preconditioned residual norms


def gmres(apply_A, apply_Minv, b, tol, restart=30, maxit=300):
    """Solve A x = b with left preconditioner Minv, x0 = 0."""
    n = b.size
    x = np.zeros(n)
    info = GmresInfo()
    r = apply_Minv(b)
    beta = np.linalg.norm(r)
    info.residuals.append(beta)
    if beta <= tol:
        info.converged = True
        return x, info
    while info.iterations < maxit:
        V = np.zeros((restart + 1, n))
        Hm = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        resid = beta
        for j in range(restart):
            w = apply_Minv(apply_A(V[j]))
            h1 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h1
            h2 = V[:j + 1] @ w
            w = w - V[:j + 1].T @ h2
            h = h1 + h2
            hn = np.linalg.norm(w)
            # previous rotations
            for i in range(j):
                t = cs[i] * h[i] + sn[i] * h[i + 1]
                h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1]
                h[i] = t
            denom = np.hypot(h[j], hn)
            cs[j] = h[j] / denom
            sn[j] = hn / denom
            h[j] = denom
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            Hm[:j + 1, j] = h
            resid = abs(g[j + 1])
            info.iterations += 1
            info.residuals.append(resid)
            j_done = j + 1
            if hn > 0:
                V[j + 1] = w / hn
            if resid <= tol or info.iterations >= maxit or hn == 0:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - Hm[i, i + 1:j_done] @ y[i + 1:]) / Hm[i, i]
        x = x + V[:j_done].T @ y
        if resid <= tol:
            info.converged = True
            break
        r = apply_Minv(b - apply_A(x))
        beta = np.linalg.norm(r)
        if beta <= tol:
            info.converged = True
            break
    return x, info
