"""Plain conjugate gradients (Hestenes-Stiefel) in numpy float64.

Test infrastructure only.  Solves (K + beta I) alpha = y, the symmetric
positive definite system of Sec. 2, with one product per iteration, no
preconditioner (Sec. 6).  Start x0 = 0; stop when ||r_k||_2 <= tol ||y||_2
or after maxit iterations.  Each right-hand side is solved independently.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List

import numpy as np


@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    relres: float          # recursive residual ||r_k|| / ||y||
    true_relres: float     # ||y - A x|| / ||y|| recomputed at exit
    converged: bool
    history: List[float]


def cg_solve(apply_A: Callable[[np.ndarray], np.ndarray], y: np.ndarray, tol: float,
             maxit: int) -> CGResult:
    y = np.asarray(y, dtype=np.float64)
    ynorm = float(np.linalg.norm(y))
    x = np.zeros_like(y)
    if ynorm == 0.0:
        return CGResult(x, 0, 0.0, 0.0, True, [0.0])
    r = y.copy()
    p = r.copy()
    rho = float(r @ r)
    hist = [1.0]
    it = 0
    converged = False
    while it < maxit:
        q = apply_A(p)
        a = rho / float(p @ q)
        x += a * p
        r -= a * q
        rho_new = float(r @ r)
        it += 1
        hist.append(np.sqrt(rho_new) / ynorm)
        if np.sqrt(rho_new) <= tol * ynorm:
            converged = True
            break
        p = r + (rho_new / rho) * p
        rho = rho_new
    true = float(np.linalg.norm(y - apply_A(x))) / ynorm
    return CGResult(x, it, hist[-1], true, converged, hist)
