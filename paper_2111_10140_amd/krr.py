"""Kernel ridge regression end to end on the fast ANOVA product.

``KernelRidge`` follows the paper's classifier: features are z-scored with
training statistics (Sec. 6), ranked by mutual information score and grouped
into windows of three (Sec. 5, weights 1/P), the coefficients solve
(K + lambda I) alpha = y by CG (Sec. 2) with the fast product (Sec. 4.3), and
new points are evaluated by the fast sum over the training points (Sec. 4.2,
Sec. 4.3); class labels in {-1, 1} are the sign of that sum.

``grid_search`` runs the paper's parameter search (Sec. 6: kernel width
sigma and regularisation lambda on a grid, accuracy on held-out data): one
plan per sigma, one shifted-CG solve for every lambda of the grid, and one
multi-column prediction.

Every product and solve runs in the HIP library; this module only moves
arrays and chooses parameters.
"""
from __future__ import annotations

import time
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import _lib as A
from . import features as F


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _windows_of(Xs: np.ndarray, y: np.ndarray, threshold: float, windows):
    if windows is not None:
        return [(tuple(w[0]), float(w[1])) for w in windows]
    wins = F.group_windows(F.mis_scores(Xs, y), threshold)
    if not wins:
        raise ValueError("no feature reaches the MIS threshold")
    return wins


class KernelRidge:
    """Fast-summation kernel ridge regression (the paper's NFFT-based
    classifier).  sigma: Gaussian width on z-scored features; lam: the
    regularisation parameter; threshold: MIS cut-off (0 keeps every
    feature); tol: CG tolerance (the paper uses 1e-3)."""

    def __init__(self, sigma: float = 1.0, lam: float = 1.0, threshold: float = 0.0,
                 precision: int = A.ANOVA_FP32_NFFT, target_err: float = 1e-4,
                 tol: float = 1e-3, maxit: int = 5000, windows=None, scale: bool = True):
        self.sigma, self.lam, self.threshold = float(sigma), float(lam), float(threshold)
        self.precision, self.target_err = precision, float(target_err)
        self.tol, self.maxit = float(tol), int(maxit)
        self.windows_in, self.scale = windows, scale

    def _params(self):
        return A.make_params(self.sigma, self.precision, target_err=self.target_err)

    def fit(self, X: np.ndarray, y: np.ndarray) -> "KernelRidge":
        X = np.asarray(X, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        if self.scale:
            self.mean_, self.std_ = F.zscore_fit(X)
            Xs = F.zscore_apply(X, self.mean_, self.std_)
        else:
            Xs = np.ascontiguousarray(X)
        self.windows_ = _windows_of(Xs, y, self.threshold, self.windows_in)
        self.X_ = Xs
        plan = A.anova_fastsum_plan(_dev(Xs), self.windows_, self._params())
        self.alpha_ = _dev(np.zeros(Xs.shape[0]))
        self.fit_info_ = A.krr_cg_solve(plan, _dev(y), self.alpha_, self.lam, self.tol,
                                        self.maxit, allow_not_converged=True)[0]
        plan.destroy()
        return self

    def _scaled(self, Z):
        Z = np.asarray(Z, dtype=np.float64)
        return F.zscore_apply(Z, self.mean_, self.std_) if self.scale else np.ascontiguousarray(Z)

    def decision_function(self, Z: np.ndarray) -> np.ndarray:
        """s(z_i) = sum_j alpha_j kappa(z_i, x_j) at the rows of Z."""
        import torch
        Zs = self._scaled(Z)
        plan = A.anova_predict_plan(_dev(self.X_), _dev(Zs), self.windows_, self._params())
        out = torch.empty(Zs.shape[0], dtype=torch.float64, device="cuda")
        A.anova_predict(plan, self.alpha_, out)
        torch.cuda.synchronize()
        plan.destroy()
        return out.cpu().numpy()

    def predict(self, Z: np.ndarray) -> np.ndarray:
        """Class labels in {-1, 1}: the sign of the decision function."""
        return np.where(self.decision_function(Z) >= 0.0, 1.0, -1.0)


def grid_search(X: np.ndarray, y: np.ndarray, Xval: np.ndarray, yval: np.ndarray,
                sigmas: Sequence[float], lambdas: Sequence[float], threshold: float = 0.0,
                precision: int = A.ANOVA_FP32_NFFT, target_err: float = 1e-4,
                tol: float = 1e-3, maxit: int = 5000) -> Dict:
    """Accuracy of sign predictions on (Xval, yval) for every (sigma, lambda)
    of the grid.  Features are z-scored with the training statistics and
    grouped once (the MIS ranking does not depend on sigma or lambda).  Per
    sigma: one prediction plan over the training and validation points, one
    shifted-CG solve for all lambdas, one prediction with a column per
    lambda.  A sigma whose plan cannot meet target_err (too narrow a kernel
    for the largest bandwidth) is reported as infeasible."""
    import torch
    X = np.asarray(X, dtype=np.float64)
    mean, std = F.zscore_fit(X)
    Xs, Vs = F.zscore_apply(X, mean, std), F.zscore_apply(Xval, mean, std)
    windows = _windows_of(Xs, np.asarray(y, dtype=np.float64), threshold, None)
    Xd, Vd, yd = _dev(Xs), _dev(Vs), _dev(y)
    lams = [float(v) for v in lambdas]
    table: List[Dict] = []
    for sg in sigmas:
        t0 = time.perf_counter()
        try:
            plan = A.anova_predict_plan(Xd, Vd, windows,
                                        A.make_params(float(sg), precision,
                                                      target_err=target_err))
        except A.AnovaError as e:
            table.append(dict(sigma=float(sg), feasible=False, reason=str(e)))
            continue
        alphas = torch.empty((len(lams), Xs.shape[0]), dtype=torch.float64, device="cuda").T
        info = A.krr_cg_solve_shifts(plan, yd, alphas, lams, tol, maxit,
                                     allow_not_converged=True)
        out = torch.empty((len(lams), Vs.shape[0]), dtype=torch.float64, device="cuda").T
        A.anova_predict(plan, alphas, out)
        torch.cuda.synchronize()
        s = out.cpu().numpy()
        plan.destroy()
        for k, lam in enumerate(lams):
            acc = float(np.mean(np.where(s[:, k] >= 0.0, 1.0, -1.0) == yval))
            table.append(dict(sigma=float(sg), lam=lam, feasible=True, accuracy=acc,
                              iters=info[k]["iters"], converged=info[k]["converged"]))
        table[-1]["sigma_seconds"] = time.perf_counter() - t0
    feas = [r for r in table if r.get("feasible")]
    best = max(feas, key=lambda r: r["accuracy"]) if feas else None
    return dict(best=best, table=table, windows=windows, mean=mean, std=std)
