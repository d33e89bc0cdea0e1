"""Helpers shared by the GPU tests: device copies in the layouts the C ABI
expects and the error metric ||K~a - K a||_inf / ||a||_1 per column."""
import numpy as np


def torch_mod():
    import torch
    return torch


def dev_rows(a: np.ndarray):
    """(N, d) row-major float64 device tensor."""
    torch = torch_mod()
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def dev_cols(a: np.ndarray):
    """(N,) or (N, nrhs) float64 device tensor, column-major."""
    torch = torch_mod()
    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    t = torch.from_numpy(np.ascontiguousarray(a.T)).cuda()
    return t.T


def empty_cols(N: int, nrhs: int = 1):
    torch = torch_mod()
    if nrhs == 1:
        return torch.empty(N, dtype=torch.float64, device="cuda")
    return torch.empty((nrhs, N), dtype=torch.float64, device="cuda").T


def to_np(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def rel_err(out: np.ndarray, ref: np.ndarray, alpha: np.ndarray) -> float:
    out = out.reshape(ref.shape)
    if ref.ndim == 1:
        return float(np.max(np.abs(out - ref)) / np.abs(alpha).sum())
    return float(np.max(np.max(np.abs(out - ref), axis=0) / np.abs(alpha).sum(axis=0)))
