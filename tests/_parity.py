"""Shared helpers for GPU-vs-oracle parity tests (error metrics, transfers).

Tolerances (FP32 arithmetic against the FP64 oracle):
  eps_x = max over systems of ||x_gpu - x_ora||_2 / ||x_ora||_2   <= 1e-4
  eps_L = max over (user, rhs) of max_b |L_gpu - L_ora| / max(1, max_b |L_ora|) <= 1e-3
Precoded vectors use eps_x's definition per vector (over antennas).
"""
import numpy as np

TOL_X = 1e-4
TOL_L = 1e-3


def dev(x, dtype=None):
    import torch
    a = np.ascontiguousarray(x)
    if np.iscomplexobj(a):
        a = a.astype(np.complex64)
    elif dtype is not None:
        a = a.astype(dtype)
    return torch.from_numpy(a).cuda()


def host(t):
    return t.detach().cpu().numpy()


def rel_err_vec(x_gpu, x_ora, axis):
    """max over vectors of the relative 2-norm error along ``axis``."""
    num = np.linalg.norm(np.asarray(x_gpu, dtype=np.complex128) - x_ora, axis=axis)
    den = np.linalg.norm(x_ora, axis=axis)
    ok = den > 0
    e = np.where(ok, num / np.where(ok, den, 1.0), num)
    return float(np.max(e)) if e.size else 0.0


def llr_err(L_gpu, L_ora):
    d = np.max(np.abs(np.asarray(L_gpu, dtype=np.float64) - L_ora), axis=-1)
    s = np.maximum(1.0, np.max(np.abs(L_ora), axis=-1))
    return float(np.max(d / s)) if d.size else 0.0


def rel_err_scalar(a, b):
    a = np.asarray(a, dtype=np.float64)
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-30))) if a.size else 0.0


def blocked16(q):
    """(n, R, C, 2) 16-bit (re, im) -> blocked (n, R/8, 2, C, 8) as int16."""
    n, R, C, _ = q.shape
    b = q.reshape(n, R // 8, 8, C, 2).transpose(0, 1, 4, 3, 2)
    return np.ascontiguousarray(b).view(np.int16)
