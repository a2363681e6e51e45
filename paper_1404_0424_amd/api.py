"""Torch-facing binding of the C ABI: argument marshalling only.

Device memory and streams come from PyTorch; every step of the computation
runs in the library's HIP kernels.  Tensors follow the layouts documented in
include/mimo_cg.h (complex64 tensors, or the blocked 16-bit storage returned
by :func:`convert`).
"""
from __future__ import annotations

import ctypes
import dataclasses
import math

import torch

from . import _lib as L


@dataclasses.dataclass
class Packed16:
    """Complex [n][R][C] array in blocked FP16/BF16 storage (mimo_convert)."""
    data: torch.Tensor     # int16, shape (n, R // 8, 2, C, 8)
    dtype_code: int        # MIMO_C16 or MIMO_CBF16
    n: int
    R: int
    C: int

    @property
    def device(self):
        return self.data.device


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else t.data_ptr()


def _check_c64(t, name, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.complex64:
        raise TypeError(f"{name} must be complex64, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on a GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def _channel(H):
    """(pointer, dtype code, n, B, U) of a complex64 or packed channel."""
    if isinstance(H, Packed16):
        return H.data.data_ptr(), H.dtype_code, H.n, H.R, H.C
    _check_c64(H, "H")
    if H.dim() != 3:
        raise ValueError("H must be (n_sc, B, U)")
    n, B, U = H.shape
    return H.data_ptr(), L.MIMO_C32, n, B, U


def _rhs(Y, code, n, B):
    if isinstance(Y, Packed16):
        if Y.dtype_code != code or Y.n != n or Y.R != B:
            raise ValueError("Y storage must match H (dtype, n_sc, B)")
        return Y.data.data_ptr(), Y.C
    if code != L.MIMO_C32:
        raise ValueError("H is packed 16-bit, so Y must be packed the same way")
    _check_c64(Y, "Y")
    if Y.dim() != 3 or Y.shape[0] != n or Y.shape[1] != B:
        raise ValueError("Y must be (n_sc, B, S)")
    return Y.data_ptr(), Y.shape[2]


def convert(X: torch.Tensor, dtype: str = "f16", stream=None) -> Packed16:
    """Round a complex64 (n, R, C) tensor to blocked FP16 / BF16 storage."""
    _check_c64(X, "X")
    n, R, C = X.shape
    code = {"f16": L.MIMO_C16, "bf16": L.MIMO_CBF16}[dtype]
    out = torch.empty((n, R // 8, 2, C, 8), dtype=torch.int16, device=X.device)
    L.check(L.lib().mimo_convert(X.data_ptr(), out.data_ptr(), code, n, R, C, _stream(stream)))
    return Packed16(out, code, n, R, C)


def gram_mf(H, Y=None, reg: float = 0.0, stream=None):
    """A = H^H H + reg I and b = H^H Y.  Returns (A, b) (b is None without Y)."""
    hp, code, n, B, U = _channel(H)
    yp, S = (None, 1) if Y is None else _rhs(Y, code, n, B)
    dev = H.device
    A = torch.empty((n, U, U), dtype=torch.complex64, device=dev)
    b = None if Y is None else torch.empty((n, U, S), dtype=torch.complex64, device=dev)
    shp = L.shape(B, U, S, 1, n)
    L.check(L.lib().mimo_gram_mf(shp, hp, yp, code, float(reg), A.data_ptr(), _ptr(b),
                                 _stream(stream)))
    return A, b


def _detect_outputs(dev, n, U, S, qam_bits, xhat, mu, sinr, out):
    """Output tensors of a detection call: (dict, llr, xhat, mu, sinr); the
    optional ones are None unless requested or supplied in ``out``."""
    out = {} if out is None else dict(out)
    res = {}

    def get(key, shape, dtype, want):
        if not want and key not in out:
            return None
        t = out.get(key)
        if t is None:
            t = torch.empty(shape, dtype=dtype, device=dev)
        elif tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_contiguous():
            raise ValueError(f"out['{key}'] must be contiguous {dtype} {shape}")
        res[key] = t
        return t

    llr = get("llr", (n, U, S, qam_bits), torch.float32, True)
    xh = get("xhat", (n, U, S), torch.complex64, xhat)
    mu_t = get("mu", (n, U, S), torch.float32, mu)
    sn = get("sinr", (n, U, S), torch.float32, sinr)
    return res, llr, xh, mu_t, sn


def _precode_outputs(H, T, out, qnorm):
    hp, code, n, B, U = _channel(H)
    _check_c64(T, "T")
    if T.dim() != 3 or T.shape[0] != n or T.shape[1] != U:
        raise ValueError("T must be (n_sc, U, S)")
    S = T.shape[2]
    dev = T.device
    Q = torch.empty((n, B, S), dtype=torch.complex64, device=dev) if out is None else out
    if tuple(Q.shape) != (n, B, S) or Q.dtype != torch.complex64:
        raise ValueError("out must be complex64 (n_sc, B, S)")
    qn = torch.empty((n, S), dtype=torch.float32, device=dev) if qnorm else None
    return hp, code, n, B, U, S, Q, qn


def detect_cg(H, Y, n0: float, es: float, K: int, qam_bits: int, sinr_mode: str = "approx",
              scalar_prec: str = "f32", xhat: bool = False, mu: bool = False,
              sinr: bool = False, out=None, stream=None) -> dict:
    """CG soft-output MMSE detection.  Returns a dict with 'llr' and the
    optional 'xhat', 'mu', 'sinr' tensors.  ``out`` may hold preallocated
    tensors under the same keys."""
    hp, code, n, B, U = _channel(H)
    yp, S = _rhs(Y, code, n, B)
    res, llr, xh, mu_t, sn = _detect_outputs(H.device, n, U, S, qam_bits, xhat, mu, sinr, out)
    mode = {"approx": L.MIMO_SINR_APPROX, "exact": L.MIMO_SINR_EXACT}[sinr_mode]
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    shp = L.shape(B, U, S, K, n)
    L.check(L.lib().mimo_detect_cg(shp, hp, yp, code, float(n0), float(es), int(qam_bits), mode,
                                   prec, llr.data_ptr(), _ptr(xh), _ptr(mu_t), _ptr(sn), None, 0,
                                   _stream(stream)))
    return res


def precode_cg(H, T: torch.Tensor, beta: float, K: int, normalize: bool = False,
               scalar_prec: str = "f32", qnorm: bool = True, out=None, stream=None):
    """CG precoding q = H_u v with (G + beta I) v = t.  Returns (Q, qnorm)."""
    hp, code, n, B, U, S, Q, qn = _precode_outputs(H, T, out, qnorm)
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    shp = L.shape(B, U, S, K, n)
    L.check(L.lib().mimo_precode_cg(shp, hp, T.data_ptr(), code, float(beta), int(bool(normalize)),
                                    prec, Q.data_ptr(), _ptr(qn), None, 0, _stream(stream)))
    return Q, qn


def _gram_ptr(frame, n, U):
    """Device pointer of a batched frame's optional cached Gram (5th entry)."""
    if len(frame) < 5 or frame[4] is None:
        return None
    return _gram_arg(frame[4], n, U)


def _gram_arg(G, n, U):
    _check_c64(G, "G")
    if tuple(G.shape) != (n, U, U) or not G.is_contiguous():
        raise ValueError("G must be contiguous complex64 (n_sc, U, U)")
    return G.data_ptr()


def detect_cg_gram(G, H, Y, n0: float, es: float, K: int, qam_bits: int,
                   scalar_prec: str = "f32", xhat: bool = False, mu: bool = False,
                   sinr: bool = False, out=None, stream=None) -> dict:
    """detect_cg (approximate SINR) with the channel's Gram matrix G = H^H H
    supplied (e.g. gram_mf(H, None, 0.0), kept while the channel holds): the
    call reads H only for the matched filter."""
    hp, code, n, B, U = _channel(H)
    yp, S = _rhs(Y, code, n, B)
    gp = _gram_arg(G, n, U)
    res, llr, xh, mu_t, sn = _detect_outputs(H.device, n, U, S, qam_bits, xhat, mu, sinr, out)
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    L.check(L.lib().mimo_detect_cg_gram(L.shape(B, U, S, K, n), gp, hp, yp, code, float(n0),
                                        float(es), int(qam_bits), prec, llr.data_ptr(), _ptr(xh),
                                        _ptr(mu_t), _ptr(sn), _stream(stream)))
    return res


def precode_cg_gram(G, H, T: torch.Tensor, beta: float, K: int, normalize: bool = False,
                    scalar_prec: str = "f32", qnorm: bool = True, out=None, stream=None):
    """precode_cg with the channel's Gram matrix G supplied; H is read only
    for q = H v.  Returns (Q, qnorm)."""
    hp, code, n, B, U, S, Q, qn = _precode_outputs(H, T, out, qnorm)
    gp = _gram_arg(G, n, U)
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    L.check(L.lib().mimo_precode_cg_gram(L.shape(B, U, S, K, n), gp, hp, T.data_ptr(), code,
                                         float(beta), int(bool(normalize)), prec, Q.data_ptr(),
                                         _ptr(qn), _stream(stream)))
    return Q, qn


def detect_precode_cg(H, Y, T: torch.Tensor, n0: float, es: float, beta: float, K_ul: int,
                      K_dl: int, qam_bits: int, normalize: bool = False,
                      scalar_prec: str = "f32", xhat: bool = False, mu: bool = False,
                      sinr: bool = False, qnorm: bool = True, out=None, stream=None):
    """One uplink + downlink slot on the reciprocal channel H: detect_cg of Y
    (approximate SINR) and precode_cg of T with one shared Gram matrix per
    subcarrier.  Returns (detection dict, Q, qnorm); ``out`` may hold
    preallocated tensors under the keys of both ('llr', 'xhat', 'mu', 'sinr',
    'Q', 'qnorm')."""
    hp, code, n, B, U = _channel(H)
    yp, Su = _rhs(Y, code, n, B)
    out = out or {}
    res, llr, xh, mu_t, sn = _detect_outputs(H.device, n, U, Su, qam_bits, xhat, mu, sinr,
                                             {k: v for k, v in out.items()
                                              if k in ("llr", "xhat", "mu", "sinr")} or None)
    _, _, _, _, _, Sd, Q, qn = _precode_outputs(H, T, out.get("Q"), qnorm)
    if "qnorm" in out and out["qnorm"] is not None:
        qn = out["qnorm"]
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    L.check(L.lib().mimo_detect_precode_cg(L.shape(B, U, Su, K_ul, n), L.shape(B, U, Sd, K_dl, n),
                                           hp, yp, T.data_ptr(), code, float(n0), float(es),
                                           int(qam_bits), float(beta), int(bool(normalize)), prec,
                                           llr.data_ptr(), _ptr(xh), _ptr(mu_t), _ptr(sn),
                                           Q.data_ptr(), _ptr(qn), _stream(stream)))
    return res, Q, qn


def workspace_bytes(B, U, S, K, n_sc, op: str = "detect", sinr_mode: str = "approx") -> int:
    opc = {"gram_mf": L.MIMO_OP_GRAM_MF, "detect": L.MIMO_OP_DETECT,
           "precode": L.MIMO_OP_PRECODE, "slot": L.MIMO_OP_SLOT}[op]
    mode = {"approx": L.MIMO_SINR_APPROX, "exact": L.MIMO_SINR_EXACT}[sinr_mode]
    return int(L.lib().mimo_workspace_bytes(L.shape(B, U, S, K, n_sc), opc, mode))


def _views(dev, dtype, shapes):
    """One allocation for a batch's outputs; a view of it per shape (each
    starting on a 64-element boundary)."""
    sizes = [math.prod(s) for s in shapes]
    offs = [0]
    for z in sizes:
        offs.append(offs[-1] + (z + 63) // 64 * 64)
    buf = torch.empty(offs[-1], dtype=dtype, device=dev)
    return [buf[o:o + z].view(s) for o, z, s in zip(offs, sizes, shapes)]


def detect_cg_batch(frames, K: int | list, qam_bits: int, scalar_prec: str = "f32",
                    xhat: bool = False, stream=None) -> list[dict]:
    """Detect up to MIMO_MAX_BATCH frames of different shapes in one launch.
    ``frames`` is a list of (H, Y, n0, es) or (H, Y, n0, es, G) with the same
    storage type (G: the frame's cached Gram matrix, as detect_cg_gram takes
    it); K is one value or one per frame.  Returns one output dict per frame
    (views of one allocation per output kind)."""
    if not frames:
        return []
    Ks = K if isinstance(K, (list, tuple)) else [K] * len(frames)
    arr = (L.MimoFrame * len(frames))()
    code0, dims = None, []
    for fr in frames:
        H, Y = fr[0], fr[1]
        hp, code, n, B, U = _channel(H)
        if code0 is None:
            code0 = code
        elif code != code0:
            raise ValueError("all frames of a batch need the same storage type")
        yp, S = _rhs(Y, code, n, B)
        dims.append((hp, yp, n, B, U, S))
    dev = frames[0][0].device
    llrs = _views(dev, torch.float32, [(n, U, S, qam_bits) for _, _, n, _, U, S in dims])
    xhs = (_views(dev, torch.complex64, [(n, U, S) for _, _, n, _, U, S in dims]) if xhat
           else [None] * len(frames))
    outs = []
    for i, ((hp, yp, n, B, U, S), fr, k) in enumerate(zip(dims, frames, Ks)):
        n0, es = fr[2], fr[3]
        arr[i] = L.MimoFrame(n, B, U, S, int(k), hp, yp, llrs[i].data_ptr(), _ptr(xhs[i]),
                             float(n0), float(es), 0.0, 0, _gram_ptr(fr, n, U))
        outs.append({"llr": llrs[i], "xhat": xhs[i]} if xhat else {"llr": llrs[i]})
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    L.check(L.lib().mimo_detect_cg_batch(ctypes.addressof(arr), len(frames), code0,
                                         int(qam_bits), prec, _stream(stream)))
    return outs


def precode_cg_batch(frames, K: int | list, scalar_prec: str = "f32", qnorm: bool = False,
                     stream=None) -> list[tuple]:
    """Precode up to MIMO_MAX_BATCH frames in one launch.  ``frames`` is a
    list of (H, T, beta, normalize) or (H, T, beta, normalize, G) (G: the
    frame's cached Gram matrix).  Returns (Q, qnorm) per frame (views of one
    allocation per output kind)."""
    if not frames:
        return []
    Ks = K if isinstance(K, (list, tuple)) else [K] * len(frames)
    arr = (L.MimoFrame * len(frames))()
    code0, dims = None, []
    for fr in frames:
        H, T = fr[0], fr[1]
        hp, code, n, B, U = _channel(H)
        if code0 is None:
            code0 = code
        elif code != code0:
            raise ValueError("all frames of a batch need the same storage type")
        _check_c64(T, "T")
        if T.dim() != 3 or T.shape[0] != n or T.shape[1] != U:
            raise ValueError(f"T shape {tuple(T.shape)} does not match H ({n}, {B}, {U})")
        dims.append((hp, n, B, U, T.shape[2]))
    dev = frames[0][1].device
    Qs = _views(dev, torch.complex64, [(n, B, S) for _, n, B, _, S in dims])
    qns = (_views(dev, torch.float32, [(n, S) for _, n, _, _, S in dims]) if qnorm
           else [None] * len(frames))
    outs = []
    for i, ((hp, n, B, U, S), fr, k) in enumerate(zip(dims, frames, Ks)):
        T, beta, normalize = fr[1], fr[2], fr[3]
        arr[i] = L.MimoFrame(n, B, U, S, int(k), hp, T.data_ptr(), Qs[i].data_ptr(),
                             _ptr(qns[i]), 0.0, 0.0, float(beta), int(bool(normalize)),
                             _gram_ptr(fr, n, U))
        outs.append((Qs[i], qns[i]))
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    L.check(L.lib().mimo_precode_cg_batch(ctypes.addressof(arr), len(frames), code0, prec,
                                          _stream(stream)))
    return outs


# ---------------------------------------------------------------- Sec. III-F

def _detect_inverse(fn, H, Y, n0, es, K, qam_bits, xhat, mu, sinr, out, stream):
    hp, code, n, B, U = _channel(H)
    yp, S = _rhs(Y, code, n, B)
    res, llr, xh, mu_t, sn = _detect_outputs(H.device, n, U, S, qam_bits, xhat, mu, sinr, out)
    L.check(fn(L.shape(B, U, S, K, n), hp, yp, code, float(n0), float(es), int(qam_bits),
               llr.data_ptr(), _ptr(xh), _ptr(mu_t), _ptr(sn), _stream(stream)))
    return res


def detect_cholesky(H, Y, n0: float, es: float, qam_bits: int, xhat: bool = False,
                    mu: bool = False, sinr: bool = False, out=None, stream=None) -> dict:
    """Exact soft-output MMSE detection through the Cholesky factorization
    of A (the paper's reference detector).  Same outputs as detect_cg."""
    return _detect_inverse(L.lib().mimo_detect_cholesky, H, Y, n0, es, 1, qam_bits, xhat, mu,
                           sinr, out, stream)


def detect_neumann(H, Y, n0: float, es: float, K: int, qam_bits: int, xhat: bool = False,
                   mu: bool = False, sinr: bool = False, out=None, stream=None) -> dict:
    """Soft-output detection with the K-term Neumann-series inverse."""
    return _detect_inverse(L.lib().mimo_detect_neumann, H, Y, n0, es, K, qam_bits, xhat, mu,
                           sinr, out, stream)


def _precode_inverse(fn, H, T, beta, K, normalize, qnorm, out, stream):
    hp, code, n, B, U, S, Q, qn = _precode_outputs(H, T, out, qnorm)
    L.check(fn(L.shape(B, U, S, K, n), hp, T.data_ptr(), code, float(beta), int(bool(normalize)),
               Q.data_ptr(), _ptr(qn), _stream(stream)))
    return Q, qn


def precode_cholesky(H, T: torch.Tensor, beta: float, normalize: bool = False,
                     qnorm: bool = True, out=None, stream=None):
    """Exact MMSE (beta > 0) or ZF (beta = 0) precoding through the
    Cholesky factorization.  Returns (Q, qnorm)."""
    return _precode_inverse(L.lib().mimo_precode_cholesky, H, T, beta, 1, normalize, qnorm, out,
                            stream)


def precode_neumann(H, T: torch.Tensor, beta: float, K: int, normalize: bool = False,
                    qnorm: bool = True, out=None, stream=None):
    """Precoding with the K-term Neumann-series inverse.  Returns (Q, qnorm)."""
    return _precode_inverse(L.lib().mimo_precode_neumann, H, T, beta, K, normalize, qnorm, out,
                            stream)


# ---------------------------------------------------------------- Sec. III-E

def detect_cgls(H, Y, n0: float, es: float, K: int, qam_bits: int, scalar_prec: str = "f32",
                xhat: bool = False, mu: bool = False, sinr: bool = False, out=None,
                stream=None) -> dict:
    """K CGLS iterations on the augmented uplink system (no Gram matrix),
    approximate in-loop SINR.  Same outputs as detect_cg."""
    hp, code, n, B, U = _channel(H)
    yp, S = _rhs(Y, code, n, B)
    res, llr, xh, mu_t, sn = _detect_outputs(H.device, n, U, S, qam_bits, xhat, mu, sinr, out)
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    L.check(L.lib().mimo_detect_cgls(L.shape(B, U, S, K, n), hp, yp, code, float(n0), float(es),
                                     int(qam_bits), prec, llr.data_ptr(), _ptr(xh), _ptr(mu_t),
                                     _ptr(sn), _stream(stream)))
    return res


def precode_cgls(H, T: torch.Tensor, beta: float, K: int, normalize: bool = False,
                 scalar_prec: str = "f32", qnorm: bool = True, out=None, stream=None):
    """K CGLS iterations on the augmented downlink system.  Returns (Q, qnorm)."""
    hp, code, n, B, U, S, Q, qn = _precode_outputs(H, T, out, qnorm)
    prec = {"f32": L.MIMO_SCALAR_F32, "f64": L.MIMO_SCALAR_F64}[scalar_prec]
    L.check(L.lib().mimo_precode_cgls(L.shape(B, U, S, K, n), hp, T.data_ptr(), code, float(beta),
                                      int(bool(normalize)), prec, Q.data_ptr(), _ptr(qn),
                                      _stream(stream)))
    return Q, qn
