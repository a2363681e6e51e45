"""FP64 CPU oracle for CG soft-output MMSE detection and CG precoding.

TEST INFRASTRUCTURE ONLY.  This module is the correctness reference for the
GPU library.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it; the product path never calls it and shares no
code with it (it does not import the package, and the package does not import
it).  Everything here is plain numpy in complex128/float64, written from the
paper ("Conjugate Gradient-based Soft-Output Detection and Precoding in
Massive MIMO Systems", Yin, Wu, Cavallaro, Studer), with each function citing
the passage it follows.

Array conventions (same as the C ABI, row-major):
  H (n, B, U)   uplink channel H_u;   H_d = H_u^H (reciprocity, Sec. II-B)
  Y (n, B, S)   receive vectors as columns;  T (n, U, S) downlink symbols
  A (n, U, U)   regularized Gram;  b (n, U, S) CG right-hand sides
  xhat, mu, rho (n, U, S);  llr (n, U, S, m);  Q (n, B, S);  qnorm (n, S)

Readings of the paper taken here (each is listed with its reason in the
design notes of the repository):
  * Gram symmetry: G is formed from its upper triangle and a real diagonal,
    mirrored to the lower triangle.
  * Zero residual: if ||r_{k-1}||^2 == 0 the system has converged (or b = 0);
    alpha_k = beta_k = 0 and every vector and tracker freezes.
  * Zero right-hand side: mu = 0 gives z = 0 and rho_i = G_ii / N0.
  * L_1 = alpha_1 I is set explicitly; the three-term recursions (12)/(13)
    run for k >= 2 (applied at k = 1 they would give 0).
  * Constellation: square Gray QAM, per-axis Gray labels, I bits before Q
    bits, MSB first, average energy E_s; LLR sign exactly as in eq. (4).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "gram", "regularized_gram", "matched_filter", "cg", "CGTrace",
    "approx_tracker_shadow", "approx_tracker_three_term",
    "cg_polynomial_coeffs", "exact_tracker_shadow", "exact_tracker_three_term",
    "exact_sinr", "qam_constellation", "llr_maxlog_bruteforce",
    "llr_maxlog_separable", "ml_maxlog_bruteforce", "detect_cg",
    "precode_cg", "cholesky", "cholesky_solve", "cholesky_inverse",
    "mmse_exact", "precode_mmse_exact", "quantize_f16", "quantize_bf16",
    "linear_soft_output", "detect_cholesky", "precode_cholesky", "neumann_inverse",
    "detect_neumann", "precode_neumann", "cgls", "CGLSTrace", "augment_uplink",
    "augment_downlink", "detect_cgls", "precode_cgls",
]


# --------------------------------------------------------------------------
# Gram matrix and matched filter (Alg. 1 initialization; eq. (8))
# --------------------------------------------------------------------------

def gram(H: np.ndarray) -> np.ndarray:
    """G = H^H H per subcarrier (Sec. III-C), upper triangle mirrored."""
    H = np.asarray(H, dtype=np.complex128)
    G = np.conj(np.swapaxes(H, -1, -2)) @ H
    U = G.shape[-1]
    iu = np.triu_indices(U, 1)
    Gh = np.zeros_like(G)
    Gh[..., iu[0], iu[1]] = G[..., iu[0], iu[1]]
    Gh = Gh + np.conj(np.swapaxes(Gh, -1, -2))
    d = np.arange(U)
    Gh[..., d, d] = G[..., d, d].real
    return Gh


def regularized_gram(H: np.ndarray, reg: float) -> np.ndarray:
    """A = H^H H + reg I (detection: reg = N0/E_s, eq. (8); precoding:
    A = H_d H_d^H + reg I = G + reg I by reciprocity, Alg. 1 / eq. (16))."""
    G = gram(H)
    U = G.shape[-1]
    return G + reg * np.eye(U)


def matched_filter(H: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """b = H^H y for every column of Y (Alg. 1 initialization, detection)."""
    H = np.asarray(H, dtype=np.complex128)
    return np.conj(np.swapaxes(H, -1, -2)) @ np.asarray(Y, dtype=np.complex128)


# --------------------------------------------------------------------------
# Conjugate gradient (Algorithm 1)
# --------------------------------------------------------------------------

@dataclasses.dataclass
class CGTrace:
    v: np.ndarray          # (n, U, S)  v_K
    alpha: np.ndarray      # (K, n, S)  alpha_1..alpha_K
    beta: np.ndarray       # (K, n, S)  beta_1..beta_K
    iterates: list         # [v_0, v_1, ..., v_K]
    residuals: list        # [r_0, ..., r_K]


def cg(A: np.ndarray, b: np.ndarray, K: int) -> CGTrace:
    """Algorithm 1 run independently for every column of b.

    v_0 = 0, r_0 = p_0 = b; for k = 1..K:
      e = A p;  alpha = ||r||^2 / (p^H e);  v += alpha p;  r -= alpha e;
      beta = ||r_new||^2 / ||r_old||^2;  p = r + beta p.
    p^H e is real for Hermitian A, so its real part is taken.  A zero
    ||r_{k-1}||^2 freezes the column (alpha = beta = 0).
    """
    A = np.asarray(A, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    n, U, S = b.shape
    v = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.sum(np.abs(r) ** 2, axis=-2)                     # (n, S)
    alphas = np.zeros((K, n, S))
    betas = np.zeros((K, n, S))
    iterates = [v.copy()]
    residuals = [r.copy()]
    for k in range(K):
        e = A @ p
        pe = np.sum(np.conj(p) * e, axis=-2).real
        live = rr > 0.0
        alpha = np.where(live, rr / np.where(live, pe, 1.0), 0.0)
        v = v + alpha[:, None, :] * p
        r = r - alpha[:, None, :] * e
        rr_new = np.sum(np.abs(r) ** 2, axis=-2)
        beta = np.where(live, rr_new / np.where(live, rr, 1.0), 0.0)
        p = np.where(live[:, None, :], r + beta[:, None, :] * p, p)
        rr = np.where(live, rr_new, rr)
        alphas[k] = alpha
        betas[k] = beta
        iterates.append(v.copy())
        residuals.append(r.copy())
    return CGTrace(v=v, alpha=alphas, beta=betas, iterates=iterates,
                   residuals=residuals)


# --------------------------------------------------------------------------
# Approximate SINR tracker (Sec. III-C-2, eqs. (13)-(15))
# --------------------------------------------------------------------------

def approx_tracker_shadow(d: np.ndarray, alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Diagonal of L~_K from recursion (13) with A replaced by D = diag(A).

    Because every matrix in (13) is diagonal, entry i follows the same
    two-term recursion as CG itself on the scalar d_i with the CG's own
    alpha_k, beta_k:  v~_0 = 0, r~_0 = p~_0 = 1,
      v~_k = v~_{k-1} + alpha_k p~_{k-1},  r~_k = r~_{k-1} - alpha_k d_i p~_{k-1},
      p~_k = r~_k + beta_k p~_{k-1},
    and L~_{ii|k} = v~_k.  Eliminating r~ and p~ gives (13) exactly (the same
    steps that turn Algorithm 1 into (12)).  d: (n, U); alpha, beta: (K, n, S).
    Returns (n, U, S).
    """
    K, n, S = alpha.shape
    U = d.shape[-1]
    vt = np.zeros((n, U, S))
    rt = np.ones((n, U, S))
    pt = np.ones((n, U, S))
    for k in range(K):
        a = alpha[k][:, None, :]
        bb = beta[k][:, None, :]
        vt = vt + a * pt
        rt = rt - a * d[:, :, None] * pt
        pt = rt + bb * pt
    return vt


def approx_tracker_three_term(d: np.ndarray, alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Diagonal of L~_K by the paper's three-term recursion (13) verbatim.

    L~_1 = alpha_1 I;  L~_k = 0, alpha_k = 1, beta_k = 0 for k < 1; for k >= 2
      L~_k = L~_{k-1} + (alpha_k (1+beta_{k-1})/alpha_{k-1} I - alpha_k D)(L~_{k-1} - L~_{k-2})
             - alpha_k beta_{k-2}/alpha_{k-2} (L~_{k-2} - L~_{k-3}).
    Divides by alpha_{k-1}, alpha_{k-2}, so it is only used where no column
    has frozen (all alpha != 0).
    """
    K, n, S = alpha.shape
    U = d.shape[-1]
    dd = d[:, :, None]

    def al(k):
        return alpha[k - 1][:, None, :] if k >= 1 else np.ones((n, 1, S))

    def be(k):
        return beta[k - 1][:, None, :] if k >= 1 else np.zeros((n, 1, S))

    Lm = {0: np.zeros((n, U, S)), -1: np.zeros((n, U, S)), -2: np.zeros((n, U, S))}
    Lm[1] = np.broadcast_to(al(1), (n, U, S)).copy()
    for k in range(2, K + 1):
        Lm[k] = (Lm[k - 1]
                 + (al(k) * (1 + be(k - 1)) / al(k - 1) - al(k) * dd) * (Lm[k - 1] - Lm[k - 2])
                 - al(k) * be(k - 2) / al(k - 2) * (Lm[k - 2] - Lm[k - 3]))
    return Lm[K]


def cg_polynomial_coeffs(alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """Coefficients c_0..c_{K-1} of the CG polynomial P_K with v_K = P_K(A) b.

    Runs Algorithm 1's recursion on polynomials (v, r, p as coefficient
    vectors in powers of A) for one system: alpha, beta are (K,) arrays.
    L_K = P_K(A) is the CG-equivalent matrix of eq. (9) and L~_K = P_K(D).
    """
    K = alpha.shape[0]
    v = np.zeros(K + 1)
    r = np.zeros(K + 1)
    r[0] = 1.0
    p = r.copy()
    for k in range(K):
        v = v + alpha[k] * p
        Ap = np.concatenate([[0.0], p[:-1]])           # multiply by A
        r = r - alpha[k] * Ap
        p = r + beta[k] * p
    return v[:K]


# --------------------------------------------------------------------------
# Exact SINR tracker (Sec. III-C-1, eqs. (9), (12))
# --------------------------------------------------------------------------

def exact_tracker_shadow(A: np.ndarray, alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """L_K with x_K = L_K H^H y (eq. (9)), by the matrix form of Algorithm 1.

    V_0 = 0, R_0 = P_0 = I; V_k = V_{k-1} + alpha_k P_{k-1};
    R_k = R_{k-1} - alpha_k A P_{k-1};  P_k = R_k + beta_k P_{k-1}.
    Since Algorithm 1 is linear in (v, r, p) for given alpha, beta, V_k b = v_k,
    and eliminating R, P gives recursion (12).  A: (n, U, U); alpha, beta:
    (K, n, S).  Returns (n, S, U, U).
    """
    K, n, S = alpha.shape
    U = A.shape[-1]
    I = np.broadcast_to(np.eye(U, dtype=np.complex128), (n, S, U, U))
    V = np.zeros((n, S, U, U), dtype=np.complex128)
    R = I.copy()
    P = I.copy()
    As = A[:, None, :, :]
    for k in range(K):
        a = alpha[k][:, :, None, None]
        bb = beta[k][:, :, None, None]
        V = V + a * P
        R = R - a * (As @ P)
        P = R + bb * P
    return V


def exact_tracker_three_term(A: np.ndarray, alpha: np.ndarray, beta: np.ndarray) -> np.ndarray:
    """L_K by the paper's recursion (12) verbatim (L_1 = alpha_1 I, L_k = 0
    and alpha_k = 1, beta_k = 0 for k < 1).  Only valid when no alpha is 0."""
    K, n, S = alpha.shape
    U = A.shape[-1]
    I = np.eye(U, dtype=np.complex128)
    As = A[:, None, :, :]

    def al(k):
        return alpha[k - 1][:, :, None, None] if k >= 1 else np.ones((n, S, 1, 1))

    def be(k):
        return beta[k - 1][:, :, None, None] if k >= 1 else np.zeros((n, S, 1, 1))

    Z = np.zeros((n, S, U, U), dtype=np.complex128)
    L = {0: Z, -1: Z, -2: Z, 1: al(1) * I}
    for k in range(2, K + 1):
        coef = al(k) * (1 + be(k - 1)) / al(k - 1)
        L[k] = (L[k - 1] + coef * (L[k - 1] - L[k - 2]) - al(k) * (As @ (L[k - 1] - L[k - 2]))
                - al(k) * be(k - 2) / al(k - 2) * (L[k - 2] - L[k - 3]))
    return L[K]


def exact_sinr(L: np.ndarray, G: np.ndarray, es: float, n0: float):
    """mu, nu^2, rho from L_K (Sec. III-C-1).

    B = L_K G, mu_i = B_ii;  C = B L_K^H,
    nu_i^2 = sum_{j != i} |B_ij|^2 E_s + C_ii N0;  rho_i = mu_i^2 / nu_i^2.
    L_K is a real polynomial in the Hermitian A, so B_ii and C_ii are real;
    the real parts are taken.  L: (n, S, U, U), G: (n, U, U).
    Returns mu, nu2, rho as (n, U, S).
    """
    Bm = L @ G[:, None, :, :]
    C = Bm @ np.conj(np.swapaxes(L, -1, -2))
    U = G.shape[-1]
    d = np.arange(U)
    mu = Bm[..., d, d].real                                  # (n, S, U)
    offmask = ~np.eye(U, dtype=bool)
    off = np.sum(np.where(offmask, np.abs(Bm) ** 2, 0.0), axis=-1)
    nu2 = off * es + C[..., d, d].real * n0
    with np.errstate(divide="ignore", invalid="ignore"):
        rho = mu ** 2 / nu2
    return (np.swapaxes(mu, -1, -2), np.swapaxes(nu2, -1, -2),
            np.swapaxes(rho, -1, -2))


# --------------------------------------------------------------------------
# Constellation and max-log LLRs (eq. (4))
# --------------------------------------------------------------------------

def qam_constellation(m: int, es: float = 1.0):
    """All M = 2^m square-QAM points and their bit labels (M, m).

    Per axis: levels 2j-(L-1), j = 0..L-1, L = 2^(m/2), labelled by the Gray
    code j ^ (j >> 1), MSB first; the in-phase label forms bits [0, m/2),
    the quadrature label bits [m/2, m); scaled to average energy es.
    """
    h = m // 2
    L = 1 << h
    j = np.arange(L)
    lev = (2 * j - (L - 1)).astype(np.float64)
    gray = j ^ (j >> 1)
    lab = ((gray[:, None] >> np.arange(h - 1, -1, -1)[None, :]) & 1)   # (L, h)
    M = L * L
    scale = math.sqrt(es * 3.0 / (2.0 * (M - 1)))
    pts = np.empty(M, dtype=np.complex128)
    labels = np.empty((M, m), dtype=np.int8)
    for a in range(L):
        for c in range(L):
            pts[a * L + c] = scale * (lev[a] + 1j * lev[c])
            labels[a * L + c, :h] = lab[a]
            labels[a * L + c, h:] = lab[c]
    return pts, labels


def llr_maxlog_bruteforce(z: np.ndarray, rho: np.ndarray, m: int, es: float = 1.0) -> np.ndarray:
    """Eq. (4): L_b = rho (min_{a in X_b^0} |z - a|^2 - min_{a in X_b^1} |z - a|^2),
    searching all M constellation points.  z, rho: (...); returns (..., m)."""
    pts, labels = qam_constellation(m, es)
    d = np.abs(np.asarray(z)[..., None] - pts) ** 2           # (..., M)
    out = np.empty(np.shape(z) + (m,))
    for bit in range(m):
        d0 = np.min(np.where(labels[:, bit] == 0, d, np.inf), axis=-1)
        d1 = np.min(np.where(labels[:, bit] == 1, d, np.inf), axis=-1)
        out[..., bit] = np.asarray(rho) * (d0 - d1)
    return out


def llr_maxlog_separable(z: np.ndarray, rho: np.ndarray, m: int, es: float = 1.0) -> np.ndarray:
    """Eq. (4) evaluated per axis: for square QAM |z-a|^2 splits into an
    in-phase and a quadrature term, and the term of the other axis is the
    same in both minima, so each bit needs only the sqrt(M) levels of its
    own axis."""
    h = m // 2
    L = 1 << h
    M = L * L
    scale = math.sqrt(es * 3.0 / (2.0 * (M - 1)))
    j = np.arange(L)
    lev = scale * (2 * j - (L - 1))
    gray = j ^ (j >> 1)
    z = np.asarray(z)
    out = np.empty(z.shape + (m,))
    for axis, comp in enumerate((z.real, z.imag)):
        d = (comp[..., None] - lev) ** 2
        for q in range(h):
            bitv = (gray >> (h - 1 - q)) & 1
            d0 = np.min(np.where(bitv == 0, d, np.inf), axis=-1)
            d1 = np.min(np.where(bitv == 1, d, np.inf), axis=-1)
            out[..., axis * h + q] = np.asarray(rho) * (d0 - d1)
    return out


def ml_maxlog_bruteforce(H: np.ndarray, y: np.ndarray, n0: float, m: int, es: float = 1.0) -> np.ndarray:
    """Exact max-log ML LLRs by exhaustive search over O^U (tiny U only):
    L_{i,b} = (min_{x: x_i in X_b^0} ||y - Hx||^2 - min_{x: x_i in X_b^1} ||y - Hx||^2) / N0.
    H: (B, U), y: (B,).  Returns (U, m)."""
    pts, labels = qam_constellation(m, es)
    B, U = H.shape
    M = pts.size
    idx = np.stack(np.meshgrid(*([np.arange(M)] * U), indexing="ij"), -1).reshape(-1, U)
    X = pts[idx]                                              # (M^U, U)
    metric = np.sum(np.abs(y[None, :] - X @ H.T) ** 2, axis=-1) / n0
    out = np.empty((U, m))
    for i in range(U):
        lab = labels[idx[:, i]]
        for bit in range(m):
            out[i, bit] = (np.min(metric[lab[:, bit] == 0])
                           - np.min(metric[lab[:, bit] == 1]))
    return out


# --------------------------------------------------------------------------
# CG-D: soft-output detection (Sec. III-B/C, Algorithm 1)
# --------------------------------------------------------------------------

def detect_cg(H, Y, n0: float, es: float, K: int, m: int, sinr_mode: str = "approx",
              llr_form: str = "bruteforce") -> dict:
    """Soft-output MMSE detection by K CG iterations with in-loop SINR.

    A = H^H H + (N0/E_s) I, b = H^H y (eq. (8)); Algorithm 1 gives
    xhat = v_K; mu, rho by the approximate tracker (eqs. (13)-(15)) or the
    exact one (eq. (12) and the B, C products); z = xhat/mu and the max-log
    LLR of eq. (4).
    """
    H = np.asarray(H, dtype=np.complex128)
    G = gram(H)
    U = G.shape[-1]
    A = G + (n0 / es) * np.eye(U)
    b = matched_filter(H, Y)
    tr = cg(A, b, K)
    xhat = tr.v
    Gii = np.diagonal(G, axis1=-2, axis2=-1).real              # (n, U)
    n, _, S = b.shape
    rho_approx = np.broadcast_to((Gii / n0)[:, :, None], (n, U, S)).copy()
    if sinr_mode == "approx":
        d = np.diagonal(A, axis1=-2, axis2=-1).real
        Lt = approx_tracker_shadow(d, tr.alpha, tr.beta)
        mu = Lt * Gii[:, :, None]                                # eq. (14)
        rho = rho_approx                                         # eq. (15)
    elif sinr_mode == "exact":
        L = exact_tracker_shadow(A, tr.alpha, tr.beta)
        mu, _, rho = exact_sinr(L, G, es, n0)
    else:
        raise ValueError(sinr_mode)
    zero = mu == 0.0
    rho = np.where(zero, rho_approx, rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(zero, 0.0, xhat / np.where(zero, 1.0, mu))
    llr_fn = llr_maxlog_bruteforce if llr_form == "bruteforce" else llr_maxlog_separable
    llr = llr_fn(z, rho, m, es)
    return dict(llr=llr, xhat=xhat, mu=mu, rho=rho, z=z, A=A, b=b, G=G, trace=tr)


# --------------------------------------------------------------------------
# CG-P: precoding (Sec. III-D, eq. (16), Algorithm 1 output)
# --------------------------------------------------------------------------

def precode_cg(H, T, beta: float, K: int, normalize: bool = False) -> dict:
    """Solve (H_d H_d^H + beta I) v = t by K CG iterations, q = H_d^H v.

    With H_d = H_u^H: A = G + beta I and q = H_u v.  beta = 0 is zero
    forcing.  Optionally s = q / ||q||_2 per vector (Sec. II-B); ||q|| = 0
    leaves s = 0.
    """
    H = np.asarray(H, dtype=np.complex128)
    A = regularized_gram(H, beta)
    tr = cg(A, np.asarray(T, dtype=np.complex128), K)
    Q = H @ tr.v
    qnorm = np.sqrt(np.sum(np.abs(Q) ** 2, axis=-2))             # (n, S)
    if normalize:
        Q = np.where(qnorm[:, None, :] > 0, Q / np.where(qnorm > 0, qnorm, 1.0)[:, None, :], 0.0)
    return dict(Q=Q, qnorm=qnorm, v=tr.v, A=A, trace=tr)


# --------------------------------------------------------------------------
# Exact references: Cholesky inversion (Sec. III-F-1)
# --------------------------------------------------------------------------

def cholesky(A: np.ndarray) -> np.ndarray:
    """Lower-triangular M with A = M M^H, column by column (one system)."""
    A = np.asarray(A, dtype=np.complex128)
    U = A.shape[0]
    M = np.zeros_like(A)
    for j in range(U):
        s = A[j, j].real - np.sum(np.abs(M[j, :j]) ** 2)
        if s <= 0.0:
            raise np.linalg.LinAlgError("matrix is not positive definite")
        M[j, j] = math.sqrt(s)
        for i in range(j + 1, U):
            M[i, j] = (A[i, j] - np.sum(M[i, :j] * np.conj(M[j, :j]))) / M[j, j]
    return M


def cholesky_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """A^{-1} b by forward and backward substitution with A = M M^H."""
    M = cholesky(A)
    U = M.shape[0]
    b = np.asarray(b, dtype=np.complex128)
    w = np.zeros_like(b)
    for i in range(U):
        w[i] = (b[i] - M[i, :i] @ w[:i]) / M[i, i]
    x = np.zeros_like(b)
    MH = np.conj(M.T)
    for i in range(U - 1, -1, -1):
        x[i] = (w[i] - MH[i, i + 1:] @ x[i + 1:]) / MH[i, i]
    return x


def cholesky_inverse(A: np.ndarray) -> np.ndarray:
    return cholesky_solve(A, np.eye(A.shape[0], dtype=np.complex128))


def mmse_exact(H, Y, n0: float, es: float) -> dict:
    """Exact MMSE (eqs. (2)-(3)) and its unbiased SINR via Cholesky, per subcarrier.

    xhat = A^{-1} H^H y;  mu_i = (A^{-1} G)_ii;  rho_i = mu_i^2 / nu_i^2 with
    nu_i^2 = sum_{j != i} |(A^{-1}G)_ij|^2 E_s + (A^{-1} G A^{-1})_ii N0.
    """
    H = np.asarray(H, dtype=np.complex128)
    n, B, U = H.shape
    G = gram(H)
    A = G + (n0 / es) * np.eye(U)
    b = matched_filter(H, Y)
    xhat = np.empty_like(b)
    mu = np.empty((n, U))
    rho = np.empty((n, U))
    Ainv = np.empty_like(A)
    for t in range(n):
        Ai = cholesky_inverse(A[t])
        Ainv[t] = Ai
        xhat[t] = Ai @ b[t]
        Bm = Ai @ G[t]
        C = Bm @ np.conj(Ai.T)
        mu[t] = np.diagonal(Bm).real
        offmask = ~np.eye(U, dtype=bool)
        nu2 = np.sum(np.where(offmask, np.abs(Bm) ** 2, 0.0), axis=1) * es \
            + np.diagonal(C).real * n0
        rho[t] = mu[t] ** 2 / nu2
    return dict(xhat=xhat, mu=mu, rho=rho, Ainv=Ainv, A=A, G=G, b=b)


def precode_mmse_exact(H, T, beta: float) -> np.ndarray:
    """q = P t with P = H_d^H (H_d H_d^H + beta I)^{-1} (eq. (6)), via Cholesky."""
    H = np.asarray(H, dtype=np.complex128)
    A = regularized_gram(H, beta)
    T = np.asarray(T, dtype=np.complex128)
    V = np.stack([cholesky_solve(A[t], T[t]) for t in range(H.shape[0])])
    return H @ V


# --------------------------------------------------------------------------
# Comparison methods built on an explicit (approximate) inverse (Sec. III-F)
# --------------------------------------------------------------------------

def linear_soft_output(Linv: np.ndarray, H, Y, n0: float, es: float, m: int,
                       llr_form: str = "bruteforce") -> dict:
    """Soft output of the linear detector W = Linv H^H (Sec. II-A with the
    exact inverse of eq. (2) replaced by Linv, one (U, U) matrix per
    subcarrier shared by all right-hand sides).

    xhat = Linv H^H y (eq. (3)); mu_i = w_i^H h_i = (Linv G)_ii;
    nu_i^2 = E_s sum_{j != i} |(Linv G)_ij|^2 + N0 (Linv G Linv^H)_ii;
    rho_i = mu_i^2 / nu_i^2; the zero-mu rule and LLRs as in detect_cg.
    """
    H = np.asarray(H, dtype=np.complex128)
    G = gram(H)
    b = matched_filter(H, Y)
    n, U, S = b.shape
    xhat = Linv @ b
    Ls = np.broadcast_to(Linv[:, None], (n, S, U, U))
    mu, _, rho = exact_sinr(Ls, G, es, n0)
    Gii = np.diagonal(G, axis1=-2, axis2=-1).real
    rho_zero = np.broadcast_to((Gii / n0)[:, :, None], (n, U, S))
    zero = mu == 0.0
    rho = np.where(zero, rho_zero, rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(zero, 0.0, xhat / np.where(zero, 1.0, mu))
    llr_fn = llr_maxlog_bruteforce if llr_form == "bruteforce" else llr_maxlog_separable
    return dict(llr=llr_fn(z, rho, m, es), xhat=xhat, mu=mu, rho=rho, z=z, G=G, b=b,
                Linv=Linv)


def detect_cholesky(H, Y, n0: float, es: float, m: int, llr_form: str = "bruteforce") -> dict:
    """Reference soft-output MMSE detector (Sec. III-F-1): A = H^H H +
    (N0/E_s) I is factored as A = M M^H, A^{-1} follows by forward and
    backward substitution, and the soft output is that of W = A^{-1} H^H."""
    H = np.asarray(H, dtype=np.complex128)
    A = regularized_gram(H, n0 / es)
    Ainv = np.stack([cholesky_inverse(A[t]) for t in range(H.shape[0])])
    return linear_soft_output(Ainv, H, Y, n0, es, m, llr_form)


def precode_cholesky(H, T, beta: float, normalize: bool = False) -> dict:
    """Exact MMSE (beta > 0) or ZF (beta = 0) precoding by Cholesky
    (Sec. III-F-1): q = H_d^H (H_d H_d^H + beta I)^{-1} t (eq. (6))."""
    H = np.asarray(H, dtype=np.complex128)
    A = regularized_gram(H, beta)
    T = np.asarray(T, dtype=np.complex128)
    V = np.stack([cholesky_solve(A[t], T[t]) for t in range(H.shape[0])])
    return _precode_output(H, V, normalize)


def _precode_output(H, V, normalize):
    Q = H @ V
    qnorm = np.sqrt(np.sum(np.abs(Q) ** 2, axis=-2))
    if normalize:
        Q = np.where(qnorm[:, None, :] > 0, Q / np.where(qnorm > 0, qnorm, 1.0)[:, None, :], 0.0)
    return dict(Q=Q, qnorm=qnorm, v=V)


def neumann_inverse(A: np.ndarray, K: int) -> np.ndarray:
    """Truncated K-term Neumann series (Sec. III-F-2): with A = D + E,
    D = diag(A), A^{-1} ~ sum_{k=0}^{K-1} (-D^{-1} E)^k D^{-1}, summed term
    by term (term_0 = D^{-1}, term_k = -D^{-1} E term_{k-1})."""
    A = np.asarray(A, dtype=np.complex128)
    U = A.shape[-1]
    d = np.diagonal(A, axis1=-2, axis2=-1).real
    E = A - d[..., :, None] * np.eye(U)
    Dinv = (1.0 / d)[..., :, None] * np.eye(U)
    term = Dinv
    acc = term.copy()
    for _ in range(1, K):
        term = -(1.0 / d)[..., :, None] * (E @ term)
        acc = acc + term
    return acc


def detect_neumann(H, Y, n0: float, es: float, K: int, m: int,
                   llr_form: str = "bruteforce") -> dict:
    """Soft-output detection with the K-term Neumann approximation of
    A^{-1} (Sec. III-F-2) in place of the exact inverse of eq. (2)."""
    H = np.asarray(H, dtype=np.complex128)
    A = regularized_gram(H, n0 / es)
    return linear_soft_output(neumann_inverse(A, K), H, Y, n0, es, m, llr_form)


def precode_neumann(H, T, beta: float, K: int, normalize: bool = False) -> dict:
    """q = H_d^H Ainv~ t with the K-term Neumann approximation of
    (H_d H_d^H + beta I)^{-1} (Sec. III-F-2, eq. (6))."""
    H = np.asarray(H, dtype=np.complex128)
    A = regularized_gram(H, beta)
    V = neumann_inverse(A, K) @ np.asarray(T, dtype=np.complex128)
    return _precode_output(H, V, normalize)


# --------------------------------------------------------------------------
# CGLS on the augmented systems (Sec. III-E, eqs. (17), (18))
# --------------------------------------------------------------------------

@dataclasses.dataclass
class CGLSTrace:
    x: np.ndarray          # (n, N, S) iterate after K steps
    alpha: np.ndarray      # (K, n, S), as CGTrace
    beta: np.ndarray       # (K, n, S)
    iterates: list         # x_1 .. x_K


def cgls(Hb: np.ndarray, yb: np.ndarray, K: int) -> CGLSTrace:
    """K steps of CGLS (the conjugate-gradient least-squares method the paper
    cites for eqs. (17)-(18)) on min ||yb - Hb x||_2 from x_0 = 0, for every
    column of yb independently:

        r_0 = yb, s_0 = Hb^H r_0, p_0 = s_0, gamma_0 = ||s_0||^2
        q = Hb p;  alpha = gamma / ||q||^2;  x += alpha p;  r -= alpha q
        s = Hb^H r;  gamma' = ||s||^2;  beta = gamma' / gamma;  p = s + beta p

    The residual r of the augmented system is kept and s recomputed from it.
    A column with gamma == 0 freezes (alpha = beta = 0), as in cg().
    Hb: (n, R, N), yb: (n, R, S).
    """
    Hb = np.asarray(Hb, dtype=np.complex128)
    yb = np.asarray(yb, dtype=np.complex128)
    n, R, N = Hb.shape
    S = yb.shape[-1]
    HbH = np.conj(np.swapaxes(Hb, -1, -2))
    x = np.zeros((n, N, S), dtype=np.complex128)
    r = yb.copy()
    s = HbH @ r
    p = s.copy()
    gamma = np.sum(np.abs(s) ** 2, axis=-2)
    alphas = np.zeros((K, n, S))
    betas = np.zeros((K, n, S))
    its = []
    for k in range(K):
        q = Hb @ p
        qq = np.sum(np.abs(q) ** 2, axis=-2)
        live = (gamma > 0) & (qq > 0)
        alpha = np.where(live, gamma / np.where(live, qq, 1.0), 0.0)
        x = x + alpha[:, None, :] * p
        r = r - alpha[:, None, :] * q
        s = HbH @ r
        gnew = np.sum(np.abs(s) ** 2, axis=-2)
        beta = np.where(live, gnew / np.where(live, gamma, 1.0), 0.0)
        p = np.where(live[:, None, :], s + beta[:, None, :] * p, p)
        gamma = np.where(live, gnew, gamma)
        alphas[k] = alpha
        betas[k] = beta
        its.append(x.copy())
    return CGLSTrace(x=x, alpha=alphas, beta=betas, iterates=its)


def augment_uplink(H, Y, reg: float):
    """Eq. (17): Hbar_u = [H_u; sqrt(reg) I_U], ybar = [y; 0_U]."""
    H = np.asarray(H, dtype=np.complex128)
    Y = np.asarray(Y, dtype=np.complex128)
    n, B, U = H.shape
    S = Y.shape[-1]
    Hb = np.concatenate([H, np.broadcast_to(math.sqrt(reg) * np.eye(U), (n, U, U))], axis=1)
    yb = np.concatenate([Y, np.zeros((n, U, S))], axis=1)
    return Hb, yb


def augment_downlink(H, beta: float):
    """Eq. (18): Hbar_d = [H_d, sqrt(beta) I_U] with H_d = H_u^H."""
    H = np.asarray(H, dtype=np.complex128)
    n, B, U = H.shape
    Hd = np.conj(np.swapaxes(H, -1, -2))
    return np.concatenate([Hd, np.broadcast_to(math.sqrt(beta) * np.eye(U), (n, U, U))],
                          axis=2)


def detect_cgls(H, Y, n0: float, es: float, K: int, m: int, sinr_mode: str = "approx",
                llr_form: str = "bruteforce") -> dict:
    """Soft-output detection by K CGLS steps on eq. (17), with the SINR
    trackers of Sec. III-C run on the CGLS step sizes (the paper notes the
    trackers carry over): approximate (eqs. (13)-(15), d_i = A_ii) or exact
    (L_K from the matrix form of the recursion with the same alpha, beta)."""
    H = np.asarray(H, dtype=np.complex128)
    reg = n0 / es
    Hb, yb = augment_uplink(H, Y, reg)
    tr = cgls(Hb, yb, K)
    G = gram(H)
    U = G.shape[-1]
    A = G + reg * np.eye(U)
    xhat = tr.x
    n, _, S = xhat.shape
    Gii = np.diagonal(G, axis1=-2, axis2=-1).real
    rho_approx = np.broadcast_to((Gii / n0)[:, :, None], (n, U, S)).copy()
    if sinr_mode == "approx":
        d = np.diagonal(A, axis1=-2, axis2=-1).real
        mu = approx_tracker_shadow(d, tr.alpha, tr.beta) * Gii[:, :, None]
        rho = rho_approx
    elif sinr_mode == "exact":
        L = exact_tracker_shadow(A, tr.alpha, tr.beta)
        mu, _, rho = exact_sinr(L, G, es, n0)
    else:
        raise ValueError(sinr_mode)
    zero = mu == 0.0
    rho = np.where(zero, rho_approx, rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        z = np.where(zero, 0.0, xhat / np.where(zero, 1.0, mu))
    llr_fn = llr_maxlog_bruteforce if llr_form == "bruteforce" else llr_maxlog_separable
    return dict(llr=llr_fn(z, rho, m, es), xhat=xhat, mu=mu, rho=rho, z=z, trace=tr)


def precode_cgls(H, T, beta: float, K: int, normalize: bool = False) -> dict:
    """Precoding by K CGLS steps on eq. (18): qbar minimizes
    ||t - Hbar_d qbar|| over the Krylov space; q = qbar[:B]."""
    H = np.asarray(H, dtype=np.complex128)
    B = H.shape[1]
    tr = cgls(augment_downlink(H, beta), np.asarray(T, dtype=np.complex128), K)
    out = _precode_output_q(tr.x[:, :B, :], normalize)
    out["trace"] = tr
    out["qbar"] = tr.x
    return out


def _precode_output_q(Q, normalize):
    qnorm = np.sqrt(np.sum(np.abs(Q) ** 2, axis=-2))
    if normalize:
        Q = np.where(qnorm[:, None, :] > 0, Q / np.where(qnorm > 0, qnorm, 1.0)[:, None, :], 0.0)
    return dict(Q=Q, qnorm=qnorm)


# --------------------------------------------------------------------------
# Ingest precision: round-to-nearest-even storage formats
# --------------------------------------------------------------------------

def quantize_f16(x: np.ndarray) -> np.ndarray:
    """Complex -> (..., 2) float16 (re, im), IEEE round-to-nearest-even."""
    x = np.asarray(x)
    return np.stack([x.real, x.imag], -1).astype(np.float32).astype(np.float16)


def quantize_bf16(x: np.ndarray) -> np.ndarray:
    """Complex -> (..., 2) uint16 bfloat16 bit patterns (re, im), RNE.

    bf16 keeps the top 16 bits of the float32 pattern; rounding adds
    0x7FFF plus the lowest kept bit before truncation (ties to even).
    NaN inputs are not expected (finite workloads only).
    """
    x = np.asarray(x)
    f = np.stack([x.real, x.imag], -1).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def dequantize_f16(q: np.ndarray) -> np.ndarray:
    q = q.astype(np.float64)
    return q[..., 0] + 1j * q[..., 1]


def dequantize_bf16(q: np.ndarray) -> np.ndarray:
    f = (q.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return f[..., 0] + 1j * f[..., 1]
