"""Pins for the oracle's comparison methods: Cholesky-based exact inversion
and the truncated Neumann series (Sec. III-F), and CGLS on the augmented
systems (Sec. III-E, eqs. (17), (18)).  Each is checked against something
other than its own formulas: LAPACK solvers and inverses, the closed form
of a finite geometric series, the least-squares characterization of the
CGLS iterates over their Krylov space, identities with the CG iterates, and
the unbiased-MMSE SINR closed form."""
import numpy as np
import pytest

from oracle import mimo_oracle as O
from paper_1404_0424_amd import workload as W


def _frame(n=4, B=32, U=8, S=4, m=4, snr=10.0, seed=3, **kw):
    return W.uplink_frame(np.random.default_rng(seed), n, B, U, S, m, snr, **kw)


def _herm(X):
    return np.conj(np.swapaxes(X, -1, -2))


# ---------------------------------------------------------------- Cholesky

@pytest.mark.parametrize("es", [1.0, 2.5])
def test_cholesky_detector_against_lapack_and_unbiased_sinr(es):
    f = _frame(n=3, B=24, U=6, S=3, m=4, snr=8.0, seed=11, es=es)
    out = O.detect_cholesky(f.H, f.Y, f.n0, es, 4)
    reg = f.n0 / es
    G = np.einsum("nbi,nbj->nij", np.conj(f.H), f.H)
    A = G + reg * np.eye(6)
    Ainv = np.linalg.inv(A)
    b = np.einsum("nbi,nbs->nis", np.conj(f.H), f.Y)
    np.testing.assert_allclose(out["xhat"], np.linalg.solve(A, b), rtol=1e-12, atol=1e-13)
    # unbiased MMSE: mu_i = (A^-1 G)_ii = 1 - reg (A^-1)_ii, rho_i = mu_i / (E_s (1 - mu_i))
    aii = np.diagonal(Ainv, axis1=1, axis2=2).real
    mu = 1.0 - reg * aii
    rho = mu / (es * (1.0 - mu))
    np.testing.assert_allclose(out["mu"], np.broadcast_to(mu[:, :, None], out["mu"].shape),
                               rtol=1e-12)
    np.testing.assert_allclose(out["rho"], np.broadcast_to(rho[:, :, None], out["rho"].shape),
                               rtol=1e-10)


def test_cholesky_detector_equals_cg_exact_tracker_at_K_equals_U():
    f = _frame(n=3, B=32, U=8, S=3, m=6, snr=12.0, seed=5)
    ch = O.detect_cholesky(f.H, f.Y, f.n0, f.es, 6)
    cg = O.detect_cg(f.H, f.Y, f.n0, f.es, 8, 6, sinr_mode="exact")
    np.testing.assert_allclose(ch["xhat"], cg["xhat"], rtol=1e-9, atol=1e-11)
    np.testing.assert_allclose(ch["mu"], cg["mu"], rtol=1e-9)
    np.testing.assert_allclose(ch["rho"], cg["rho"], rtol=1e-8)
    scale = np.maximum(1.0, np.abs(ch["llr"]).max(-1, keepdims=True))
    assert np.max(np.abs(ch["llr"] - cg["llr"]) / scale) < 1e-8


@pytest.mark.parametrize("m", [2, 4])
def test_cholesky_single_user_llr_equals_ml(m):
    f = _frame(n=5, B=8, U=1, S=2, m=m, snr=6.0, seed=2)
    out = O.detect_cholesky(f.H, f.Y, f.n0, f.es, m)
    for t in range(5):
        for s in range(2):
            ml = O.ml_maxlog_bruteforce(f.H[t], f.Y[t, :, s], f.n0, m, f.es)
            np.testing.assert_allclose(out["llr"][t, :, s], ml, rtol=1e-9, atol=1e-9)


def test_cholesky_precoder_zf_and_mmse():
    rng = np.random.default_rng(9)
    f = _frame(n=3, B=20, U=5, S=3, seed=9)
    T = W.qam_map(W.random_bits(rng, (3, 5, 3), 4), 4)
    zf = O.precode_cholesky(f.H, T, 0.0)
    np.testing.assert_allclose(_herm(f.H) @ zf["Q"], T, atol=1e-12)          # H_d q = t
    beta = 0.3
    mm = O.precode_cholesky(f.H, T, beta, normalize=True)
    G = _herm(f.H) @ f.H
    q = f.H @ np.linalg.solve(G + beta * np.eye(5), T)                        # eq. (6)
    nq = np.linalg.norm(q, axis=1)
    np.testing.assert_allclose(mm["qnorm"], nq, rtol=1e-12)
    np.testing.assert_allclose(mm["Q"], q / nq[:, None, :], rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------- Neumann

def test_neumann_series_closed_form():
    # sum_{k<K} N^k D^-1 with N = -D^-1 E equals (I - N^K) A^-1 (finite
    # geometric series; I - N = D^-1 A)
    f = _frame(n=2, B=32, U=6, seed=4)
    A = O.regularized_gram(f.H, 0.2)
    for K in (1, 2, 3, 5):
        X = O.neumann_inverse(A, K)
        for t in range(2):
            d = np.diag(A[t]).real
            N = -(A[t] - np.diag(d)) / d[:, None]
            ref = (np.eye(6) - np.linalg.matrix_power(N, K)) @ np.linalg.inv(A[t])
            np.testing.assert_allclose(X[t], ref, rtol=1e-11, atol=1e-13)
            np.testing.assert_allclose(X[t], _herm(X[t]), rtol=1e-12, atol=1e-14)


def test_neumann_K1_and_convergence():
    f = _frame(n=2, B=128, U=8, seed=6)           # B >> U: D^-1 E has small spectral radius
    A = O.regularized_gram(f.H, 0.1)
    X1 = O.neumann_inverse(A, 1)
    np.testing.assert_allclose(X1, np.stack([np.diag(1 / np.diag(a).real) for a in A]))
    X60 = O.neumann_inverse(A, 60)
    np.testing.assert_allclose(X60, np.linalg.inv(A), rtol=1e-10, atol=1e-12)


def test_neumann_detector_is_exact_mmse_for_orthogonal_users():
    # E = 0 when the channel columns are orthogonal: every K gives A^-1
    rng = np.random.default_rng(8)
    n, B, U, S = 3, 16, 4, 2
    Z = rng.standard_normal((n, B, U)) + 1j * rng.standard_normal((n, B, U))
    Qm, _ = np.linalg.qr(Z)
    H = Qm * rng.uniform(0.5, 2.0, (n, 1, U))
    X = W.qam_map(W.random_bits(rng, (n, U, S), 4), 4)
    Y = H @ X + W.awgn(rng, (n, B, S), 0.1)
    ref = O.detect_cholesky(H, Y, 0.1, 1.0, 4)
    for K in (1, 2):
        out = O.detect_neumann(H, Y, 0.1, 1.0, K, 4)
        np.testing.assert_allclose(out["xhat"], ref["xhat"], rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(out["rho"], ref["rho"], rtol=1e-10)


def test_neumann_detector_sinr_matches_definitions():
    # mu = (X G)_ii and nu^2 written out entry by entry for one system
    f = _frame(n=1, B=32, U=4, S=1, seed=12)
    out = O.detect_neumann(f.H, f.Y, f.n0, f.es, 2, 4)
    H = f.H[0]
    A = H.conj().T @ H + f.n0 / f.es * np.eye(4)
    X = O.neumann_inverse(A[None], 2)[0]
    Wm = X @ H.conj().T                                   # rows w_i^H
    for i in range(4):
        mu = (Wm[i] @ H[:, i]).real
        nu2 = sum(abs(Wm[i] @ H[:, j]) ** 2 for j in range(4) if j != i) * f.es \
            + np.sum(np.abs(Wm[i]) ** 2) * f.n0
        assert abs(out["mu"][0, i, 0] - mu) < 1e-12 * abs(mu)
        assert abs(out["rho"][0, i, 0] - mu * mu / nu2) < 1e-10 * mu * mu / nu2


def test_neumann_precoder_K1():
    rng = np.random.default_rng(10)
    f = _frame(n=2, B=16, U=4, S=2, seed=10)
    T = W.qam_map(W.random_bits(rng, (2, 4, 2), 2), 2)
    out = O.precode_neumann(f.H, T, 0.5, 1)
    d = np.linalg.norm(f.H, axis=1) ** 2 + 0.5
    np.testing.assert_allclose(out["Q"], f.H @ (T / d[:, :, None]), rtol=1e-13)


# ---------------------------------------------------------------- CGLS

def _krylov_lsq(Hb, yb, k):
    """argmin ||yb - Hb x|| over span{s, M s, ..., M^{k-1} s}, M = Hb^H Hb,
    s = Hb^H yb: the defining property of the k-th CGLS iterate."""
    M = _herm(Hb) @ Hb
    s = _herm(Hb) @ yb
    Kr = np.stack([np.linalg.matrix_power(M, j) @ s for j in range(k)], -1)
    Qk, _ = np.linalg.qr(Kr)
    c, *_ = np.linalg.lstsq(Hb @ Qk, yb, rcond=None)
    return Qk @ c


def test_cgls_uplink_matches_krylov_least_squares_and_cg():
    f = _frame(n=2, B=24, U=6, S=2, snr=5.0, seed=13)
    reg = f.n0 / f.es
    Hb, yb = O.augment_uplink(f.H, f.Y, reg)
    A = O.regularized_gram(f.H, reg)
    b = O.matched_filter(f.H, f.Y)
    for K in range(1, 7):
        tr = O.cgls(Hb, yb, K)
        cg = O.cg(A, b, K)
        np.testing.assert_allclose(tr.x, cg.v, rtol=1e-9, atol=1e-11)   # same iterates
        np.testing.assert_allclose(tr.alpha, cg.alpha, rtol=1e-9)
        np.testing.assert_allclose(tr.beta, cg.beta, rtol=1e-8, atol=1e-14)
        for t in range(2):
            for s in range(2):
                x = _krylov_lsq(Hb[t], yb[t, :, s], K)
                err = np.linalg.norm(tr.x[t, :, s] - x) / np.linalg.norm(x)
                assert err < 1e-9, (K, err)


def test_cgls_downlink_krylov_least_squares_and_exact_at_K_equals_U():
    rng = np.random.default_rng(14)
    f = _frame(n=2, B=16, U=5, S=2, seed=14)
    T = W.qam_map(W.random_bits(rng, (2, 5, 2), 4), 4)
    beta = 0.25
    Hb = O.augment_downlink(f.H, beta)
    assert Hb.shape == (2, 5, 21)
    np.testing.assert_allclose(Hb[:, :, :16], _herm(f.H))
    for K in range(1, 6):
        tr = O.cgls(Hb, T, K)
        for t in range(2):
            for s in range(2):
                x = _krylov_lsq(Hb[t], T[t, :, s], K)
                err = np.linalg.norm(tr.x[t, :, s] - x) / np.linalg.norm(x)
                assert err < 1e-9, (K, err)
    out = O.precode_cgls(f.H, T, beta, 5)
    ref = f.H @ np.linalg.solve(_herm(f.H) @ f.H + beta * np.eye(5), T)
    np.testing.assert_allclose(out["Q"], ref, rtol=1e-9, atol=1e-11)


def test_cgls_downlink_K1_closed_form_and_differs_from_cg_below_U():
    rng = np.random.default_rng(15)
    f = _frame(n=2, B=16, U=6, S=2, seed=15)
    T = W.qam_map(W.random_bits(rng, (2, 6, 2), 4), 4)
    beta = 0.4
    out = O.precode_cgls(f.H, T, beta, 1)
    # qbar_1 = alpha_1 s_0, s_0 = Hbar_d^H t = [H t; sqrt(beta) t],
    # alpha_1 = ||s_0||^2 / ||Hbar_d s_0||^2 with Hbar_d s_0 = (G + beta I) t
    G = _herm(f.H) @ f.H
    s0 = np.concatenate([f.H @ T, np.sqrt(beta) * T], axis=1)
    Gt = (G + beta * np.eye(6)) @ T
    a1 = np.sum(np.abs(s0) ** 2, axis=1) / np.sum(np.abs(Gt) ** 2, axis=1)
    np.testing.assert_allclose(out["Q"], a1[:, None, :] * (f.H @ T), rtol=1e-12)
    # CG-P minimizes the A-norm error of v instead: the iterates differ for K < U
    cgp = O.precode_cg(f.H, T, beta, 2)
    cgl = O.precode_cgls(f.H, T, beta, 2)
    assert np.min(np.linalg.norm(cgp["Q"] - cgl["Q"], axis=1)
                  / np.linalg.norm(cgp["Q"], axis=1)) > 1e-4


def test_cgls_detector_trackers_use_cgls_steps():
    # with the CGLS alpha/beta equal to CG's, both trackers reproduce CG-D
    f = _frame(n=2, B=32, U=8, S=3, m=4, snr=10.0, seed=16)
    for mode in ("approx", "exact"):
        a = O.detect_cgls(f.H, f.Y, f.n0, f.es, 3, 4, sinr_mode=mode)
        b = O.detect_cg(f.H, f.Y, f.n0, f.es, 3, 4, sinr_mode=mode)
        np.testing.assert_allclose(a["mu"], b["mu"], rtol=1e-9)
        np.testing.assert_allclose(a["rho"], b["rho"], rtol=1e-8)
        scale = np.maximum(1.0, np.abs(b["llr"]).max(-1, keepdims=True))
        assert np.max(np.abs(a["llr"] - b["llr"]) / scale) < 1e-8


def test_cgls_zero_rhs_freezes():
    f = _frame(n=1, B=16, U=4, S=2, seed=17)
    Y = f.Y.copy()
    Y[..., 1] = 0
    out = O.detect_cgls(f.H, Y, f.n0, f.es, 3, 4)
    assert np.all(out["xhat"][..., 1] == 0)
    assert np.all(out["trace"].alpha[:, :, 1] == 0)
    assert np.all(np.isfinite(out["llr"]))
