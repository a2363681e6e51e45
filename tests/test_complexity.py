"""The real-multiplication counter of Sec. IV-A.

Pins: (1) the crossovers the paper states (tests/golden/complexity_crossovers.json);
(2) its qualitative ordering at small K; (3) an independent count: small
instrumented implementations of each detector that tally every real
multiplication as they execute (skipping the same structural zeros) and
whose results are checked against numpy, so a slip in the counter's loop
bounds or per-operation costs shows up as a mismatch."""
import json
import os

import numpy as np
import pytest

from paper_1404_0424_amd import complexity as C

HERE = os.path.dirname(os.path.abspath(__file__))


def test_crossovers_match_the_paper():
    gold = json.load(open(os.path.join(HERE, "golden", "complexity_crossovers.json")))
    for row in gold["crossovers"]:
        assert C.crossover(row["B"], row["U"]) == row["k_max"], row


@pytest.mark.parametrize("B,U", [(32, 8), (128, 8), (32, 16), (128, 16)])
def test_cgls_and_neumann_cheaper_than_cg_at_small_K(B, U):
    assert C.cgls_detect(B, U, 1) < C.cg_detect(B, U, 1)
    assert C.neumann_detect(B, U, 1) < C.cg_detect(B, U, 1)
    # CGLS saves the Gram but pays two B x U products per iteration
    assert C.cgls_detect(B, U, 8) > C.cg_detect(B, U, 8)
    # the counts grow with K; the Cholesky detector does not depend on it
    assert all(C.cg_detect(B, U, k) < C.cg_detect(B, U, k + 1) for k in range(1, 20))


# ---------------------------------------------------------------- instrumented count

class Tally:
    def __init__(self):
        self.n = 0

    def rmul(self, a, b):
        self.n += 1
        return a * b

    def div(self, a, b):
        self.n += 1
        return a / b

    def cmul(self, a, b):
        self.n += 4
        return a * b

    def rcmul(self, r, z):
        self.n += 2
        return r * z

    def abs2(self, z):
        self.n += 2
        return z.real * z.real + z.imag * z.imag

    def redot(self, a, b):                # Re(a conj(b))
        self.n += 2
        return a.real * b.real + a.imag * b.imag


def _system(B, U, seed):
    rng = np.random.default_rng(seed)
    H = (rng.standard_normal((B, U)) + 1j * rng.standard_normal((B, U))) / np.sqrt(2 * B)
    y = rng.standard_normal(B) + 1j * rng.standard_normal(B)
    return H, y, 0.3


def _gram_mf(t, H, y, reg):
    B, U = H.shape
    A = np.zeros((U, U), complex)
    for i in range(U):
        for j in range(i, U):
            if i == j:
                A[i, i] = sum(t.abs2(H[b, i]) for b in range(B))
            else:
                A[i, j] = sum(t.cmul(np.conj(H[b, i]), H[b, j]) for b in range(B))
                A[j, i] = np.conj(A[i, j])
    G = A.copy()
    A = A + reg * np.eye(U)
    bv = np.array([sum(t.cmul(np.conj(H[b, i]), y[b]) for b in range(B)) for i in range(U)])
    return G, A, bv


def _herm_matvec(t, A, p):
    U = len(p)
    return np.array([t.rcmul(A[i, i].real, p[i]) + sum(t.cmul(A[i, j], p[j])
                                                     for j in range(U) if j != i)
                     for i in range(U)])


def _cg(t, H, y, reg, K):
    B, U = H.shape
    G, A, bv = _gram_mf(t, H, y, reg)
    v = np.zeros(U, complex)
    r = bv.copy()
    p = r.copy()
    rr = sum(t.abs2(x) for x in r)
    tv, trr, tp = np.zeros(U), np.ones(U), np.ones(U)
    for _ in range(K):
        e = _herm_matvec(t, A, p)
        alpha = t.div(rr, sum(t.redot(p[i], e[i]) for i in range(U)))
        v = v + np.array([t.rcmul(alpha, x) for x in p])
        r = r - np.array([t.rcmul(alpha, x) for x in e])
        rn = sum(t.abs2(x) for x in r)
        beta = t.div(rn, rr)
        rr = rn
        p = r + np.array([t.rcmul(beta, x) for x in p])
        t.n += U                                             # diagonal tracker (eq. (13))
        tv = tv + alpha * tp
        trr = trr - alpha * A.diagonal().real * tp
        tp = trr + beta * tp
        mu = np.array([t.rmul(tv[i], G[i, i].real) for i in range(U)])
        rho = np.array([t.rmul(G[i, i].real, 1.0 / 0.7) for i in range(U)])
    return v, A, bv


def _cholesky(t, H, y, reg):
    B, U = H.shape
    G, A, bv = _gram_mf(t, H, y, reg)
    M = np.zeros((U, U), complex)
    for j in range(U):
        d = A[j, j].real - sum(t.abs2(M[j, k]) for k in range(j))
        inv = t.div(1.0, np.sqrt(d))
        M[j, j] = np.sqrt(d)
        for i in range(j + 1, U):
            s = A[i, j] - sum(t.cmul(M[i, k], np.conj(M[j, k])) for k in range(j))
            M[i, j] = t.rcmul(inv, s)
    Z = np.zeros((U, U), complex)
    for j in range(U):                                       # M Z = I
        for i in range(j, U):
            s = (1.0 if i == j else 0.0) - sum(t.cmul(M[i, k], Z[k, j]) for k in range(j, i))
            Z[i, j] = t.rcmul(1.0 / M[i, i].real, s)
    X = np.zeros((U, U), complex)
    for j in range(U):                                       # M^H X = Z
        for i in range(U - 1, -1, -1):
            s = Z[i, j] - sum(t.cmul(np.conj(M[k, i]), X[k, j]) for k in range(i + 1, U))
            X[i, j] = t.rcmul(1.0 / M[i, i].real, s)
    xhat = _herm_matvec(t, X, bv)
    mu = np.array([1.0 - t.rmul(reg, X[i, i].real) for i in range(U)])
    rho = np.array([t.div(mu[i], t.rmul(1.0, 1.0 - mu[i])) for i in range(U)])
    return X, A, xhat


def _cgls(t, H, y, reg, K):
    B, U = H.shape
    sr = np.sqrt(reg)
    s = np.array([sum(t.cmul(np.conj(H[b, i]), y[b]) for b in range(B)) for i in range(U)])
    g = [sum(t.abs2(H[b, i]) for b in range(B)) for i in range(U)]
    r_top, r_bot = y.astype(complex).copy(), np.zeros(U, complex)
    x = np.zeros(U, complex)
    p = s.copy()
    gam = sum(t.abs2(v) for v in s)
    for _ in range(K):
        q_top = np.array([sum(t.cmul(H[b, i], p[i]) for i in range(U)) for b in range(B)])
        q_bot = np.array([t.rcmul(sr, v) for v in p])
        alpha = t.div(gam, sum(t.abs2(v) for v in q_top) + sum(t.abs2(v) for v in q_bot))
        x = x + np.array([t.rcmul(alpha, v) for v in p])
        r_top = r_top - np.array([t.rcmul(alpha, v) for v in q_top])
        r_bot = r_bot - np.array([t.rcmul(alpha, v) for v in q_bot])
        s = np.array([sum(t.cmul(np.conj(H[b, i]), r_top[b]) for b in range(B))
                      + t.rcmul(sr, r_bot[i]) for i in range(U)])
        gn = sum(t.abs2(v) for v in s)
        beta = t.div(gn, gam)
        gam = gn
        p = s + np.array([t.rcmul(beta, v) for v in p])
        t.n += U                                             # tracker
        for i in range(U):
            t.rmul(1.0, g[i])                                # mu_{i|k}
            t.rmul(g[i], 1.0)                                # rho_{i|k}
    return x


def _neumann(t, H, y, reg, K):
    B, U = H.shape
    G, A, bv = _gram_mf(t, H, y, reg)
    dinv = np.array([t.div(1.0, A[i, i].real) for i in range(U)])
    X = np.diag(dinv).astype(complex)
    term = np.diag(dinv).astype(complex)
    if K >= 2:
        term = np.zeros((U, U), complex)
        for i in range(U):
            for j in range(i + 1, U):
                term[i, j] = -t.rcmul(t.rmul(dinv[i], dinv[j]), A[i, j])
                term[j, i] = np.conj(term[i, j])
        X = X + term
    for _ in range(3, K + 1):
        new = np.zeros((U, U), complex)
        for i in range(U):
            for j in range(i, U):
                s = sum(t.cmul(A[i, l], term[l, j]) for l in range(U)
                        if l != i and term[l, j] != 0)
                new[i, j] = -t.rcmul(dinv[i], s)
                new[j, i] = np.conj(new[i, j])
        term = new
        X = X + term
    xhat = (np.array([t.rcmul(dinv[i], bv[i]) for i in range(U)]) if K == 1
            else _herm_matvec(t, X, bv))
    if K == 1:
        mu = [t.rmul(dinv[i], G[i, i].real) for i in range(U)]
    else:
        mu = [t.rmul(X[i, i].real, G[i, i].real)
              + sum(t.redot(X[i, l], np.conj(G[l, i])) for l in range(U) if l != i)
              for i in range(U)]
    for i in range(U):
        t.div(mu[i], t.rmul(1.0, 1.0 - mu[i]))
    return X, A, xhat


@pytest.mark.parametrize("B,U", [(6, 3), (9, 4), (12, 5)])
@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_counter_matches_instrumented_execution(B, U, K):
    H, y, reg = _system(B, U, 100 * B + 10 * U + K)
    t = Tally()
    v, A, bv = _cg(t, H, y, reg, K)
    assert t.n == C.cg_detect(B, U, K)
    if K == U:
        np.testing.assert_allclose(v, np.linalg.solve(A, bv), rtol=1e-9)
    t = Tally()
    X, A, xh = _cholesky(t, H, y, reg)
    np.testing.assert_allclose(X, np.linalg.inv(A), rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(xh, np.linalg.solve(A, bv), rtol=1e-10)
    assert t.n == C.cholesky_detect(B, U)
    t = Tally()
    x = _cgls(t, H, y, reg, K)
    assert t.n == C.cgls_detect(B, U, K)
    t2 = Tally()
    v2, _, _ = _cg(t2, H, y, reg, K)
    np.testing.assert_allclose(x, v2, rtol=1e-9, atol=1e-12)      # CGLS iterates = CG's
    t = Tally()
    X, A, xh = _neumann(t, H, y, reg, K)
    d = np.diag(A).real
    N = -(A - np.diag(d)) / d[:, None]
    np.testing.assert_allclose(X, (np.eye(U) - np.linalg.matrix_power(N, K)) @ np.linalg.inv(A),
                               rtol=1e-10, atol=1e-12)
    assert t.n == C.neumann_detect(B, U, K)
