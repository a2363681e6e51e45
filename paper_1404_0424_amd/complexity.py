"""Real-multiplication counts of the uplink detectors compared in Sec. IV-A.

The paper compares the exact Cholesky-based soft-output MMSE detector, the
truncated Neumann series, CG-D (Algorithm 1 with the approximate SINR of
eqs. (13)-(15)) and CGLS (eq. (17)) by the number of real-valued
multiplications, counting four per complex multiplication, exploiting
Hermitian symmetry and skipping multiplications with zeros.  The remaining
rules are not spelled out; this module fixes them as follows and counts
every method by walking its loops:

* complex x complex = 4, real x complex = 2, |z|^2 = 2, Re(a conj(b)) = 2,
  real x real = 1; a real division or reciprocal counts as 1; square roots
  and additions are free.
* Hermitian results are formed from their upper triangle; real diagonals
  (of G, A, the Cholesky factor) make their products real x complex.
* Structural zeros (of triangular factors, of the identity right-hand
  sides, of the zero lower block of the augmented receive vector) are
  skipped.
* Algorithm 1 is counted as printed: mu_{i|k} (eq. (14)) and rho_{i|k}
  (eq. (15)) are evaluated in every iteration, and the diagonal tracker of
  eq. (13) costs U multiplications per iteration, the figure the paper
  gives for it.
* The Cholesky-based inverse follows the paper's description: A = M M^H,
  then forward substitution M Z = I and backward substitution
  M^H A^{-1} = Z over all U columns.
* The LLR evaluation of eq. (4) is the same for every method and is left
  out.

With these rules CG-D needs fewer multiplications than the Cholesky-based
detector up to K = 5 for U = 8 and up to K = 12 for U = 16, at B = 32 and
B = 128, the crossovers stated in Sec. IV-A.
"""
from __future__ import annotations

CMUL, RCMUL, ABS2, REDOT, RMUL, DIV = 4, 2, 2, 2, 1, 1


def gram(B: int, U: int) -> int:
    """A = H^H H + reg I: upper triangle, real diagonal."""
    off = U * (U - 1) // 2 * B * CMUL
    diag = U * B * ABS2
    return off + diag


def matched_filter(B: int, U: int) -> int:
    """b = H^H y."""
    return U * B * CMUL


def hermitian_matvec(U: int) -> int:
    """e = A p with A Hermitian with a real diagonal."""
    return U * (U - 1) * CMUL + U * RCMUL


def cg_detect(B: int, U: int, K: int) -> int:
    """CG-D: Gram, matched filter, K iterations of Algorithm 1 with the
    approximate SINR (eqs. (13)-(15)) evaluated in every iteration."""
    n = gram(B, U) + matched_filter(B, U)
    n += U * ABS2                               # ||r_0||^2
    per_it = (hermitian_matvec(U)               # e = A p
              + U * REDOT + DIV                 # alpha = ||r||^2 / Re(p^H e)
              + U * RCMUL                       # v += alpha p
              + U * RCMUL                       # r -= alpha e
              + U * ABS2 + DIV                  # beta = ||r_k||^2 / ||r_{k-1}||^2
              + U * RCMUL                       # p = r + beta p
              + U                               # diagonal tracker, eq. (13)
              + U * RMUL                        # mu_{i|k} = L~_ii G_ii, eq. (14)
              + U * RMUL)                       # rho_{i|k} = G_ii / N0, eq. (15)
    return n + K * per_it


def cholesky_detect(B: int, U: int) -> int:
    """Exact soft-output MMSE via Cholesky (Sec. III-F-1)."""
    n = gram(B, U) + matched_filter(B, U)
    for j in range(U):                          # A = M M^H, column j
        n += j * ABS2 + DIV                     # M_jj^2 = A_jj - sum |M_jk|^2, 1/M_jj
        n += (U - 1 - j) * (j * CMUL + RCMUL)   # M_ij = (A_ij - sum M_ik conj(M_jk)) / M_jj
    for j in range(U):                          # M Z = I: Z lower triangular
        for i in range(j, U):
            n += (i - j) * CMUL + RCMUL         # (e_j - sum_{j<=k<i} M_ik Z_kj) / M_ii
    for j in range(U):                          # M^H X = Z, every column of X
        for i in range(U):
            n += (U - 1 - i) * CMUL + RCMUL     # (Z_ij - sum_{k>i} conj(M_ki) X_kj) / M_ii
    n += hermitian_matvec(U)                    # xhat = A^{-1} b
    n += U * RMUL                               # mu_i = 1 - reg (A^{-1})_ii
    n += U * (RMUL + DIV)                       # rho_i = mu_i / (E_s (1 - mu_i))
    return n


def neumann_detect(B: int, U: int, K: int, sinr: str = "mmse_identity") -> int:
    """K-term Neumann series (Sec. III-F-2): Ainv~ = sum_{k<K} (-D^{-1}E)^k D^{-1}
    formed term by term (every term Hermitian, upper triangle; term_1 is
    diagonal and term_2 has a zero diagonal), xhat = Ainv~ b, then the SINR:

    * ``"mmse_identity"``: mu_i = (Ainv~ G)_ii and rho_i = mu_i / (E_s (1 - mu_i)),
      the unbiased-MMSE relation applied to the approximate inverse (the
      low-cost form the comparison relies on);
    * ``"definition"``: the Sec. II-A quantities of W = Ainv~ H^H through the
      full B = Ainv~ G (mu_i = B_ii, nu_i^2 = E_s sum_{j != i} |B_ij|^2 +
      N0 (B Ainv~^H)_ii), which is what the GPU Neumann detector evaluates.
    """
    n = gram(B, U) + matched_filter(B, U)
    n += U * DIV                                            # term_1 = D^{-1}
    if K >= 2:                                              # term_2 = -D^{-1} E D^{-1}
        n += U * (U - 1) // 2 * (RMUL + RCMUL)
    for k in range(3, K + 1):                               # term_k = -D^{-1} E term_{k-1}
        for i in range(U):
            for j in range(i, U):
                terms = U - 1 if (k > 3 or i == j) else U - 2   # term_2 has a zero diagonal
                n += terms * CMUL + RCMUL
    diag = K == 1
    n += U * RCMUL if diag else hermitian_matvec(U)         # xhat = Ainv~ b
    if sinr == "mmse_identity":
        n += U * RMUL if diag else U * (RMUL + (U - 1) * REDOT)   # mu_i = (Ainv~ G)_ii
        n += U * (RMUL + DIV)                               # rho_i
    elif sinr == "definition":
        if diag:
            n += U * (U - 1) * RCMUL + U * RMUL             # B = D^{-1} G
            n += U * (U - 1) * ABS2 + U * RMUL              # sum |B_ij|^2, C_ii = B_ii X_ii
        else:
            n += U * U * ((U - 1) * CMUL + RCMUL)           # B = Ainv~ G (G: real diagonal)
            n += U * (U - 1) * ABS2 + U * U * REDOT         # sum |B_ij|^2, C_ii
        n += U * (2 * RMUL) + U * (RMUL + DIV)              # nu^2, rho = mu^2 / nu^2
    else:
        raise ValueError(sinr)
    return n


def cgls_detect(B: int, U: int, K: int) -> int:
    """CGLS on eq. (17): no Gram; per iteration q = Hbar p and s = Hbar^H r,
    with the approximate SINR tracker on the CGLS steps (d_i = ||h_i||^2 +
    reg needs the column norms)."""
    R = B + U
    n = matched_filter(B, U)                    # s_0 = Hbar^H ybar = H^H y
    n += U * B * ABS2                           # ||h_i||^2 for d_i and rho_i
    n += U * ABS2                               # gamma_0
    per_it = (B * U * CMUL + U * RCMUL          # q = [H p; sqrt(reg) p]
              + R * ABS2 + DIV                  # alpha = gamma / ||q||^2
              + U * RCMUL                       # x += alpha p
              + R * RCMUL                       # r -= alpha q
              + U * B * CMUL + U * RCMUL        # s = H^H r_top + sqrt(reg) r_bot
              + U * ABS2 + DIV                  # beta
              + U * RCMUL                       # p = s + beta p
              + U + U * RMUL + U * RMUL)        # tracker, mu_{i|k}, rho_{i|k}
    return n + K * per_it


def crossover(B: int, U: int, k_max: int = 200) -> int:
    """Largest K with CG-D no more expensive than the Cholesky detector."""
    ref = cholesky_detect(B, U)
    best = 0
    for K in range(1, k_max + 1):
        if cg_detect(B, U, K) <= ref:
            best = K
    return best


def table(B: int, U: int, K_values=range(1, 17)) -> list[dict]:
    """Counts of every method for each K (the Cholesky count does not depend on K)."""
    ch = cholesky_detect(B, U)
    return [{"K": K, "cg": cg_detect(B, U, K), "cgls": cgls_detect(B, U, K),
             "neumann": neumann_detect(B, U, K),
             "neumann_definition_sinr": neumann_detect(B, U, K, "definition"),
             "cholesky": ch} for K in K_values]


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="real-multiplication counts (Sec. IV-A)")
    ap.add_argument("--B", type=int, nargs="+", default=[32, 128])
    ap.add_argument("--U", type=int, nargs="+", default=[8, 16])
    ap.add_argument("--K", type=int, default=16)
    args = ap.parse_args(argv)
    for B in args.B:
        for U in args.U:
            print(f"B={B} U={U}: CG-D cheaper than Cholesky for K <= {crossover(B, U)}")
            print("   K       CG     CGLS  Neumann  Cholesky")
            for r in table(B, U, range(1, args.K + 1)):
                print(f"  {r['K']:2d} {r['cg']:8d} {r['cgls']:8d} {r['neumann']:8d} {r['cholesky']:9d}")


if __name__ == "__main__":
    main()
