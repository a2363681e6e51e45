/*
 * mimo_cg.h -- C ABI of the MI355X (gfx950) library for conjugate-gradient
 * soft-output MMSE detection and CG precoding in massive MIMO.
 *
 * Method: B. Yin, M. Wu, J. R. Cavallaro, C. Studer, "Conjugate
 * Gradient-based Soft-Output Detection and Precoding in Massive MIMO
 * Systems" (Sec. II system models, Sec. III and Algorithm 1).
 *
 * General rules for every entry point
 *  - Data pointers are DEVICE pointers (HBM) owned by the caller; the library
 *    never frees or retains them past the call.  Outputs must not alias
 *    inputs.  Pointers must be 16-byte aligned.
 *  - Calls validate their arguments synchronously and return a negative
 *    mimo_status before anything is enqueued.  Valid calls enqueue kernels
 *    on `stream` (a hipStream_t passed as void*; NULL = the default stream)
 *    and return MIMO_OK without waiting.  A device fault surfaces as a HIP
 *    error at the caller's next synchronization; a launch failure returns
 *    MIMO_EHIP and mimo_last_error() names it.
 *  - The library allocates no device memory.
 *  - Complex numbers are interleaved {re, im}.  complex64 = 2 x float.
 *  - All arrays are dense and row-major, indexed by subcarrier first:
 *      H    [n_sc][B][U]   uplink channel H_u (B x U per subcarrier);
 *                          the downlink channel is H_d = H_u^H (Sec. II-B)
 *      Y    [n_sc][B][S]   S receive vectors y (columns) sharing one H
 *      T    [n_sc][U][S]   S downlink symbol vectors t (complex64)
 *      A    [n_sc][U][U]   regularized Gram matrix (complex64)
 *      b    [n_sc][U][S]   matched-filter outputs (complex64)
 *      xhat [n_sc][U][S]   equalized symbols v_K (complex64)
 *      mu, sinr [n_sc][U][S]  equalized gain and post-equalization SINR
 *      llr  [n_sc][U][S][qam_bits]
 *      Q    [n_sc][B][S]   precoded vectors q (or s = q/||q||), complex64
 *      qnorm [n_sc][S]     ||q||_2 of each precoded vector
 *  - Reduced-precision channel/receive storage (MIMO_C16, MIMO_CBF16) uses
 *    the blocked layout written by mimo_convert: for a [n][R][C] complex
 *    array (R = B, a multiple of 8), element (n, r, c) sits in block
 *    [n][r/8][part][c][r%8] with part 0 = real, part 1 = imaginary, i.e.
 *    8 consecutive antennas of one column are contiguous per part.
 */
#ifndef MIMO_CG_H
#define MIMO_CG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MIMO_MAX_USERS 64          /* largest U: mimo_detect_cg (approximate SINR),
                                      mimo_precode_cg, mimo_detect_precode_cg and
                                      mimo_gram_mf with complex64 storage */
#define MIMO_MAX_USERS_COMMON 32   /* largest U of every other call, of 16-bit
                                      storage and of the exact SINR; a larger U
                                      there returns MIMO_EUNSUPPORTED */
#define MIMO_MAX_ANTENNAS 4096
/* Bound on one subcarrier's arrays: S * 8 * max(B, 4 U) bytes must be below
 * this (2^31), i.e. Y and Q (8 B S bytes) and the LLRs (up to 32 U S bytes)
 * of a subcarrier; larger S returns MIMO_EUNSUPPORTED. */
#define MIMO_MAX_SPAN_BYTES 2147483648LL

typedef struct mimo_shape {
  int32_t B;     /* base-station antennas, U <= B <= MIMO_MAX_ANTENNAS */
  int32_t U;     /* single-antenna users, 1 <= U <= B; U <= MIMO_MAX_USERS
                    or MIMO_MAX_USERS_COMMON per entry point */
  int32_t S;     /* right-hand sides per subcarrier (OFDM symbols), >= 1,
                    S * 8 * max(B, 4 U) < MIMO_MAX_SPAN_BYTES */
  int32_t K;     /* CG iterations (Algorithm 1), 1 <= K <= 1024 */
  int64_t n_sc;  /* independent subcarrier systems, >= 0 (0 = no-op) */
} mimo_shape;

/* Storage type of H (and Y) */
enum { MIMO_C32 = 0, MIMO_C16 = 1, MIMO_CBF16 = 2 };
/* In-loop SINR computation (Sec. III-C) */
enum { MIMO_SINR_APPROX = 0, MIMO_SINR_EXACT = 1 };
/* Precision of the CG scalar recurrences (||r||^2, p^H e, alpha, beta) */
enum { MIMO_SCALAR_F32 = 0, MIMO_SCALAR_F64 = 1 };
/* Operations, for mimo_workspace_bytes and the schedule table */
enum { MIMO_OP_GRAM_MF = 0, MIMO_OP_DETECT = 1, MIMO_OP_PRECODE = 2, MIMO_OP_SLOT = 3 };

typedef enum mimo_status {
  MIMO_OK = 0,
  MIMO_EINVAL = -1,        /* bad pointer, size, or parameter value */
  MIMO_EUNSUPPORTED = -2,  /* valid per the paper but not built here */
  MIMO_EWORKSPACE = -3,    /* workspace missing or too small */
  MIMO_EHIP = -4           /* HIP runtime error at launch */
} mimo_status;

/*
 * mimo_gram_mf -- regularized Gram matrix and matched filter.
 * Algorithm 1, initialization (detection): A = H^H H + reg I and b = H^H y
 * for every column y of Y (eq. (8)).  With reg = N0/E_s this is the uplink
 * system; with reg = beta it is the precoding matrix of eq. (16) by
 * reciprocity (H_d H_d^H = H_u^H H_u).
 *   H      [n_sc][B][U], storage type in_dtype
 *   Y      [n_sc][B][S], storage type in_dtype, or NULL (then b is not written)
 *   reg    >= 0, added to the diagonal
 *   A      out, complex64 [n_sc][U][U]; the upper triangle is computed, the
 *          lower triangle is its conjugate mirror, the diagonal is real
 *   b      out, complex64 [n_sc][U][S], or NULL
 * Uses shape->B, U, S, n_sc (K is ignored).  U beyond MIMO_MAX_USERS_COMMON
 * (up to MIMO_MAX_USERS) with complex64 storage only.
 */
mimo_status mimo_gram_mf(const mimo_shape* shape, const void* H, const void* Y,
                 int in_dtype, float reg, void* A, void* b, void* stream);

/*
 * mimo_detect_cg -- CG-based soft-output MMSE detection (Sec. III-B/C).
 * Per subcarrier and right-hand side: A = H^H H + (n0/es) I, b = H^H y,
 * K iterations of Algorithm 1 (v_0 = 0, r_0 = p_0 = b), xhat = v_K; the
 * equalized gain mu and SINR rho tracked inside the recursion, either
 *   MIMO_SINR_APPROX: eq. (13) with A replaced by its diagonal D, giving
 *     mu_i = L~_ii G_ii (eq. (14)) and rho_i = G_ii / N0 (eq. (15)); or
 *   MIMO_SINR_EXACT: the CG-equivalent matrix L_K of eqs. (9), (12), with
 *     mu_i = (L_K G)_ii and rho_i = mu_i^2 / nu_i^2 (Sec. III-C-1);
 * then max-log LLRs (eq. (4)) of z = xhat/mu over square Gray QAM:
 *   llr[..][b] = rho * (min_{a in X_b^0} |z-a|^2 - min_{a in X_b^1} |z-a|^2)
 * (positive favours bit 1).  Constellation: per axis, levels
 * 2j-(L-1), j=0..L-1, L = 2^(qam_bits/2), labelled by the Gray code of j
 * (MSB first); bits [0, qam_bits/2) are the in-phase label, the rest the
 * quadrature label; scaled to average energy es.
 * Degenerate systems: a right-hand side whose residual norm is 0 freezes
 * (alpha = beta = 0); mu = 0 gives z = 0 and rho = G_ii / N0.
 *   n0 > 0, es > 0; qam_bits in {2, 4, 6, 8}
 *   scalar_prec  MIMO_SCALAR_F32 or MIMO_SCALAR_F64 (CG scalars in FP64,
 *                vectors stay FP32)
 *   llr   out, float [n_sc][U][S][qam_bits]            (required)
 *   xhat  out, complex64 [n_sc][U][S] or NULL
 *   mu    out, float [n_sc][U][S] or NULL
 *   sinr  out, float [n_sc][U][S] or NULL
 *   workspace / workspace_bytes: may be NULL / 0 when
 *         mimo_workspace_bytes(shape, MIMO_OP_DETECT, sinr_mode) is 0.
 * U up to MIMO_MAX_USERS_COMMON in every mode and storage type; beyond it,
 * up to MIMO_MAX_USERS, with complex64 storage and MIMO_SINR_APPROX (four
 * wavefronts per subcarrier, one per 16 users, any B and S); other calls
 * with U > MIMO_MAX_USERS_COMMON return MIMO_EUNSUPPORTED.
 */
mimo_status mimo_detect_cg(const mimo_shape* shape, const void* H, const void* Y,
                   int in_dtype, float n0, float es, int qam_bits,
                   int sinr_mode, int scalar_prec, float* llr, void* xhat,
                   float* mu, float* sinr, void* workspace,
                   size_t workspace_bytes, void* stream);

/*
 * mimo_precode_cg -- CG-based linear precoding (Sec. III-D).
 * Solves (H_d H_d^H + beta I) v = t (eq. (16)) by K iterations of
 * Algorithm 1 and returns q = H_d^H v = H_u v (Algorithm 1 output);
 * beta = 0 is zero forcing, beta = N0/E_s the MMSE precoder of eq. (6).
 * With normalize != 0 the output is s = q / ||q||_2 per vector (Sec. II-B;
 * ||q|| = 0 gives s = 0).  qnorm receives ||q||_2 either way.
 *   H  [n_sc][B][U] storage type in_dtype;  T complex64 [n_sc][U][S]
 *   beta >= 0;  Q out complex64 [n_sc][B][S];  qnorm out float [n_sc][S] or NULL
 * U beyond MIMO_MAX_USERS_COMMON (up to MIMO_MAX_USERS) with complex64
 * storage only, as mimo_detect_cg.
 */
mimo_status mimo_precode_cg(const mimo_shape* shape, const void* H, const void* T,
                    int in_dtype, float beta, int normalize, int scalar_prec,
                    void* Q, float* qnorm, void* workspace,
                    size_t workspace_bytes, void* stream);

/*
 * mimo_detect_precode_cg -- one uplink + downlink slot on a reciprocal
 * channel: mimo_detect_cg (approximate SINR) of Y and mimo_precode_cg of T
 * with the same H.  By reciprocity (Sec. II-B, H_d = H_u^H) the two systems
 * share the Gram matrix G = H_u^H H_u = H_d H_d^H, A_u = G + (n0/es) I for
 * detection and A_d = G + beta I for precoding (eq. (16)); the fused kernel
 * forms G once per subcarrier and reads H once for both directions.
 *   ul  B, U, n_sc; S = receive vectors per subcarrier, K = detection
 *       iterations;  dl  the same B, U, n_sc; S = downlink vectors,
 *       K = precoding iterations (S and K may differ between ul and dl)
 *   H   [n_sc][B][U] storage in_dtype;  Y [n_sc][B][ul.S] storage in_dtype;
 *   T   complex64 [n_sc][U][dl.S]
 *   n0, es, qam_bits, scalar_prec, llr, xhat, mu, sinr as mimo_detect_cg;
 *   beta, normalize, Q, qnorm as mimo_precode_cg (scalar_prec applies to
 *   both directions)
 * Outputs are bitwise those of mimo_detect_cg(ul, ...) followed by
 * mimo_precode_cg(dl, ...) on the same inputs.  The fused kernel covers
 * complex64 storage with U <= 16, B <= 128 and S <= 16 in both directions;
 * other calls (and the schedule variant "separate") run the two operations
 * as two launches on `stream`.  U up to MIMO_MAX_USERS as mimo_detect_cg
 * and mimo_precode_cg (complex64 storage beyond MIMO_MAX_USERS_COMMON).
 */
mimo_status mimo_detect_precode_cg(const mimo_shape* ul, const mimo_shape* dl, const void* H,
                           const void* Y, const void* T, int in_dtype, float n0, float es,
                           int qam_bits, float beta, int normalize, int scalar_prec,
                           float* llr, void* xhat, float* mu, float* sinr, void* Q,
                           float* qnorm, void* stream);

/*
 * mimo_detect_cg_gram, mimo_precode_cg_gram -- the same operations with the
 * Gram matrix of the channel supplied instead of formed: G = H^H H (Sec.
 * II-A; = H_d H_d^H by reciprocity, Sec. II-B) of this H, without
 * regularization, e.g. written once per channel by mimo_gram_mf with reg = 0
 * and kept while the channel holds.  The call adds reg = n0/es (detection) or
 * beta (precoding) to the diagonal and reads H only for the matched filter
 * b = H^H y or the output q = H_u v, skipping the Gram's products.
 *   G  complex64 [n_sc][U][U], Hermitian with a real diagonal and an exactly
 *      conjugate lower triangle (mimo_gram_mf's layout)
 * Other arguments, outputs and rules as mimo_detect_cg (approximate SINR)
 * and mimo_precode_cg; U <= MIMO_MAX_USERS_COMMON.  With a G from
 * mimo_gram_mf of the same H (and storage type) and U > 8, outputs are
 * bitwise those of mimo_detect_cg / mimo_precode_cg; at U <= 8 those calls
 * form the Gram in a packed form that rounds differently.
 */
mimo_status mimo_detect_cg_gram(const mimo_shape* shape, const void* G, const void* H,
                                const void* Y, int in_dtype, float n0, float es, int qam_bits,
                                int scalar_prec, float* llr, void* xhat, float* mu, float* sinr,
                                void* stream);
mimo_status mimo_precode_cg_gram(const mimo_shape* shape, const void* G, const void* H,
                                 const void* T, int in_dtype, float beta, int normalize,
                                 int scalar_prec, void* Q, float* qnorm, void* stream);

/*
 * mimo_convert -- channel / receive-vector ingest into reduced precision.
 * Rounds a complex64 array [n][R][C] (R rows = antennas, a multiple of 8)
 * to FP16 or BF16 with round-to-nearest-even and writes the blocked layout
 * described above (dst_dtype MIMO_C16 or MIMO_CBF16).  dst holds
 * n*R*C*2 16-bit values.  Storage format only; no method arithmetic.
 */
mimo_status mimo_convert(const void* src, void* dst, int dst_dtype, int64_t n,
                 int32_t R, int32_t C, void* stream);

/*
 * Batched calls: up to MIMO_MAX_BATCH frames of different shapes in one
 * kernel launch (the serving loop's continuous batching).  Each frame is an
 * independent problem exactly as in mimo_detect_cg / mimo_precode_cg; all
 * frames of one call share in_dtype, qam_bits (detection) and scalar_prec.
 * Detection uses the approximate SINR of eq. (13)-(15).  Every frame is
 * validated before anything is enqueued; a frame with n_sc = 0 is skipped.
 * The descriptor array is read during the call only.
 *   detection:  H [n_sc][B][U], Y [n_sc][B][S] (storage in_dtype),
 *               out = llr float [n_sc][U][S][qam_bits],
 *               out2 = xhat complex64 [n_sc][U][S] or NULL; uses n0, es
 *   precoding:  H [n_sc][B][U] (storage in_dtype), Y = T complex64
 *               [n_sc][U][S], out = Q complex64 [n_sc][B][S],
 *               out2 = qnorm float [n_sc][S] or NULL; uses beta, normalize
 * A frame with gram != NULL runs as mimo_detect_cg_gram / mimo_precode_cg_gram.
 * Results are bitwise identical to the corresponding single-frame calls.
 */
#define MIMO_MAX_BATCH 32

typedef struct mimo_frame {
  int64_t n_sc;
  int32_t B, U, S, K;
  const void* H;
  const void* Y;
  void* out;
  void* out2;
  float n0, es;          /* detection */
  float beta;            /* precoding */
  int32_t normalize;     /* precoding */
  const void* gram;      /* cached G of the frame's H (as mimo_detect_cg_gram), or NULL */
} mimo_frame;

mimo_status mimo_detect_cg_batch(const mimo_frame* frames, int n_frames, int in_dtype, int qam_bits,
                         int scalar_prec, void* stream);
mimo_status mimo_precode_cg_batch(const mimo_frame* frames, int n_frames, int in_dtype,
                          int scalar_prec, void* stream);

/*
 * Comparison methods (Sec. III-F), same layouts and conventions as
 * mimo_detect_cg / mimo_precode_cg.  They form A = H^H H + reg I on MFMA and
 * an explicit inverse X of A per subcarrier, shared by its S right-hand
 * sides, in FP32:
 *   *_cholesky  exact inverse: A = M M^H (Cholesky), X = M^{-H} M^{-1} by
 *               forward substitution (Sec. III-F-1).  shape->K is ignored.
 *               A must be positive definite (reg > 0, or full column rank
 *               for zero-forcing precoding); otherwise outputs are not finite.
 *   *_neumann   X = sum_{k=0}^{K-1} (-D^{-1} E)^k D^{-1}, A = D + E with
 *               D = diag(A), K = shape->K terms (Sec. III-F-2).  Needs
 *               A_ii > 0.
 * Detection: xhat = X H^H y (eq. (3) with X for the inverse of eq. (2));
 * mu_i = (X G)_ii, nu_i^2 = E_s sum_{j != i} |(X G)_ij|^2 + N0 (X G X^H)_ii,
 * rho_i = mu_i^2 / nu_i^2 (Sec. II-A); for the exact inverse these reduce
 * to mu_i = 1 - (N0/E_s)(A^{-1})_ii and rho_i = mu_i / (N0 (A^{-1})_ii),
 * which is what the Cholesky detector evaluates.  mu and sinr are the same
 * for all right-hand sides of a subcarrier.  LLRs and the mu = 0 rule as in
 * mimo_detect_cg.  Precoding: v = X t, q = H_u v (eq. (5) with P of eq. (6)),
 * normalization and qnorm as in mimo_precode_cg.
 */
mimo_status mimo_detect_cholesky(const mimo_shape* shape, const void* H, const void* Y,
                         int in_dtype, float n0, float es, int qam_bits,
                         float* llr, void* xhat, float* mu, float* sinr, void* stream);
mimo_status mimo_detect_neumann(const mimo_shape* shape, const void* H, const void* Y,
                        int in_dtype, float n0, float es, int qam_bits,
                        float* llr, void* xhat, float* mu, float* sinr, void* stream);
mimo_status mimo_precode_cholesky(const mimo_shape* shape, const void* H, const void* T,
                          int in_dtype, float beta, int normalize, void* Q,
                          float* qnorm, void* stream);
mimo_status mimo_precode_neumann(const mimo_shape* shape, const void* H, const void* T,
                         int in_dtype, float beta, int normalize, void* Q,
                         float* qnorm, void* stream);
/*
 * CGLS on the augmented systems (Sec. III-E).  No Gram matrix is formed;
 * each of the K iterations runs q = Hbar p and s = Hbar^H r with H on MFMA.
 *   mimo_detect_cgls   min_x ||[y; 0] - [H; sqrt(N0/E_s) I] x|| (eq. (17))
 *                      from x_0 = 0; xhat = x_K.  The approximate SINR of
 *                      eqs. (13)-(15) runs on the CGLS step sizes
 *                      (d_i = ||h_i||^2 + N0/E_s); exact SINR is not offered.
 *                      LLRs, outputs and degenerate-case rules as
 *                      mimo_detect_cg (a zero ||s||^2 freezes the rhs).
 *   mimo_precode_cgls  min ||t - [H_d, sqrt(beta) I] qbar|| (eq. (18)) from
 *                      qbar_0 = 0; q = the first B entries of qbar_K (the
 *                      minimum-norm solution at K = U, eq. (6)); normalization
 *                      and qnorm as mimo_precode_cg.
 * Recursion per rhs (residual kept, s recomputed):
 *   r_0 = ybar, s_0 = Hbar^H r_0, p_0 = s_0, gamma_0 = ||s_0||^2;
 *   q = Hbar p, alpha = gamma/||q||^2, x += alpha p, r -= alpha q,
 *   s = Hbar^H r, gamma' = ||s||^2, beta_k = gamma'/gamma, p = s + beta_k p.
 * scalar_prec as mimo_detect_cg.  Antenna-length vectors of 16 right-hand
 * sides stay in LDS (B/16 x 2 KiB for detection, 3x that for precoding);
 * a B beyond the device's LDS per block returns MIMO_EUNSUPPORTED.
 */
mimo_status mimo_detect_cgls(const mimo_shape* shape, const void* H, const void* Y,
                     int in_dtype, float n0, float es, int qam_bits, int scalar_prec,
                     float* llr, void* xhat, float* mu, float* sinr, void* stream);
mimo_status mimo_precode_cgls(const mimo_shape* shape, const void* H, const void* T,
                      int in_dtype, float beta, int normalize, int scalar_prec,
                      void* Q, float* qnorm, void* stream);
/*
 * Kernel schedules (not part of the paper's method: how the same arithmetic
 * is mapped onto the GPU).  Each operation has kernel variants and a grid
 * size; the pair used for (op, user class, storage type) comes from a
 * process-wide table that an autotuner fills by timing the variants.
 *   user_class    0: U <= 16, 1: 16 < U <= 32 (calls with a larger U run
 *                 the four-wavefront kernels whatever the table holds)
 *   variant       0 .. mimo_tune_variant_count(op) - 1 (detection: 0 generic,
 *                 1 stream = next subcarrier's loads in flight during CG,
 *                 2 stream with half-size load blocks; variant 1/2 apply for
 *                 S <= 16, larger S always uses 0; 3 plain = the baseline
 *                 mapping with VALU Gram/CG and one right-hand side at a time,
 *                 complex64 storage only, other storage uses 0; precoding:
 *                 0 generic, 1 stream, 2 stream-small, the same prefetching
 *                 forms, for S <= 16; 3 resident = H kept in registers from
 *                 the Gram to q = H v so that it is read once, for U <= 16,
 *                 S <= 16 and B <= 128 in any storage type; other shapes use
 *                 1, or 0 when S > 16; Gram + matched filter: 0 generic,
 *                 1 stream = next block and next subcarrier in flight, for
 *                 S <= 16 or no Y, larger S uses 0; uplink + downlink slot:
 *                 0 separate = two launches with the detection and precoding
 *                 schedules, 1 fused = one H-resident kernel where
 *                 mimo_detect_precode_cg allows it, else 0)
 *                 Further detection variants (measured forms, correct for
 *                 every shape, never faster on the workloads measured):
 *                 4 ring = chunks of H and Y loaded straight into an LDS
 *                 ring (complex64, U <= 16, S <= 16, LLRs only), 5 split =
 *                 four wavefronts per subcarrier over antenna quarters
 *                 (complex64, U <= 32, S <= 16), 6 stream-valu = stream with
 *                 the CG mat-vec on VALU FMAs; precoding 4 split (complex64,
 *                 U <= 32, S <= 16, B <= 256).  Where a variant does not
 *                 cover a call, stream-small runs.  split and stream-valu
 *                 sum in another order: equal to the others to rounding.
 *   blocks_per_cu 0: one wavefront per subcarrier; k in [1, 64]: persistent
 *                 grid of k four-wavefront blocks per compute unit
 * Results do not depend on the schedule (every variant other than split
 * and stream-valu performs the same operations in the same order per
 * system).  mimo_tune_set is not
 * synchronized with launches already enqueued; it affects later calls.
 */
mimo_status mimo_tune_set(int op, int user_class, int in_dtype, int variant, int blocks_per_cu);
mimo_status mimo_tune_get(int op, int user_class, int in_dtype, int* variant, int* blocks_per_cu);
int mimo_tune_variant_count(int op);
const char* mimo_tune_variant_name(int op, int variant);   /* NULL if out of range */

/* Device workspace (bytes) that an operation needs; 0 means none. */
size_t mimo_workspace_bytes(const mimo_shape* shape, int op, int sinr_mode);

/* Static description of a status code. */
const char* mimo_status_string(mimo_status status);

/* Text of the last error recorded by this thread (validation or HIP). */
const char* mimo_last_error(void);

/* Library version string. */
const char* mimo_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MIMO_CG_H */
