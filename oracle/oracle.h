/*
 * CoR-UTV FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded implementation of Compressed Randomized UTV
 * with power iteration (Kaloorazi & de Lamare, "Compressed Randomized UTV
 * Decompositions for Low-Rank Approximations and Big Data Applications",
 * Sec. III, Alg. 2 and Alg. 3).  It exists to check the GPU library; only the
 * test suite, the smoke check and the CPU baseline leg of the benchmark may
 * load it.  It shares no code, header, table or constant with the GPU path.
 *
 * Conventions: every matrix is row-major, element (i, j) of an r x c matrix
 * with leading dimension ld lives at [i*ld + j].  All arithmetic is IEEE
 * binary64 in plain loops; no BLAS, no LAPACK, no threads.
 *
 * Readings of the paper that the oracle fixes (the paper is silent or
 * inconsistent on these points):
 *   - the second sketch is Y2 = A^T Q1 (the paper writes C2 = A^T C1; both
 *     give the same Q2 in exact arithmetic, since C1 = Q1 R1);
 *   - inside the power loop every product with A is orthonormalised before
 *     the next one (same column spaces in exact arithmetic; the
 *     un-normalised loop loses all precision after one power step);
 *   - every QR has a non-negative diagonal in R (unique thin QR);
 *   - the QRCP is Businger-Golub: the pivot is the trailing column of largest
 *     exactly recomputed 2-norm, lowest index on ties, Householder
 *     reflections, and finally T_jj >= 0;
 *   - the right factor is V = Q2 P (the algorithm boxes print Q2 P^T, which
 *     does not reproduce A from D = Q~ R~ P^T);
 *   - T is upper triangular for every shape.
 */
#ifndef COR_ORACLE_H
#define COR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2 };

/* Standard Gaussian test matrix (Alg. 3, first step): n x l, row-major, from a
 * counter-based stream.  Integer t of the stream is output t of SplitMix64
 * (Steele, Lea & Flood, OOPSLA 2014) started from `seed`; element pair
 * (2j, 2j+1) of the row-major array is the Box-Muller transform of the
 * 53-bit uniforms u1 = (s(2j) >> 11 + 1) 2^-53 in (0,1] and
 * u2 = (s(2j+1) >> 11) 2^-53 in [0,1):  r = sqrt(-2 ln u1), z = r cos(2 pi u2),
 * r sin(2 pi u2). */
void orc_omega(uint64_t seed, int64_t n, int32_t l, double* out);
uint64_t orc_splitmix64(uint64_t seed, uint64_t index);

/* Thin Householder QR Y = Q R of an r x c matrix (r >= c), diag(R) >= 0. */
int orc_qr(const double* Y, int64_t r, int32_t c, int64_t ldy, double* Q, double* R);

/* Column-pivoted QR of an l x l matrix: M P = Qt T with P = I[:, perm].
 * min_gap (optional) receives the smallest relative gap, over all steps,
 * between the largest and second largest trailing column norm. */
int orc_qrcp(const double* M, int32_t l, double* Qt, double* T, int32_t* perm, double* min_gap);

/* CoR-UTV with power iteration.  Inputs: A (m x n, lda), k, p, q, Omega
 * (n x l, row-major, l = k + p).  Outputs: U (m x l), T (l x l, upper, exact
 * zeros below), V (n x l), perm (l).  Optional (NULL to skip): Q1 (m x l),
 * Q2 (n x l), M = Q1^T A Q2 (l x l, computed explicitly), R2 (l x l, the
 * R factor of the last Y2).  diag (optional, 4 doubles):
 *   [0] ||M - R2^T||_F / ||M||_F, [1] min relative pivot gap of the QRCP,
 *   [2] ||Q1^T Q1 - I||_F, [3] ||Q2^T Q2 - I||_F. */
int orc_cor_utv(const double* A, int64_t m, int64_t n, int64_t lda, int32_t k, int32_t p,
                int32_t q, const double* omega, double* U, double* T, double* V,
                int32_t* perm, double* Q1, double* Q2, double* M, double* R2, double* diag);

/* Alg. 3 with the passes over A read in a storage format, as the reduced-
 * precision modes compute it: fmt is ORC_FMT_F64 (the plain method),
 * ORC_FMT_F32, ORC_FMT_BF16 or ORC_FMT_FP8.  Aq holds the decoded stored
 * values of A (FP8: the decoded codes; A = Aq diag(colscale)).  Each pass
 * reads its skinny operand in the same format (binary32; bfloat16 of the
 * binary32 value; FP8 with per-column scales over diag(colscale) X on the n
 * side), forms the product exactly in FP64 and applies the scales; the
 * compression is D = Q1q^T A Q2 with Q1q the operand the second product read.
 * Everything else is FP64 as in orc_cor_utv.  Outputs as orc_cor_utv. */
enum { ORC_FMT_F64 = 0, ORC_FMT_F32 = 1, ORC_FMT_BF16 = 2, ORC_FMT_FP8 = 3 };
int orc_cor_utv_fmt(const double* Aq, int64_t m, int64_t n, int64_t lda, int32_t fmt,
                    const float* colscale, int32_t k, int32_t p, int32_t q,
                    const double* omega, double* U, double* T, double* V, int32_t* perm,
                    double* diag);

/* Accuracy report: out[0] = ||A - U T V^T||_F / ||A||_F,
 * out[1] = ||A - U[:, :k] T[:k, :] V^T||_F / ||A||_F, out[2] = ||U^T U - I||_F,
 * out[3] = ||V^T V - I||_F. */
void orc_metrics(const double* A, int64_t m, int64_t n, int64_t lda, const double* U,
                 const double* T, const double* V, int32_t l, int32_t k, double* out);

/* Plain products used by the tests to evaluate single steps on samples:
 * C (r x c) = A (r x kk, lda) B (kk x c, ldb);  C (kk x c) = A^T B with A r x kk. */
void orc_gemm_nn(const double* A, int64_t r, int64_t kk, int64_t lda, const double* B,
                 int64_t c, int64_t ldb, double* C);
void orc_gemm_tn(const double* A, int64_t r, int64_t kk, int64_t lda, const double* B,
                 int64_t c, int64_t ldb, double* C);

/* Storage formats of the reduced-precision modes.
 * bf16: round-to-nearest-even of binary32 to its upper 16 bits.
 * fp8 : OCP E4M3FN (bias 7, no infinities, 0x7F/0xFF NaN, max 448), nearest
 *       value with ties to the even code, saturating at +-448.
 * Per-column FP8 storage: s_j = max_i |A_ij| / 448 in binary32 (s_j = 1 for an
 * all-zero column) and code_ij = fp8(A_ij / s_j) with a binary32 division. */
uint16_t orc_bf16_from_f32(float x);
double orc_bf16_to_f64(uint16_t h);
uint8_t orc_fp8_from_f32(float x);
double orc_fp8_to_f64(uint8_t c);
void orc_quantize_bf16(const float* A, int64_t m, int64_t n, int64_t lda, uint16_t* out);
void orc_quantize_fp8(const float* A, int64_t m, int64_t n, int64_t lda, uint8_t* out,
                      float* colscale);

#ifdef __cplusplus
}
#endif
#endif
