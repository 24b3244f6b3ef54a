/*
 * CoR-UTV FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Follows Sec. III of the paper: Alg. 2 (no power iteration) and Alg. 3
 * (power method), the compression D = Q1^T A Q2 of eq. (14), the QRCP
 * D = Q~ R~ P~^T of eq. (15) and the assembly U = Q1 Q~, T = R~,
 * V = Q2 P~ of eq. (16).  Accuracy measures follow the rank-l error
 * (eq. (43), here in the Frobenius norm) and the rank-k truncation
 * U(:,1:k) T(1:k,:) V^T of Sec. VI-B.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((int64_t)(i) * (int64_t)(ld) + (int64_t)(j))

/* ------------------------------------------------------------------------ */
/* Gaussian test matrix Psi (Alg. 2 / Alg. 3, first step).                   */
/* ------------------------------------------------------------------------ */
uint64_t orc_splitmix64(uint64_t seed, uint64_t index) {
    /* Output `index` (0-based) of SplitMix64: state advances by the golden
     * gamma before each output; the output is the state run through the
     * variant-13 finaliser of MurmurHash3. */
    uint64_t z = seed + (index + 1u) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

void orc_omega(uint64_t seed, int64_t n, int32_t l, double* out) {
    const int64_t total = n * (int64_t)l;
    const double two_pi = 6.283185307179586; /* 2 pi rounded to binary64 */
    for (int64_t t = 0; t < total; t += 2) {
        uint64_t pair = (uint64_t)(t / 2);
        double u1 = (double)((orc_splitmix64(seed, 2 * pair) >> 11) + 1u) * 0x1.0p-53;
        double u2 = (double)(orc_splitmix64(seed, 2 * pair + 1) >> 11) * 0x1.0p-53;
        double r = sqrt(-2.0 * log(u1));
        double th = two_pi * u2;
        out[t] = r * cos(th);
        if (t + 1 < total) out[t + 1] = r * sin(th);
    }
}

/* ------------------------------------------------------------------------ */
/* Plain products.                                                           */
/* ------------------------------------------------------------------------ */
void orc_gemm_nn(const double* A, int64_t r, int64_t kk, int64_t lda, const double* B,
                 int64_t c, int64_t ldb, double* C) {
    for (int64_t i = 0; i < r; i++) {
        double* ci = C + i * c;
        for (int64_t j = 0; j < c; j++) ci[j] = 0.0;
        for (int64_t t = 0; t < kk; t++) {
            double a = A[IDX(i, t, lda)];
            const double* bt = B + t * ldb;
            for (int64_t j = 0; j < c; j++) ci[j] += a * bt[j];
        }
    }
}

void orc_gemm_tn(const double* A, int64_t r, int64_t kk, int64_t lda, const double* B,
                 int64_t c, int64_t ldb, double* C) {
    for (int64_t i = 0; i < kk * c; i++) C[i] = 0.0;
    for (int64_t t = 0; t < r; t++) {
        const double* at = A + t * lda;
        const double* bt = B + t * ldb;
        for (int64_t i = 0; i < kk; i++) {
            double a = at[i];
            double* ci = C + i * c;
            for (int64_t j = 0; j < c; j++) ci[j] += a * bt[j];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Householder reflections.                                                  */
/* Column j of the r x c work matrix W (rows j..r-1) is reflected onto       */
/* beta e_1 by H = I - tau v v^T with v_j = 1; v_{i>j} overwrite W[i][j].    */
/* ------------------------------------------------------------------------ */
static void house_column(double* W, int64_t r, int32_t c, int32_t j, double* tau) {
    double ss = 0.0;
    for (int64_t i = j; i < r; i++) ss += W[IDX(i, j, c)] * W[IDX(i, j, c)];
    double xnorm = sqrt(ss);
    double alpha = W[IDX(j, j, c)];
    if (xnorm == 0.0) {
        *tau = 0.0;
        return;
    }
    double beta = alpha >= 0.0 ? -xnorm : xnorm;
    double scale = 1.0 / (alpha - beta);
    for (int64_t i = j + 1; i < r; i++) W[IDX(i, j, c)] *= scale;
    *tau = (beta - alpha) / beta;
    W[IDX(j, j, c)] = beta;
}

/* Apply H_j (stored in column j of W) to columns j+1..c-1 of W. */
static void house_apply_trailing(double* W, int64_t r, int32_t c, int32_t j, double tau) {
    if (tau == 0.0) return;
    for (int32_t cc = j + 1; cc < c; cc++) {
        double w = W[IDX(j, cc, c)];
        for (int64_t i = j + 1; i < r; i++) w += W[IDX(i, j, c)] * W[IDX(i, cc, c)];
        w *= tau;
        W[IDX(j, cc, c)] -= w;
        for (int64_t i = j + 1; i < r; i++) W[IDX(i, cc, c)] -= w * W[IDX(i, j, c)];
    }
}

/* Q (r x c) = H_0 H_1 ... H_{c-1} [I_c; 0], reflectors stored in W. */
static void house_form_q(const double* W, int64_t r, int32_t c, const double* tau, double* Q) {
    for (int64_t i = 0; i < r; i++)
        for (int32_t j = 0; j < c; j++) Q[IDX(i, j, c)] = (i == j) ? 1.0 : 0.0;
    for (int32_t j = c - 1; j >= 0; j--) {
        if (tau[j] == 0.0) continue;
        for (int32_t cc = j; cc < c; cc++) {
            double w = Q[IDX(j, cc, c)];
            for (int64_t i = j + 1; i < r; i++) w += W[IDX(i, j, c)] * Q[IDX(i, cc, c)];
            w *= tau[j];
            Q[IDX(j, cc, c)] -= w;
            for (int64_t i = j + 1; i < r; i++) Q[IDX(i, cc, c)] -= w * W[IDX(i, j, c)];
        }
    }
}

int orc_qr(const double* Y, int64_t r, int32_t c, int64_t ldy, double* Q, double* R) {
    if (r < c || c < 1 || ldy < c) return ORC_EINVAL;
    double* W = (double*)malloc(sizeof(double) * (size_t)(r * c));
    double* tau = (double*)malloc(sizeof(double) * (size_t)c);
    if (!W || !tau) {
        free(W);
        free(tau);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < r; i++)
        for (int32_t j = 0; j < c; j++) W[IDX(i, j, c)] = Y[IDX(i, j, ldy)];
    for (int32_t j = 0; j < c; j++) {
        house_column(W, r, c, j, &tau[j]);
        house_apply_trailing(W, r, c, j, tau[j]);
    }
    for (int32_t i = 0; i < c; i++)
        for (int32_t j = 0; j < c; j++) R[IDX(i, j, c)] = (j >= i) ? W[IDX(i, j, c)] : 0.0;
    house_form_q(W, r, c, tau, Q);
    /* Unique thin QR: make diag(R) non-negative. */
    for (int32_t j = 0; j < c; j++) {
        if (R[IDX(j, j, c)] < 0.0) {
            for (int32_t cc = j; cc < c; cc++) R[IDX(j, cc, c)] = -R[IDX(j, cc, c)];
            for (int64_t i = 0; i < r; i++) Q[IDX(i, j, c)] = -Q[IDX(i, j, c)];
        }
    }
    free(W);
    free(tau);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* QRCP of the compressed matrix, eq. (15): D P~ = Q~ R~.               */
/* ------------------------------------------------------------------------ */
int orc_qrcp(const double* M, int32_t l, double* Qt, double* T, int32_t* perm, double* min_gap) {
    if (l < 1) return ORC_EINVAL;
    double* W = (double*)malloc(sizeof(double) * (size_t)l * (size_t)l);
    double* tau = (double*)malloc(sizeof(double) * (size_t)l);
    double* nrm = (double*)malloc(sizeof(double) * (size_t)l);
    if (!W || !tau || !nrm) {
        free(W);
        free(tau);
        free(nrm);
        return ORC_ENOMEM;
    }
    memcpy(W, M, sizeof(double) * (size_t)l * (size_t)l);
    for (int32_t j = 0; j < l; j++) perm[j] = j;
    double gap = 1.0;
    for (int32_t j = 0; j < l; j++) {
        /* Exact trailing column norms, recomputed at every step. */
        for (int32_t c = j; c < l; c++) {
            double ss = 0.0;
            for (int32_t i = j; i < l; i++) ss += W[IDX(i, c, l)] * W[IDX(i, c, l)];
            nrm[c] = sqrt(ss);
        }
        int32_t p = j;
        for (int32_t c = j + 1; c < l; c++)
            if (nrm[c] > nrm[p]) p = c; /* strict: lowest index wins a tie */
        if (l - j >= 2 && nrm[p] > 0.0) {
            double second = -1.0;
            for (int32_t c = j; c < l; c++)
                if (c != p && nrm[c] > second) second = nrm[c];
            double g = (nrm[p] - second) / nrm[p];
            if (g < gap) gap = g;
        }
        if (p != j) {
            for (int32_t i = 0; i < l; i++) {
                double t = W[IDX(i, j, l)];
                W[IDX(i, j, l)] = W[IDX(i, p, l)];
                W[IDX(i, p, l)] = t;
            }
            int32_t t = perm[j];
            perm[j] = perm[p];
            perm[p] = t;
        }
        house_column(W, l, l, j, &tau[j]);
        house_apply_trailing(W, l, l, j, tau[j]);
    }
    for (int32_t i = 0; i < l; i++)
        for (int32_t j = 0; j < l; j++) T[IDX(i, j, l)] = (j >= i) ? W[IDX(i, j, l)] : 0.0;
    house_form_q(W, l, l, tau, Qt);
    /* Diagonal of T approximates singular values: make it non-negative. */
    for (int32_t j = 0; j < l; j++) {
        if (T[IDX(j, j, l)] < 0.0) {
            for (int32_t cc = j; cc < l; cc++) T[IDX(j, cc, l)] = -T[IDX(j, cc, l)];
            for (int32_t i = 0; i < l; i++) Qt[IDX(i, j, l)] = -Qt[IDX(i, j, l)];
        }
    }
    if (min_gap) *min_gap = gap;
    free(W);
    free(tau);
    free(nrm);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Helpers for the diagnostics.                                              */
/* ------------------------------------------------------------------------ */
static double orth_loss(const double* Q, int64_t r, int32_t c) {
    /* G = Q^T Q accumulated row by row: every entry still sums over i in
     * increasing order, while the reads of Q stay contiguous. */
    double* G = (double*)calloc((size_t)c * (size_t)c, sizeof(double));
    if (!G) return NAN;
    for (int64_t i = 0; i < r; i++) {
        const double* qi = Q + i * (int64_t)c;
        for (int32_t a = 0; a < c; a++) {
            const double qa = qi[a];
            double* ga = G + (int64_t)a * c;
            for (int32_t b = 0; b < c; b++) ga[b] += qa * qi[b];
        }
    }
    double s = 0.0;
    for (int32_t a = 0; a < c; a++)
        for (int32_t b = 0; b < c; b++) {
            double g = G[IDX(a, b, c)];
            if (a == b) g -= 1.0;
            s += g * g;
        }
    free(G);
    return sqrt(s);
}

/* ------------------------------------------------------------------------ */
/* Alg. 3 (Alg. 2 when q = 0).                                               */
/* ------------------------------------------------------------------------ */
/* Skinny operand of a pass in a stored-format mode: the FP64 factor F
 * (r x l) as the pass reads it.  FP32: binary32 rounding; BF16: the binary32
 * value rounded to bfloat16; FP8: F' = diag(rowscale) F (rowscale = the
 * column scales of A on the n side, none on the m side), column scales
 * t_c = max_r |binary32(F'[r][c])| / 448 (1 for a zero column) and codes
 * E4M3(binary32(F'[r][c]) / t_c).  out receives the decoded values (without
 * t), tsc the column scales (1 except in FP8). */
static void quantize_operand(int32_t fmt, const double* F, int64_t r, int32_t l,
                             const float* rowscale, double* out, double* tsc) {
    for (int32_t c = 0; c < l; c++) tsc[c] = 1.0;
    if (fmt == ORC_FMT_F32) {
        for (int64_t i = 0; i < r * l; i++) out[i] = (double)(float)F[i];
    } else if (fmt == ORC_FMT_BF16) {
        for (int64_t i = 0; i < r * l; i++) out[i] = orc_bf16_to_f64(orc_bf16_from_f32((float)F[i]));
    } else {
        for (int32_t c = 0; c < l; c++) {
            float mx = 0.0f;
            for (int64_t i = 0; i < r; i++) {
                double x = F[IDX(i, c, l)];
                if (rowscale) x *= (double)rowscale[i];
                float v = fabsf((float)x);
                if (v > mx) mx = v;
            }
            const float t = mx > 0.0f ? mx / 448.0f : 1.0f;
            tsc[c] = (double)t;
            for (int64_t i = 0; i < r; i++) {
                double x = F[IDX(i, c, l)];
                if (rowscale) x *= (double)rowscale[i];
                out[IDX(i, c, l)] = orc_fp8_to_f64(orc_fp8_from_f32((float)x / t));
            }
        }
    }
}

/* Alg. 3 with the passes over A read in a storage format (FP64 when fmt is
 * ORC_FMT_F64, which is the plain method).  Aq holds the decoded stored
 * values of A (for FP8 the decoded codes, without the column scales).  In the
 * other formats the two products are
 *   C1 = Aq Xq diag(t)                       (Xq: quantize_operand of X, with
 *                                             rowscale = colscale in FP8)
 *   C2 = diag(colscale) Aq^T Q1q diag(t)     (Q1q: quantize_operand of Q1)
 * with colscale = 1 outside FP8, and the compression is eq. (14) with the
 * operand the pass read on the left, D = Q1q^T (A Q2) (in exact arithmetic
 * the R2^T of that second sketch).  U, T, V are assembled from the FP64
 * factors as in eq. (16). */
static int cor_utv_core(const double* A, int64_t m, int64_t n, int64_t lda, int32_t fmt,
                        const float* colscale, int32_t k, int32_t p, int32_t q,
                        const double* omega, double* U, double* T, double* V, int32_t* perm,
                        double* Q1o, double* Q2o, double* Mo, double* R2o, double* diag) {
    const int32_t l = k + p;
    const int64_t mn = m < n ? m : n;
    if (k < 1 || p < 0 || q < 0 || l < 2 || (int64_t)l >= mn || lda < n) return ORC_EINVAL;
    if (!A || !omega || !U || !T || !V || !perm) return ORC_EINVAL;
    if (fmt < ORC_FMT_F64 || fmt > ORC_FMT_FP8 || (fmt == ORC_FMT_FP8 && !colscale))
        return ORC_EINVAL;

    size_t sz_m = sizeof(double) * (size_t)m * (size_t)l;
    size_t sz_n = sizeof(double) * (size_t)n * (size_t)l;
    size_t sz_l = sizeof(double) * (size_t)l * (size_t)l;
    double* X = (double*)malloc(sz_n);
    double* Y1 = (double*)malloc(sz_m);
    double* Q1 = (double*)malloc(sz_m);
    double* R1 = (double*)malloc(sz_l);
    double* Y2 = (double*)malloc(sz_n);
    double* Q2 = (double*)malloc(sz_n);
    double* R2 = (double*)malloc(sz_l);
    double* Z = (double*)malloc(sz_m);
    double* M = (double*)malloc(sz_l);
    double* Qt = (double*)malloc(sz_l);
    if (!X || !Y1 || !Q1 || !R1 || !Y2 || !Q2 || !R2 || !Z || !M || !Qt) {
        free(X); free(Y1); free(Q1); free(R1); free(Y2);
        free(Q2); free(R2); free(Z); free(M); free(Qt);
        return ORC_ENOMEM;
    }
    memcpy(X, omega, sz_n);
    /* Operands of the stored-format passes (unused in FP64). */
    double* Xq = NULL;
    double* Q1q = NULL;
    double* tsc = NULL;
    if (fmt != ORC_FMT_F64) {
        Xq = (double*)malloc(sz_n);
        Q1q = (double*)malloc(sz_m);
        tsc = (double*)malloc(sizeof(double) * (size_t)l);
        if (!Xq || !Q1q || !tsc) {
            free(Xq); free(Q1q); free(tsc);
            free(X); free(Y1); free(Q1); free(R1); free(Y2);
            free(Q2); free(R2); free(Z); free(M); free(Qt);
            return ORC_ENOMEM;
        }
    }
    const float* rs = fmt == ORC_FMT_FP8 ? colscale : NULL;

    /* Power loop (Alg. 3): C1 = A C2, C2 = A^T C1, q + 1 times, each product
     * orthonormalised before it is used. */
    for (int32_t it = 0; it <= q; it++) {
        if (fmt == ORC_FMT_F64) {
            orc_gemm_nn(A, m, n, lda, X, l, l, Y1);    /* C1 = A X        */
        } else {
            quantize_operand(fmt, X, n, l, rs, Xq, tsc);
            orc_gemm_nn(A, m, n, lda, Xq, l, l, Y1);
            for (int64_t i = 0; i < m; i++)
                for (int32_t c = 0; c < l; c++) Y1[IDX(i, c, l)] *= tsc[c];
        }
        orc_qr(Y1, m, l, l, Q1, R1);               /* C1 = Q1 R1      */
        if (fmt == ORC_FMT_F64) {
            orc_gemm_tn(A, m, n, lda, Q1, l, l, Y2);   /* C2 = A^T Q1     */
        } else {
            quantize_operand(fmt, Q1, m, l, NULL, Q1q, tsc);
            orc_gemm_tn(A, m, n, lda, Q1q, l, l, Y2);
            for (int64_t i = 0; i < n; i++)
                for (int32_t c = 0; c < l; c++)
                    Y2[IDX(i, c, l)] *= (rs ? (double)rs[i] : 1.0) * tsc[c];
        }
        orc_qr(Y2, n, l, l, Q2, R2);               /* C2 = Q2 R2      */
        memcpy(X, Q2, sz_n);
    }

    /* Compression D = Q1^T A Q2, eq. (14), by its definition (with the left
     * operand the second sketch read, in a stored format). */
    if (fmt == ORC_FMT_F64) {
        orc_gemm_nn(A, m, n, lda, Q2, l, l, Z);
        orc_gemm_tn(Q1, m, l, l, Z, l, l, M);
    } else {
        double* Q2s = (double*)malloc(sz_n); /* diag(colscale) Q2: A = Aq diag(colscale) */
        if (!Q2s) {
            free(Xq); free(Q1q); free(tsc);
            free(X); free(Y1); free(Q1); free(R1); free(Y2);
            free(Q2); free(R2); free(Z); free(M); free(Qt);
            return ORC_ENOMEM;
        }
        for (int64_t i = 0; i < n; i++)
            for (int32_t c = 0; c < l; c++)
                Q2s[IDX(i, c, l)] = (rs ? (double)rs[i] : 1.0) * Q2[IDX(i, c, l)];
        orc_gemm_nn(A, m, n, lda, Q2s, l, l, Z);
        orc_gemm_tn(Q1q, m, l, l, Z, l, l, M);
        if (fmt == ORC_FMT_FP8)
            for (int32_t a = 0; a < l; a++)
                for (int32_t b = 0; b < l; b++) M[IDX(a, b, l)] *= tsc[a];
        free(Q2s);
    }
    free(Xq); free(Q1q); free(tsc);

    double gap = 1.0;
    orc_qrcp(M, l, Qt, T, perm, &gap);            /* D P~ = Q~ R~     */

    /* Assembly: U = Q1 Q~, T = R~, V = Q2 P~. */
    orc_gemm_nn(Q1, m, l, l, Qt, l, l, U);
    for (int64_t i = 0; i < n; i++)
        for (int32_t j = 0; j < l; j++) V[IDX(i, j, l)] = Q2[IDX(i, perm[j], l)];

    if (diag) {
        double num = 0.0, den = 0.0;
        for (int32_t a = 0; a < l; a++)
            for (int32_t b = 0; b < l; b++) {
                double d = M[IDX(a, b, l)] - R2[IDX(b, a, l)];
                num += d * d;
                den += M[IDX(a, b, l)] * M[IDX(a, b, l)];
            }
        diag[0] = den > 0.0 ? sqrt(num / den) : 0.0;
        diag[1] = gap;
        diag[2] = orth_loss(Q1, m, l);
        diag[3] = orth_loss(Q2, n, l);
    }
    if (Q1o) memcpy(Q1o, Q1, sz_m);
    if (Q2o) memcpy(Q2o, Q2, sz_n);
    if (Mo) memcpy(Mo, M, sz_l);
    if (R2o) memcpy(R2o, R2, sz_l);

    free(X); free(Y1); free(Q1); free(R1); free(Y2);
    free(Q2); free(R2); free(Z); free(M); free(Qt);
    return ORC_OK;
}

int orc_cor_utv(const double* A, int64_t m, int64_t n, int64_t lda, int32_t k, int32_t p,
                int32_t q, const double* omega, double* U, double* T, double* V,
                int32_t* perm, double* Q1o, double* Q2o, double* Mo, double* R2o,
                double* diag) {
    return cor_utv_core(A, m, n, lda, ORC_FMT_F64, NULL, k, p, q, omega, U, T, V, perm, Q1o,
                        Q2o, Mo, R2o, diag);
}

int orc_cor_utv_fmt(const double* Aq, int64_t m, int64_t n, int64_t lda, int32_t fmt,
                    const float* colscale, int32_t k, int32_t p, int32_t q,
                    const double* omega, double* U, double* T, double* V, int32_t* perm,
                    double* diag) {
    return cor_utv_core(Aq, m, n, lda, fmt, colscale, k, p, q, omega, U, T, V, perm, NULL, NULL,
                        NULL, NULL, diag);
}

/* ------------------------------------------------------------------------ */
/* Accuracy report.                                                          */
/* ------------------------------------------------------------------------ */
void orc_metrics(const double* A, int64_t m, int64_t n, int64_t lda, const double* U,
                 const double* T, const double* V, int32_t l, int32_t k, double* out) {
    /* W = T V^T (l x n), stored transposed (Wt[j][a] = W[a][j]) so that the
     * sums below run over contiguous memory. */
    double* Wt = (double*)malloc(sizeof(double) * (size_t)l * (size_t)n);
    if (!Wt) {
        out[0] = out[1] = out[2] = out[3] = NAN;
        return;
    }
    for (int32_t a = 0; a < l; a++)
        for (int64_t j = 0; j < n; j++) {
            double s = 0.0;
            for (int32_t b = 0; b < l; b++) s += T[IDX(a, b, l)] * V[IDX(j, b, l)];
            Wt[IDX(j, a, l)] = s;
        }
    double na = 0.0, rl = 0.0, rk = 0.0;
    for (int64_t i = 0; i < m; i++) {
        for (int64_t j = 0; j < n; j++) {
            double hk = 0.0;
            for (int32_t a = 0; a < k; a++) hk += U[IDX(i, a, l)] * Wt[IDX(j, a, l)];
            double hl = hk;
            for (int32_t a = k; a < l; a++) hl += U[IDX(i, a, l)] * Wt[IDX(j, a, l)];
            double x = A[IDX(i, j, lda)];
            na += x * x;
            rl += (x - hl) * (x - hl);
            rk += (x - hk) * (x - hk);
        }
    }
    out[0] = na > 0.0 ? sqrt(rl / na) : 0.0;
    out[1] = na > 0.0 ? sqrt(rk / na) : 0.0;
    out[2] = orth_loss(U, m, l);
    out[3] = orth_loss(V, n, l);
    free(Wt);
}

/* ------------------------------------------------------------------------ */
/* Storage formats of the reduced-precision modes.                           */
/* ------------------------------------------------------------------------ */
static float f32_from_bits(uint32_t b) {
    float f;
    memcpy(&f, &b, 4);
    return f;
}
static uint32_t bits_from_f32(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    return b;
}

/* Exact value of a binary32 bit pattern, with the all-ones exponent read as
 * the next power of two (2^128) so that overflow rounds like any other step. */
static double f32_pattern_value(uint32_t b) {
    if ((b & 0x7F800000u) == 0x7F800000u) return (b & 0x80000000u) ? -0x1p128 : 0x1p128;
    return (double)f32_from_bits(b);
}

uint16_t orc_bf16_from_f32(float x) {
    uint32_t b = bits_from_f32(x);
    if (isnan(x)) return (uint16_t)((b >> 16) | 0x0040u);
    if (isinf(x)) return (uint16_t)(b >> 16);
    /* The two bf16 neighbours of x: truncation toward zero and the next one
     * away from zero; take the nearer, the one with an even last bit on a tie. */
    uint32_t lo = b & 0xFFFF0000u;
    if (lo == b) return (uint16_t)(b >> 16);
    uint32_t hi = lo + 0x10000u;
    double dx = (double)x;
    double elo = fabs(dx - f32_pattern_value(lo));
    double ehi = fabs(f32_pattern_value(hi) - dx);
    if (elo < ehi) return (uint16_t)(lo >> 16);
    if (ehi < elo) return (uint16_t)(hi >> 16);
    return ((lo >> 16) & 1u) ? (uint16_t)(hi >> 16) : (uint16_t)(lo >> 16);
}

double orc_bf16_to_f64(uint16_t h) { return (double)f32_from_bits((uint32_t)h << 16); }

double orc_fp8_to_f64(uint8_t c) {
    int s = (c >> 7) & 1, e = (c >> 3) & 15, m = c & 7;
    if (e == 15 && m == 7) return NAN;
    double v = (e == 0) ? ldexp((double)m / 8.0, -6) : ldexp(1.0 + (double)m / 8.0, e - 7);
    return s ? -v : v;
}

uint8_t orc_fp8_from_f32(float x) {
    if (isnan(x)) return 0x7F;
    double a = fabs((double)x);
    uint8_t sign = signbit(x) ? 0x80 : 0x00;
    if (a >= 448.0) return sign | 0x7E; /* saturate */
    /* Nearest of the 127 finite non-negative codes, ties to the even code. */
    uint8_t best = 0;
    double berr = a;
    for (int c = 1; c <= 0x7E; c++) {
        double err = fabs(orc_fp8_to_f64((uint8_t)c) - a);
        if (err < berr || (err == berr && (c & 1) == 0)) {
            best = (uint8_t)c;
            berr = err;
        }
    }
    return sign | best;
}

void orc_quantize_bf16(const float* A, int64_t m, int64_t n, int64_t lda, uint16_t* out) {
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++) out[IDX(i, j, n)] = orc_bf16_from_f32(A[IDX(i, j, lda)]);
}

void orc_quantize_fp8(const float* A, int64_t m, int64_t n, int64_t lda, uint8_t* out,
                      float* colscale) {
    for (int64_t j = 0; j < n; j++) {
        float mx = 0.0f;
        for (int64_t i = 0; i < m; i++) {
            float v = fabsf(A[IDX(i, j, lda)]);
            if (v > mx) mx = v;
        }
        colscale[j] = (mx > 0.0f) ? mx / 448.0f : 1.0f;
    }
    for (int64_t i = 0; i < m; i++)
        for (int64_t j = 0; j < n; j++)
            out[IDX(i, j, n)] = orc_fp8_from_f32(A[IDX(i, j, lda)] / colscale[j]);
}
