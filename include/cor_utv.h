/*
 * cor_utv.h -- C ABI of the MI355X (gfx950) CoR-UTV library, libcorutv.so.
 *
 * Compressed Randomized UTV with power iteration (Kaloorazi & de Lamare,
 * "Compressed Randomized UTV Decompositions for Low-Rank Approximations and
 * Big Data Applications", Sec. III, Alg. 2 and Alg. 3).  Given A (m x n) and
 * integers k <= l = k + p < min(m, n) and q >= 0, the library returns a
 * rank-l approximation A ~ U T V^T with U (m x l) and V (n x l) orthonormal
 * and T (l x l) upper triangular whose diagonal tracks the leading singular
 * values of A (the URV form of eq. (16)).
 *
 * What runs, per decomposition (all on the GPU):
 *   X = Omega (i.i.d. N(0,1), n x l)                      [Alg. 3, step 1]
 *   repeat q+1 times:                                      [Alg. 3, loop]
 *     Y1 = A X          -> Q1 R1 = Y1 (CholeskyQR2, FP64)  [eq. (11)]
 *     Y2 = A^T Q1       -> Q2 R2 = Y2 (CholeskyQR2, FP64)  [eq. (12)]
 *     X  = Q2
 *   M = Q1^T A Q2 = R2^T                                   [eq. (14)]
 *   M P = Qt T  (column-pivoted QR, FP64)                  [eq. (15)]
 *   U = Q1 Qt,  V = Q2 P                                   [eq. (16)]
 * The second sketch uses Q1 instead of the paper's un-normalised C1 and every
 * product with A is orthonormalised before the next one; both leave Q1, Q2 and
 * M unchanged in exact arithmetic.  M = R2^T holds because
 * Q1^T A Q2 = (A^T Q1)^T Q2 = (Q2 R2)^T Q2.
 *
 * Conventions
 *   - Matrices are row-major: element (i, j) of an r x c matrix with leading
 *     dimension ld is at index i*ld + j.
 *   - Every matrix pointer is a DEVICE pointer (hipMalloc'd or a torch CUDA
 *     tensor's data pointer) unless stated otherwise.  The caller owns A and
 *     the outputs; the library never writes A.  The library owns its
 *     workspace (a per-device pool that grows on demand and is released by
 *     cor_release() or at unload).
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Outputs are always FP64.  T has exact zeros below the diagonal and a
 *     non-negative diagonal.  perm (optional) receives the QRCP permutation:
 *     V[:, j] = Q2[:, perm[j]].
 *   - Every call returns a cor_status; no C++ exception crosses the ABI.
 *     cor_last_error() returns a message for the last failure on the calling
 *     thread.
 */
#ifndef COR_UTV_H
#define COR_UTV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    COR_OK = 0,
    COR_E_INVAL = 1,    /* bad argument (shape, rank parameters, null pointer, lda)        */
    COR_E_NOMEM = 2,    /* device or host allocation failed                                 */
    COR_E_DEVICE = 3,   /* a HIP call failed                                                */
    COR_E_NUMERIC = 4,  /* a non-finite value reached a Gram matrix (NaN/Inf in A)          */
    COR_E_BUSY = 5,     /* served request still running (cor_server_poll)                   */
    COR_E_NOTFOUND = 6  /* unknown ticket                                                   */
} cor_status;

/* Storage format of A, which is also the arithmetic format of the passes over
 * A (MFMA with FP32 accumulation; FP64 MFMA in COR_F64).  The Gram matrices,
 * Cholesky factors, orthonormal bases and the l x l core stay FP64. */
typedef enum {
    COR_F64 = 0,   /* double                                                      */
    COR_F32 = 1,   /* float                                                       */
    COR_BF16 = 2,  /* bfloat16 (binary32 rounded to nearest even), 2 bytes         */
    COR_FP8 = 3    /* OCP FP8 E4M3FN codes with a per-column FP32 scale, 1 byte:   */
                   /* A[i][j] ~ fp8(code[i][j]) * colscale[j]                       */
} cor_prec;

/* cor_info.flags (bit 0 is unused).  A Cholesky pivot of a sketch's Gram
 * matrix at or below l 2^-52 max_i G_ii (a numerically rank-deficient sketch,
 * or one too ill-conditioned for CholeskyQR) is clamped to that threshold;
 * at the final orthonormalisation the columns whose pivot was clamped are
 * replaced by Gaussian columns, so U and V stay orthonormal. */
#define COR_FLAG_RANK_DEFICIENT 2 /* a pivot was clamped in some orthonormalisation    */
#define COR_FLAG_NONFINITE 4      /* a non-finite value reached a Gram matrix          */
#define COR_FLAG_SYNC_TIMEOUT 8   /* l > 224: the QRCP's work-groups gave up waiting   */
                                  /* for each other (results unusable; COR_E_DEVICE)   */

typedef struct {
    double err_l;     /* ||A - U T V^T||_F / ||A||_F  (report >= 1; identity 1 - ||T||^2/||A||^2) */
    double err_k;     /* ||A - U[:, :k] T[:k, :] V^T||_F / ||A||_F (report >= 1)                  */
    double orth_u;    /* ||U^T U - I||_F (report >= 1)                                            */
    double orth_v;    /* ||V^T V - I||_F (report >= 1)                                            */
    double device_ms; /* device time of the call, or submit-to-completion for served requests    */
    int32_t flags;    /* COR_FLAG_*                                                               */
    int32_t l;        /* k + p                                                                    */
    double m_check;   /* COR_M_EXPLICIT / COR_M_APPROX with report: ||M - R2^T||_F / ||M||_F,   */
                      /* the compressed matrix against the identity M = R2^T (0 otherwise)      */
} cor_info;

/* One decomposition request. */
typedef struct {
    const void* A;         /* device, m x n row-major with leading dimension lda, format `prec`  */
    const float* colscale; /* device, n floats; required for COR_FP8, ignored otherwise          */
    int64_t m, n, lda;     /* lda >= n                                                            */
    int32_t k, p, q;       /* l = k + p; k >= 1, p >= 0, 2 <= l < min(m, n), l <= 264, 0 <= q <= 16 */
    int32_t prec;          /* cor_prec                                                            */
    uint64_t seed;         /* Omega from the counter-based generator of cor_omega()               */
    const double* omega;   /* optional device n x l FP64 test matrix; overrides seed             */
    double* U;             /* device out, m x l                                                   */
    double* T;             /* device out, l x l                                                   */
    double* V;             /* device out, n x l                                                   */
    int32_t* perm;         /* optional device out, l int32                                        */
} cor_problem;

/* Compression of A to the l x l core M (cor_opts.compress):
 *   COR_M_R2T      (default) M = Q1^T A Q2 = R2^T: no further pass over A, since
 *                  A^T Q1 = Q2 R2 (eq. (14) without its product);
 *   COR_M_EXPLICIT M = Q1^T (A Q2) as eq. (14) prints it: one more pass over A
 *                  (a check of the identity, reported as cor_info.m_check);
 *   COR_M_APPROX   M = Q1^T Y1 (Q2^T X)^+ = R1 (Q2^T X)^-1, eq. (18), with Y1 = A X
 *                  the last power step's sketch (X = Omega when q = 0, else the
 *                  previous Q2; the non-updated C2 of Alg. 3): no further pass,
 *                  an l x l solve (Gauss-Jordan, partial pivoting) instead.
 * Orientation (cor_opts.orient): COR_URV (default) returns T upper triangular
 * for every shape; COR_ULV returns A ~ U L V^T with L lower triangular
 * (Sec. III: the other orientation, for m < n), computed as the URV of A^T
 * (a transposed copy of A in the workspace; not available for COR_FP8):
 * U = V', L = T'^T, V = U'.  For ULV the optional test matrix `omega` is
 * m x l, perm permutes the columns of U (U[:, j] = Q[:, perm[j]] for the
 * row-space basis Q), and the rank-k truncation is U L[:, :k] V[:, :k]^T. */
/* Fused power step (cor_opts.fused_power = 1): for the q steps before the
 * final pair, one pass over A forms Y = A^T (A X) (each block of rows of A is
 * read from HBM once and used for both products), then R1 = chol(X^T Y), the
 * Cholesky factor of the first sketch's Gram (A X)^T (A X), and Y R1^{-1} =
 * A^T Q1 as in the two-pass step.  Passes over A: q + 2 instead of 2q + 2.
 * It pays where the passes are bound by HBM bandwidth (FP32 with l < 20,
 * FP64 with l < 39, e.g. tall matrices with a small rank).  Each block of a
 * pass keeps its share of the n x l result in registers, so it requires
 * COR_F32 or COR_F64 passes, l <= 64, n <= 2400 (FP32) or n <= 1024 (FP64),
 * and ceil(n / 16) * ceil(l / 16) <= 8 T with T = 24 (FP32, l <= 32), 16
 * (FP32, l > 32), 12 (FP64, l <= 32) or 8 (FP64, l > 32) -- n is the column
 * count of the matrix the passes read, m for COR_ULV -- and one q for all
 * problems of a batched call; else COR_E_INVAL. */
#define COR_M_R2T 0
#define COR_M_EXPLICIT 1
#define COR_M_APPROX 2
#define COR_URV 0
#define COR_ULV 1

typedef struct {
    int32_t report;      /* 0: nothing; 1: fill err_l, err_k, orth_u, orth_v of cor_info         */
    int32_t cholqr2_all; /* 0 (default): one CholeskyQR pass after each product inside the power  */
                         /*   loop and two for the final pair (the spans are the same in exact    */
                         /*   arithmetic); 1: two passes after every product                      */
    int32_t compress;    /* COR_M_R2T (0, default), COR_M_EXPLICIT, COR_M_APPROX                 */
    int32_t orient;      /* COR_URV (0, default) or COR_ULV                                       */
    int32_t fused_power; /* 1: each power step before the final pair reads A once, forming        */
                         /*   A^T (A X) as Alg. 3's loop prints it (see below); 0 (default): two  */
                         /*   passes, A X then A^T Q1                                             */
} cor_opts;

/* ---------------------------------------------------------------------------
 * Single decomposition with the inputs of Alg. 3 (A, k, l = k + p, q) plus the
 * seed of the Gaussian test matrix.  A has lda = n.  COR_FP8 needs a column
 * scale and is only reachable through cor_utv_ex.  Returns after the work on
 * `stream` has completed; `info` may be NULL.
 * ------------------------------------------------------------------------- */
cor_status cor_utv(const void* A, int64_t m, int64_t n, int32_t k, int32_t p, int32_t q,
                   uint64_t seed, int32_t prec, double* U, double* T, double* V,
                   cor_info* info, void* stream);

/* Same with every option; opts may be NULL (defaults: report 0, cholqr2_all 0). */
cor_status cor_utv_ex(const cor_problem* prob, const cor_opts* opts, cor_info* info,
                      void* stream);

/* `count` independent decompositions of uneven shapes, run as grouped launches
 * (one launch per stage and per column-tile class covers every problem).
 * infos (optional) receives count records.  Returns after completion. */
cor_status cor_utv_batched(const cor_problem* probs, int32_t count, const cor_opts* opts,
                           cor_info* infos, void* stream);

/* ---------------------------------------------------------------------------
 * A in host memory (larger than HBM, or not resident): the pass model of
 * Sec. III with A stored outside the fast memory, where each pass over A is
 * the cost (2q + 2 passes, q + 2 with cor_opts.fused_power).  prob->A is a
 * HOST pointer (m x n, leading dimension lda, format prec; page-locked memory
 * from hipHostMalloc gives full copy bandwidth, pageable memory also works);
 * colscale, omega and the outputs are device pointers as for cor_utv_ex.
 * Every pass streams A in panels of `panel_rows` rows (<= 0: about 256 MiB per
 * panel; rounded up to a multiple of 128) through two device staging
 * buffers, the copy of the next panel overlapping the kernels of the current
 * one.  The device holds the m x l and n x l factors and the panels only.
 * Results equal cor_utv_ex's up to the order of the K-split partial sums.
 * Not available with report = 1, COR_M_EXPLICIT or COR_ULV (COR_E_INVAL).
 * Returns after the work on `stream` has completed; device_ms covers the
 * whole call, copies included.
 * ------------------------------------------------------------------------- */
cor_status cor_utv_host(const cor_problem* prob, const cor_opts* opts, int64_t panel_rows,
                        cor_info* info, void* stream);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code that must not call
 * hipMalloc: tight serving loops, harnesses that forbid allocation): the
 * decomposition of cor_utv_ex run entirely inside a fixed array of
 * COR_NOALLOC_SCRATCH_BYTES of device memory that the library holds per
 * device from the time its code is loaded until the process ends.  Same
 * arguments, kernels and results (bit for bit) as cor_utv_ex; device_ms is
 * not measured (0).  The plan (descriptor, launch tables, workspace) must fit
 * the array: cor_workspace_bytes(m, n, l, prec) <= COR_NOALLOC_SCRATCH_BYTES,
 * else COR_E_INVAL with the sizes in cor_last_error().  No hipMalloc, hipFree
 * or other allocating device call is made.  Returns after the work on
 * `stream` has completed.  All calls on one device share that device's
 * array, which keeps the last call's contents (each call clears what must
 * start at zero): calls from several threads of one process are serialised
 * by the library; work that overlaps a call on the same device and touches
 * the array by other means races with it.
 * ------------------------------------------------------------------------- */
#define COR_NOALLOC_SCRATCH_BYTES (64u << 20)
cor_status cor_utv_ex_noalloc(const cor_problem* prob, const cor_opts* opts, cor_info* info,
                              void* stream);

/* ---------------------------------------------------------------------------
 * Robust PCA, M = L + S with L of low rank and S sparse, by the augmented
 * Lagrange multiplier method with CoR-UTV as its low-rank step (Sec. V,
 * ALM-CoRUTV).  Iteration j, penalty mu_j, delta = 1 / mu_j:
 *   B = M - S_j + Y_j / mu_j (B_0 = M);  U T V = CoR-UTV(B) with k, p, q, the
 *   same Gaussian test matrix (seed) every iteration;  r = #{i : T_ii > delta};
 *   L_j+1 = U[:, :r] (T[:r, :] - delta [I_r 0]) V^T;
 *   S_j+1 = shrink(M - L_j+1 + Y_j / mu_j, lambda / mu_j) with
 *   shrink(x, d) = sgn(x) max(|x| - d, 0);  Y_j+1 = Y_j + mu_j (M - L_j+1 - S_j+1);
 *   mu_j+1 = min(rho mu_j, mu_bar),
 * until zeta = ||M - L - S||_F / ||M||_F < tol or max_iter iterations.
 * mu_0 = 1.25 / T_11 of the first decomposition (an estimate of ||M||_2),
 * mu_bar = mu_bar_ratio mu_0.  Fields <= 0 take the defaults named below.
 * M: device, m x n FP64 row-major, leading dimension ldm >= n (read only).
 * L, S: device out, m x n FP64 with leading dimension n (the last iterate).
 * The library allocates its workspace (Y, B in `prec`, the factors; about
 * (16 + 8 or 4) m n bytes) for the call and frees it before returning.
 * Returns after the work on `stream` has completed (the host reads zeta and
 * r back after every iteration).  COR_E_INVAL for bad shapes or rank
 * parameters (as cor_utv), COR_E_NUMERIC if M is zero or not finite.
 * ------------------------------------------------------------------------- */
typedef struct {
    int32_t k, p, q;      /* rank parameters of the CoR-UTV step (as cor_problem)              */
    int32_t prec;         /* COR_F64 or COR_F32: format of B and of the passes over it           */
    uint64_t seed;        /* Gaussian test matrix (cor_omega's stream)                           */
    double lambda;        /* sparsity weight (<= 0: 1 / sqrt(max(m, n)))                          */
    double rho;           /* penalty growth (<= 0: 1.5)                                           */
    double mu_bar_ratio;  /* penalty cap over mu_0 (<= 0: 1e7)                                    */
    double tol;           /* stop when zeta < tol (<= 0: 1e-5)                                    */
    int32_t max_iter;     /* iteration cap (<= 0: 100)                                            */
} cor_rpca_opts;
typedef struct {
    int32_t iters;        /* iterations run                                                       */
    int32_t rank;         /* r of the last iteration (the rank of L)                              */
    double zeta;          /* ||M - L - S||_F / ||M||_F after the last iteration                   */
    double mu;            /* penalty of the last iteration                                        */
    double ms;            /* host wall time of the call                                           */
} cor_rpca_info;
cor_status cor_rpca_alm(const double* M, int64_t m, int64_t n, int64_t ldm,
                        const cor_rpca_opts* opts, double* L, double* S, cor_rpca_info* info,
                        void* stream);

/* ---------------------------------------------------------------------------
 * Plans: the executor behind the calls above, exposed for callers that replay
 * the same decomposition(s) many times.  A plan owns its workspace and
 * device-side descriptors; cor_plan_run() only enqueues kernels on `stream`
 * (no allocation, no host synchronisation, no memset), so it may be captured
 * into a HIP graph.  cor_plan_capture() records one run into a graph that
 * later cor_plan_run() calls replay with hipGraphLaunch.
 * ------------------------------------------------------------------------- */
typedef struct cor_plan cor_plan;
cor_status cor_plan_create(const cor_problem* probs, int32_t count, const cor_opts* opts,
                           cor_plan** plan);
cor_status cor_plan_run(cor_plan* plan, void* stream);
cor_status cor_plan_capture(cor_plan* plan, void* stream);
/* Waits for `stream`, then reads back flags and the report of each problem. */
cor_status cor_plan_info(cor_plan* plan, cor_info* infos, void* stream);
cor_status cor_plan_destroy(cor_plan* plan);

/* ---------------------------------------------------------------------------
 * Served decompositions with continuous batching.  A server thread admits
 * queued requests while their workspace fits the HBM budget and a slot is
 * free.  The requests admitted together form a round: one grouped launch per
 * stage covers all of them, on a stream of its own, so rounds run
 * concurrently on the device.  A round retires as soon as its own pipeline
 * completes; requests that arrive while rounds run form the next round
 * without waiting for the device to drain.  A request's result does not
 * depend on what runs beside it (fixed reduction orders).
 * A, outputs and colscale must stay valid until the request completes.
 * ------------------------------------------------------------------------- */
typedef struct cor_server cor_server;
typedef struct {
    size_t hbm_budget;  /* bytes of workspace the server may hold (0: 64 GiB)               */
    int32_t max_slots;  /* requests in flight at once (0: 32)                                */
    int32_t convert_f32_to; /* COR_F32 (0 = keep) or COR_BF16: FP32 requests are converted    */
                            /* once on the device and their passes run in BF16                */
} cor_server_cfg;
typedef struct {
    double p50_ms, p99_ms, mean_ms; /* submit-to-completion latency of completed requests      */
    double decomps_per_s;           /* completed / (last completion - first submission)        */
    int64_t completed, queued, active, rejected;
    size_t hbm_in_use, hbm_high_water;
} cor_server_stats;

cor_status cor_server_create(const cor_server_cfg* cfg, cor_server** server);
/* Enqueue a request (thread-safe).  COR_E_INVAL if it is malformed or can never
 * fit the budget. */
cor_status cor_server_submit(cor_server* server, const cor_problem* prob, const cor_opts* opts,
                             uint64_t* ticket);
/* COR_OK and *info filled when done, COR_E_BUSY while queued or running. */
cor_status cor_server_poll(cor_server* server, uint64_t ticket, cor_info* info);
cor_status cor_server_wait(cor_server* server, uint64_t ticket, cor_info* info);
cor_status cor_server_stats_get(cor_server* server, cor_server_stats* stats);
cor_status cor_server_destroy(cor_server* server);

/* ---------------------------------------------------------------------------
 * Split tuner with a JSON cache.  The K-split counts of the two passes over A
 * follow a fixed rule of the shape (about 512 blocks per launch).  cor_tune
 * measures, on the caller's matrix (prob: URV, default options), the pass
 * kernels' mean time over `reps` launches for candidate split counts (A X
 * first, then A^T X) and stores the fastest pair in the library's tuning
 * table under (m, n, l, prec); every plan created afterwards for that shape
 * uses them (cached plans are dropped).  s_ax, s_atx (optional) receive the
 * chosen counts.  cor_tune_save writes the table as JSON:
 *   {"version": 1, "entries": [{"m": .., "n": .., "l": .., "prec": ..,
 *    "s_ax": .., "s_atx": .., "us_ax": .., "us_atx": ..}, ...]}
 * cor_tune_load merges such a file into the table (COR_E_INVAL if it is
 * unreadable or an entry is out of range: 1 <= s <= 64); the file named by
 * the environment variable COR_TUNE_FILE is loaded before the first plan.
 * A shape's result depends only on the shape and the table, not on what it
 * is batched with.
 * ------------------------------------------------------------------------- */
cor_status cor_tune(const cor_problem* prob, int32_t reps, int32_t* s_ax, int32_t* s_atx,
                    void* stream);
cor_status cor_tune_save(const char* path);
cor_status cor_tune_load(const char* path);
cor_status cor_tune_clear(void);

/* ---------------------------------------------------------------------------
 * Helpers
 * ------------------------------------------------------------------------- */
/* Device workspace of one decomposition of an m x n matrix with l = k + p
 * (the unit of the server's admission control). */
size_t cor_workspace_bytes(int64_t m, int64_t n, int32_t l, int32_t prec);

/* Convert an FP32 device matrix (m x n, lda) to the storage format `to`
 * (COR_BF16: out is m x n uint16 with ld n; COR_FP8: out is m x n bytes with
 * ld n and colscale receives n floats, s_j = max_i |A_ij| / 448 (1 for an
 * all-zero column), code = E4M3FN(A_ij / s_j) rounded to nearest even with
 * saturation at +-448). */
cor_status cor_quantize(const float* A32, int64_t m, int64_t n, int64_t lda, int32_t to,
                        void* out, float* colscale, void* stream);

/* The Gaussian test matrix of Alg. 3, step 1, written to device memory as an
 * n x l FP64 row-major array.  Integer t of the stream is output t of
 * SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) started at `seed`; the pair
 * (2j, 2j+1) of the row-major array is the Box-Muller transform of
 * u1 = ((s(2j) >> 11) + 1) 2^-53 and u2 = (s(2j+1) >> 11) 2^-53:
 * sqrt(-2 ln u1) * (cos, sin)(2 pi u2).  Device libm: values agree with a host
 * implementation of the same definition to a few ulp. */
cor_status cor_omega(uint64_t seed, int64_t n, int32_t l, double* out, void* stream);

/* Kernel timing of the passes over A for roofline reports: while enabled, each
 * launch of the pass kernels is bracketed by HIP events on its own stream.
 * on: 0 off; 1 the two-pass kernels (A X, A^T X); 2 the fused power step's
 * kernel (A^T (A X)); 3 both.
 * cor_profile_read() synchronises those events and returns the summed time
 * (ms), the number of launches and the algorithmic bytes and flops of those
 * launches, then resets the counters. */
cor_status cor_profile_enable(int32_t on);
cor_status cor_profile_read(double* ms, int64_t* launches, double* bytes, double* flops);

const char* cor_status_string(int32_t status);
const char* cor_last_error(void);
/* Free the workspace pool and cached plans of every device. */
cor_status cor_release(void);

#ifdef __cplusplus
}
#endif
#endif /* COR_UTV_H */
