// Robust PCA by ALM with CoR-UTV as the low-rank step (ALM-CoRUTV, Sec. V):
// M = L + S with L of low rank and S sparse.  Iteration j (mu_j the penalty,
// delta = 1 / mu_j):
//   B      = M - S_j + Y_j / mu_j                    (B_0 = M)
//   U T V  = CoR-UTV(B)                              (a plan over the B buffer)
//   r      = #{i : T_ii > delta},  T'' = T[:r, :] - delta [I_r 0] (rows >= r zero)
//   L_j+1  = U T'' V^T                               (the operator C_delta)
//   S_j+1  = shrink(M - L_j+1 + Y_j / mu_j, lambda / mu_j)
//   Y_j+1  = Y_j + mu_j (M - L_j+1 - S_j+1)
//   mu_j+1 = min(rho mu_j, mu_bar)
// until zeta = ||M - L - S||_F / ||M||_F < tol.  The product L = Z V^T with
// Z = U T'' runs on the FP64 MFMA and the updates of S, Y and the next B are
// its epilogue, so one kernel reads M, S, Y once and writes L, S, Y, B once
// per iteration.  mu_0 = 1.25 / T_11 of the first decomposition (whose input
// is M), mu_bar = mu_0 * mu_bar_ratio; lambda defaults to 1/sqrt(max(m, n)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "../../include/cor_utv.h"
#include "common.h"
#include "runtime.h"

namespace cor {

constexpr int RP_TILE = 64;  // output tile of the product kernels (4 waves of 32 x 32)
constexpr int RP_KC = 16;    // K per LDS stage
constexpr int RP_LD = RP_KC + 1;  // LDS row stride in doubles (odd: 8-byte reads spread over banks)

// One block's 64 x 64 tile of sum_{k < l} A(i, k) B(k, j) on the FP64 MFMA
// (16x16x4), each wave a 32 x 32 block (2 x 2 MFMA tiles).  A(i, k) is row i
// of a row-major array with l columns (rows clamped to the matrix: rows past
// it only feed entries that are never written).  B(k, j) is either row j of
// such an array (B_ROWS: B = X^T) or entry (k, j) of an l x l row-major array
// (rows k >= bk read as zero).  Every K chunk of 16 is staged through LDS by
// coalesced loads (four threads per 128-byte row segment), double-buffered:
// the loads of chunk c + 1 are in flight while chunk c feeds the MFMAs.
template <bool B_ROWS>
__device__ __forceinline__ void rp_product(const double* __restrict__ A, int64_t arows,
                                           int64_t i0, const double* __restrict__ Bm,
                                           int64_t brows, int64_t j0, int l, int bk,
                                           double* __restrict__ sa, double* __restrict__ sb,
                                           f64x4 (&acc)[2][2]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int wr = 32 * (wave >> 1), wc = 32 * (wave & 1);
    // staging map: A (and B_ROWS) rows: thread -> (row tid / 4, K quarter tid % 4);
    // B as [k][j]: thread -> (k = tid / 16, j = 4 (tid % 16) .. + 3)
    const int srow = tid >> 2, sq = 4 * (tid & 3);
    const double* ar = A + std::min<int64_t>(i0 + srow, arows - 1) * l;
    const double* br = B_ROWS ? Bm + std::min<int64_t>(j0 + srow, brows - 1) * l : nullptr;
    const int bkk = tid >> 4, bj = 4 * (tid & 15);
    double ra[4], rb[4];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int k = k0 + sq + e;
            ra[e] = k < l ? ar[k] : 0.0;
            if (B_ROWS) {
                rb[e] = k < l ? br[k] : 0.0;
            } else {
                const int kb = k0 + bkk;
                const int64_t j = std::min<int64_t>(j0 + bj + e, brows - 1);
                rb[e] = kb < bk ? Bm[(int64_t)kb * l + j] : 0.0;
            }
        }
    };
    auto stash = [&](int buf) {
        double* a = sa + buf * RP_TILE * RP_LD;
        double* b = sb + buf * RP_TILE * RP_LD;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            a[srow * RP_LD + sq + e] = ra[e];
            if (B_ROWS) b[srow * RP_LD + sq + e] = rb[e];
            else b[(bj + e) * RP_LD + bkk] = rb[e];  // stored [j][k] like the row case
        }
    };
#pragma unroll
    for (int x = 0; x < 2; x++)
#pragma unroll
        for (int y = 0; y < 2; y++) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
    const int nc = (l + RP_KC - 1) / RP_KC;
    fetch(0);
    stash(0);
    __syncthreads();
    for (int c = 0; c < nc; c++) {
        const int buf = c & 1;
        if (c + 1 < nc) fetch((c + 1) * RP_KC);
        const double* a = sa + buf * RP_TILE * RP_LD;
        const double* b = sb + buf * RP_TILE * RP_LD;
#pragma unroll
        for (int kk = 0; kk < RP_KC; kk += 4) {
            double x[2], y[2];
#pragma unroll
            for (int t = 0; t < 2; t++) {
                x[t] = a[(wr + 16 * t + li) * RP_LD + kk + lg];
                y[t] = b[(wc + 16 * t + li) * RP_LD + kk + lg];
            }
#pragma unroll
            for (int t = 0; t < 2; t++)
#pragma unroll
                for (int u = 0; u < 2; u++)
                    acc[t][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[t], y[u], acc[t][u], 0, 0, 0);
        }
        if (c + 1 < nc) stash(buf ^ 1);
        __syncthreads();
    }
}

// r = #{i : T_ii > delta} for the whole block (every thread gets it).
__device__ __forceinline__ int rp_rank(const double* __restrict__ T, int l, double delta) {
    int r = 0;
    for (int i0 = 0; i0 < l; i0 += 256) {
        const int i = i0 + (int)threadIdx.x;
        r += __syncthreads_count(i < l && T[i * l + i] > delta);
    }
    return r;
}

// Z = U T'' (m x l) with T'' = rows < r of T, its diagonal shrunk by delta:
// T''(k, j) = T(k, j) - delta [k == j] for k < r, 0 below.  One 64 x 64 tile
// of Z per block; block 0 also stores r.
__global__ __launch_bounds__(256) void k_rpca_z(const double* __restrict__ U,
                                                const double* __restrict__ T, int64_t m, int l,
                                                double delta, double* __restrict__ Z,
                                                int* __restrict__ rout) {
    __shared__ double sa[2 * RP_TILE * RP_LD], sb[2 * RP_TILE * RP_LD];
    const int r = rp_rank(T, l, delta);
    if (blockIdx.x == 0 && threadIdx.x == 0) *rout = r;
    const int tcs = (l + RP_TILE - 1) / RP_TILE;
    const int64_t i0 = (int64_t)(blockIdx.x / tcs) * RP_TILE;
    const int j0 = (blockIdx.x % tcs) * RP_TILE;
    f64x4 acc[2][2];
    rp_product<false>(U, m, i0, T, l, j0, l, r, sa, sb, acc);
    // the shrink: Z(i, j) -= delta U(i, j) for j < r
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t wi = i0 + 32 * (wave >> 1);
    const int wj = j0 + 32 * (wave & 1);
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                // f64 MFMA output: lane (li, lg), entry e -> row lg + 4 e, column li
                const int64_t i = wi + 16 * a + lg + 4 * e;
                const int j = wj + 16 * b + li;
                if (i >= m || j >= l) continue;
                const double u = U[i * l + j];
                Z[i * l + j] = j < r ? fma(-delta, u, acc[a][b][e]) : acc[a][b][e];
            }
}

// The L product and the ALM updates, one 64 x 64 tile of (i, j) per block:
// L = Z V^T on the FP64 MFMA, then per entry
//   W = M - L + Y / mu, S = shrink(W, lam / mu), R = M - L - S, Y += mu R,
//   B = M - S + Y / mu_next (in B's format),
// and the block's sum of R^2 (for zeta) in a fixed order.
template <typename TB>
__global__ __launch_bounds__(256) void k_rpca_update(
    const double* __restrict__ Z, const double* __restrict__ V, int l, const double* __restrict__ M,
    int64_t ldm, double* __restrict__ L, double* __restrict__ S, double* __restrict__ Y,
    TB* __restrict__ B, int64_t m, int64_t n, double mu, double mu_next, double lam,
    double* __restrict__ zpart) {
    __shared__ double red[4];
    __shared__ double sa[2 * RP_TILE * RP_LD], sb[2 * RP_TILE * RP_LD];
    const int64_t tcs = (n + RP_TILE - 1) / RP_TILE;
    const int64_t i0 = (int64_t)(blockIdx.x / tcs) * RP_TILE;
    const int64_t j0 = (int64_t)(blockIdx.x % tcs) * RP_TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t wi = i0 + 32 * (wave >> 1), wj = j0 + 32 * (wave & 1);
    f64x4 acc[2][2];
    rp_product<true>(Z, m, i0, V, n, j0, l, l, sa, sb, acc);
    const double imu = 1.0 / mu, imun = 1.0 / mu_next, thr = lam / mu;
    double zs = 0.0;
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                // f64 MFMA output: lane (li, lg), entry e -> row lg + 4 e, column li
                const int64_t i = wi + 16 * a + lg + 4 * e, j = wj + 16 * b + li;
                if (i >= m || j >= n) continue;
                const int64_t o = i * n + j;
                const double lv = acc[a][b][e];
                const double mv = M[i * ldm + j];
                const double yv = Y[o];
                const double w = mv - lv + yv * imu;
                const double sv = w > thr ? w - thr : (w < -thr ? w + thr : 0.0);
                const double rv = mv - lv - sv;
                const double yn = fma(mu, rv, yv);
                L[o] = lv;
                S[o] = sv;
                Y[o] = yn;
                B[o] = (TB)(mv - sv + yn * imun);
                zs = fma(rv, rv, zs);
            }
    // block sum of R^2 in a fixed order: wave shuffles, then the four waves
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) zs += __shfl_xor(zs, off, 64);
    if (lane == 0) red[wave] = zs;
    __syncthreads();
    if (threadIdx.x == 0) zpart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// B = M (the first iteration), in B's format; and ||M||_F^2 partials.
template <typename TB>
__global__ __launch_bounds__(256) void k_rpca_init(const double* __restrict__ M, int64_t ldm,
                                                   int64_t m, int64_t n, TB* __restrict__ B,
                                                   double* __restrict__ S, double* __restrict__ Y,
                                                   double* __restrict__ npart) {
    __shared__ double red[4];
    const int64_t e0 = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    for (int64_t e = e0; e < m * n; e += (int64_t)gridDim.x * 256) {
        const int64_t i = e / n, j = e - (e / n) * n;
        const double v = M[i * ldm + j];
        B[e] = (TB)v;
        S[e] = 0.0;
        Y[e] = 0.0;
        s = fma(v, v, s);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) npart[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// Sum of `count` partials in a fixed order: thread t adds entries t, t + 1024,
// ... in turn, then a pairwise tree over the threads (one block of 1024).
__global__ __launch_bounds__(1024) void k_rpca_sum(const double* __restrict__ part, int count,
                                                   double* __restrict__ out) {
    __shared__ double sh[1024];
    double v = 0.0;
    for (int i = threadIdx.x; i < count; i += 1024) v += part[i];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

}  // namespace cor

using namespace cor;

extern "C" cor_status cor_rpca_alm(const double* M, int64_t m, int64_t n, int64_t ldm,
                                   const cor_rpca_opts* opts, double* Lout, double* Sout,
                                   cor_rpca_info* info, void* stream) {
    if (!M || !Lout || !Sout || !opts) return fail(COR_E_INVAL, "null argument");
    if (m < 2 || n < 2 || ldm < n) return fail(COR_E_INVAL, "bad shape");
    const int k = opts->k, p = opts->p, q = opts->q;
    const int l = k + p;
    if (k < 1 || p < 0 || q < 0 || q > 16 || l < 2 || l >= std::min(m, n) || l > LMAX)
        return fail(COR_E_INVAL, "k, p, q as for cor_utv");
    if (opts->prec != COR_F64 && opts->prec != COR_F32)
        return fail(COR_E_INVAL, "the low-rank step runs in COR_F64 or COR_F32");
    const double lam = opts->lambda > 0.0 ? opts->lambda : 1.0 / std::sqrt((double)std::max(m, n));
    const double rho = opts->rho > 0.0 ? opts->rho : 1.5;
    const double ratio = opts->mu_bar_ratio > 0.0 ? opts->mu_bar_ratio : 1e7;
    const double tol = opts->tol > 0.0 ? opts->tol : 1e-5;
    const int max_iter = opts->max_iter > 0 ? opts->max_iter : 100;
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = opts->prec == COR_F32;
    const int64_t mn = m * n;
    const int64_t tiles = ((m + RP_TILE - 1) / RP_TILE) * ((n + RP_TILE - 1) / RP_TILE);
    const int ztiles = (int)(((m + RP_TILE - 1) / RP_TILE) * ((l + RP_TILE - 1) / RP_TILE));
    const int init_blocks = (int)std::min<int64_t>(4096, (mn + 255) / 256);
    // workspace: Y, B, U, T, V, Z, partials, scalars
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t bY = al(mn * 8), bB = al(mn * (f32 ? 4 : 8)), bU = al((size_t)m * l * 8),
                 bT = al((size_t)l * l * 8), bV = al((size_t)n * l * 8), bZ = bU,
                 bP = al((size_t)std::max<int64_t>(tiles, init_blocks) * 8), bS = 256;
    char* ws = nullptr;
    hipError_t e = hipMalloc(&ws, bY + bB + bU + bT + bV + bZ + bP + bS);
    if (e != hipSuccess) return fail(COR_E_NOMEM, "robust PCA workspace");
    double* Y = (double*)ws;
    void* B = ws + bY;
    double* U = (double*)(ws + bY + bB);
    double* T = (double*)((char*)U + bU);
    double* V = (double*)((char*)T + bT);
    double* Zm = (double*)((char*)V + bV);
    double* part = (double*)((char*)Zm + bZ);
    char* sc = (char*)part + bP;
    double* dsum = (double*)sc;
    int* dr = (int*)(sc + 16);

    cor_status st = COR_OK;
    Plan* P = nullptr;
    auto done = [&](cor_status r) {
        if (P) plan_destroy(P, nullptr);
        (void)hipStreamSynchronize(s);
        (void)hipFree(ws);
        return r;
    };
    const auto t0 = std::chrono::steady_clock::now();
    // B = M, S = Y = 0, ||M||_F
    if (f32)
        hipLaunchKernelGGL(k_rpca_init<float>, dim3(init_blocks), dim3(256), 0, s, M, ldm, m, n,
                           (float*)B, Sout, Y, part);
    else
        hipLaunchKernelGGL(k_rpca_init<double>, dim3(init_blocks), dim3(256), 0, s, M, ldm, m, n,
                           (double*)B, Sout, Y, part);
    hipLaunchKernelGGL(k_rpca_sum, dim3(1), dim3(1024), 0, s, part, init_blocks, dsum);
    double nM2 = 0.0;
    if ((e = hipGetLastError()) != hipSuccess ||
        (e = hipMemcpyAsync(&nM2, dsum, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
        return done(hip_fail(e, "robust PCA set-up"));
    // the CoR-UTV plan over the B buffer (same test matrix every iteration)
    cor_problem pr{};
    pr.A = B;
    pr.m = m;
    pr.n = n;
    pr.lda = n;
    pr.k = k;
    pr.p = p;
    pr.q = q;
    pr.prec = opts->prec;
    pr.seed = opts->seed;
    pr.U = U;
    pr.T = T;
    pr.V = V;
    st = plan_create(&pr, 1, nullptr, &P, s, false);
    if (st != COR_OK) return done(st);

    double mu = 0.0, mubar = 0.0, zeta = 1.0, mu_last = 0.0;
    int iters = 0, r = 0;
    while (true) {
        st = plan_run(P, s);
        if (st != COR_OK) return done(st);
        if (iters == 0) {  // mu_0 = 1.25 / ||M||_2, ||M||_2 taken as T_11
            double t11 = 0.0;
            if ((e = hipMemcpyAsync(&t11, T, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
                (e = hipStreamSynchronize(s)) != hipSuccess)
                return done(hip_fail(e, "robust PCA T_11"));
            if (!(t11 > 0.0)) return done(fail(COR_E_NUMERIC, "M has no nonzero singular value"));
            mu = 1.25 / t11;
            mubar = mu * ratio;
        }
        const double mu_next = std::min(rho * mu, mubar);
        hipLaunchKernelGGL(k_rpca_z, dim3(ztiles), dim3(256), 0, s, U, T, m, l, 1.0 / mu, Zm, dr);
        if (f32)
            hipLaunchKernelGGL(k_rpca_update<float>, dim3((unsigned)tiles), dim3(256), 0, s, Zm, V,
                               l, M, ldm, Lout, Sout, Y, (float*)B, m, n, mu, mu_next, lam, part);
        else
            hipLaunchKernelGGL(k_rpca_update<double>, dim3((unsigned)tiles), dim3(256), 0, s, Zm,
                               V, l, M, ldm, Lout, Sout, Y, (double*)B, m, n, mu, mu_next, lam,
                               part);
        hipLaunchKernelGGL(k_rpca_sum, dim3(1), dim3(1024), 0, s, part, (int)tiles, dsum);
        double z2 = 0.0;
        if ((e = hipGetLastError()) != hipSuccess ||
            (e = hipMemcpyAsync(&z2, dsum, 8, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipMemcpyAsync(&r, dr, 4, hipMemcpyDeviceToHost, s)) != hipSuccess ||
            (e = hipStreamSynchronize(s)) != hipSuccess)
            return done(hip_fail(e, "robust PCA iteration"));
        zeta = nM2 > 0.0 ? std::sqrt(z2 / nM2) : 0.0;
        iters++;
        mu_last = mu;
        mu = mu_next;
        if (zeta < tol || iters >= max_iter) break;
    }
    const double ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (info) {
        info->iters = iters;
        info->rank = r;
        info->zeta = zeta;
        info->mu = mu_last;
        info->ms = ms;
    }
    return done(COR_OK);
}
