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

// T'' = rows < r of T with the diagonal shrunk by delta, r = #{T_ii > delta};
// one block (r is written to *rout).
__global__ __launch_bounds__(256) void k_rpca_tshrink(const double* __restrict__ T, int l,
                                                      double delta, double* __restrict__ T2,
                                                      int* __restrict__ rout) {
    __shared__ int s_r;
    if (threadIdx.x == 0) {
        int r = 0;
        for (int i = 0; i < l; i++) r += T[i * l + i] > delta ? 1 : 0;
        s_r = r;
        *rout = r;
    }
    __syncthreads();
    const int r = s_r;
    for (int e = threadIdx.x; e < l * l; e += 256) {
        const int a = e / l, b = e - (e / l) * l;
        T2[e] = a < r ? T[e] - (a == b ? delta : 0.0) : 0.0;
    }
}

// Z = U T'' (m x l): a thread per entry, the rows of T'' read through the cache.
__global__ __launch_bounds__(256) void k_rpca_z(const double* __restrict__ U,
                                                const double* __restrict__ T2, int64_t m, int l,
                                                double* __restrict__ Z) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= m * l) return;
    const int64_t i = e / l;
    const int c = (int)(e - i * l);
    const double* u = U + i * l;
    double s0 = 0.0, s1 = 0.0;
    int t = 0;
    for (; t + 1 < l; t += 2) {
        s0 = fma(u[t], T2[t * l + c], s0);
        s1 = fma(u[t + 1], T2[(t + 1) * l + c], s1);
    }
    if (t < l) s0 = fma(u[t], T2[t * l + c], s0);
    Z[e] = s0 + s1;
}

// The L product and the ALM updates, one 64 x 64 tile of (i, j) per block:
// four waves, each 2 x 2 FP64 MFMA tiles (16x16x4) over K = l, operands
// streamed from Z (m x l) and V (n x l) rows.  Epilogue per entry:
//   L = (Z V^T)_ij, W = M - L + Y / mu, S = shrink(W, lam / mu),
//   R = M - L - S, Y += mu R, B = M - S + Y / mu_next (in B's format),
// and the block's sum of R^2 (for zeta) in a fixed order.
constexpr int RP_TILE = 64;

template <typename TB>
__global__ __launch_bounds__(256) void k_rpca_update(
    const double* __restrict__ Z, const double* __restrict__ V, int l, const double* __restrict__ M,
    int64_t ldm, double* __restrict__ L, double* __restrict__ S, double* __restrict__ Y,
    TB* __restrict__ B, int64_t m, int64_t n, double mu, double mu_next, double lam,
    double* __restrict__ zpart) {
    __shared__ double red[4];
    const int64_t tcs = (n + RP_TILE - 1) / RP_TILE;
    const int64_t i0 = (int64_t)(blockIdx.x / tcs) * RP_TILE;
    const int64_t j0 = (int64_t)(blockIdx.x % tcs) * RP_TILE;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t wi = i0 + 32 * (wave >> 1), wj = j0 + 32 * (wave & 1);
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // operand rows of this lane (clamped: rows past m or n only feed entries
    // that are never written)
    const double* za[2];
    const double* vb[2];
#pragma unroll
    for (int a = 0; a < 2; a++) {
        za[a] = Z + std::min<int64_t>(wi + 16 * a + li, m - 1) * l;
        vb[a] = V + std::min<int64_t>(wj + 16 * a + li, n - 1) * l;
    }
    for (int k0 = 0; k0 < l; k0 += 4) {
        const int k = k0 + lg;
        const bool ok = k < l;
        double x[2], y[2];
#pragma unroll
        for (int a = 0; a < 2; a++) {
            x[a] = ok ? za[a][k] : 0.0;
            y[a] = ok ? vb[a][k] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
                acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], y[b], acc[a][b], 0, 0, 0);
    }
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

// Sum of `count` partials in index order (one thread).
__global__ void k_rpca_sum(const double* __restrict__ part, int count, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < count; i++) s += part[i];
    *out = s;
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
    const int init_blocks = (int)std::min<int64_t>(4096, (mn + 255) / 256);
    // workspace: Y, B, U, T, V, T'', Z, partials, scalars
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t bY = al(mn * 8), bB = al(mn * (f32 ? 4 : 8)), bU = al((size_t)m * l * 8),
                 bT = al((size_t)l * l * 8), bV = al((size_t)n * l * 8), bZ = bU,
                 bP = al((size_t)std::max<int64_t>(tiles, init_blocks) * 8), bS = 256;
    char* ws = nullptr;
    hipError_t e = hipMalloc(&ws, bY + bB + bU + 2 * bT + bV + bZ + bP + bS);
    if (e != hipSuccess) return fail(COR_E_NOMEM, "robust PCA workspace");
    double* Y = (double*)ws;
    void* B = ws + bY;
    double* U = (double*)(ws + bY + bB);
    double* T = (double*)((char*)U + bU);
    double* T2 = (double*)((char*)T + bT);
    double* V = (double*)((char*)T2 + bT);
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
    hipLaunchKernelGGL(k_rpca_sum, dim3(1), dim3(64), 0, s, part, init_blocks, dsum);
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
        hipLaunchKernelGGL(k_rpca_tshrink, dim3(1), dim3(256), 0, s, T, l, 1.0 / mu, T2, dr);
        hipLaunchKernelGGL(k_rpca_z, dim3((unsigned)((m * l + 255) / 256)), dim3(256), 0, s, U, T2,
                           m, l, Zm);
        if (f32)
            hipLaunchKernelGGL(k_rpca_update<float>, dim3((unsigned)tiles), dim3(256), 0, s, Zm, V,
                               l, M, ldm, Lout, Sout, Y, (float*)B, m, n, mu, mu_next, lam, part);
        else
            hipLaunchKernelGGL(k_rpca_update<double>, dim3((unsigned)tiles), dim3(256), 0, s, Zm,
                               V, l, M, ldm, Lout, Sout, Y, (double*)B, m, n, mu, mu_next, lam,
                               part);
        hipLaunchKernelGGL(k_rpca_sum, dim3(1), dim3(64), 0, s, part, (int)tiles, dsum);
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
