// l x l stages of CoR-UTV and the assembly of the factors.
//   - Cholesky of the Gram matrix (CholeskyQR of C1, C2 in Alg. 3) and the
//     accumulated R factor of the orthonormalisation;
//   - the column-pivoted QR of the compressed matrix M = Q1^T A Q2 = R2^T,
//     eq. (eq_Drrqr): Businger-Golub pivoting on exactly recomputed trailing
//     column norms (lowest index on ties), Householder reflections, T_jj >= 0;
//   - U = Q1 Qt and V = Q2 P of eq. (eq_T_basic);
//   - the accuracy report and the stand-alone format conversion.
#include "common.h"
#include "kernels.h"

namespace cor {

constexpr int SMALL_THREADS = 1024;
constexpr int CHOL_LDS_MAX = 140;  // l*l doubles + scratch fit in 160 KB of LDS
constexpr int QRCP_LDS_MAX = 136;

__device__ __forceinline__ const Prob& group_prob2(const Prob* probs, const int32_t* pidx,
                                                   const int32_t* toff, int cnt, int& local) {
    const int j = find_group(toff, cnt, blockIdx.x);
    local = blockIdx.x - toff[j];
    return probs[pidx[j]];
}

// ---------------------------------------------------------------------------
// Cholesky G = R^T R, right-looking with one barrier per column; row j is
// scaled by 1/sqrt(d_j) one step later so no thread reads a row while it is
// rescaled.  A pivot d_j <= l 2^-52 max_i G_ii is clamped to that threshold
// (numerically rank-deficient sketch) and flagged.  mode FIRST: Racc = R;
// SECOND: Racc = R Racc (the R factor of the two CholeskyQR passes).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SMALL_THREADS) void k_chol(const Prob* __restrict__ probs,
                                                        const int32_t* __restrict__ pidx,
                                                        const int32_t* __restrict__ toff, int cnt,
                                                        int mode, int iter) {
    extern __shared__ __align__(16) double sm[];
    __shared__ double s_tol;
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    if (iter >= 0 && iter > P.q) return;
    const int l = P.l;
    const int tid = threadIdx.x;
    const bool in_lds = l <= CHOL_LDS_MAX;
    double* W = in_lds ? sm : P.R;

    for (int e = tid; e < l * l; e += SMALL_THREADS) W[e] = P.G[e];
    if (tid < 64) {
        double mx = 0.0;
        for (int i = tid; i < l; i += 64) mx = fmax(mx, fabs(P.G[i * l + i]));
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        if (tid == 0) s_tol = (double)l * 0x1.0p-52 * mx;
    }
    __syncthreads();
    const double tol = s_tol > 0.0 ? s_tol : 0x1.0p-1000;

    double dprev = 1.0;
    bool clamped = false;
    for (int j = 0; j < l; j++) {
        double d = W[j * l + j];
        if (!(d > tol)) {
            clamped = true;
            d = tol;
        }
        const double inv_d = 1.0 / d;
        if (j > 0) {
            const double sc = 1.0 / sqrt(dprev);
            for (int c = j - 1 + tid; c < l; c += SMALL_THREADS)
                W[(j - 1) * l + c] = (c == j - 1) ? sqrt(dprev) : W[(j - 1) * l + c] * sc;
        }
        const int n1 = l - j - 1;
        const double* wj = W + j * l;
        for (int idx = tid; idx < n1 * n1; idx += SMALL_THREADS) {
            const int a = j + 1 + idx / n1, b = j + 1 + idx % n1;
            if (b >= a) W[a * l + b] -= wj[a] * wj[b] * inv_d;
        }
        dprev = d;
        __syncthreads();
    }
    if (tid == 0) W[(l - 1) * l + (l - 1)] = sqrt(dprev);
    if (clamped && tid == 0) atomicOr(P.flags, FLAG_RANK_DEF);
    __syncthreads();
    for (int e = tid; e < l * l; e += SMALL_THREADS) {
        const int a = e / l, b = e % l;
        if (b < a) W[e] = 0.0;
    }
    __syncthreads();
    if (in_lds)
        for (int e = tid; e < l * l; e += SMALL_THREADS) P.R[e] = W[e];
    if (mode == CHOL_FIRST) {
        for (int e = tid; e < l * l; e += SMALL_THREADS) P.Racc[e] = W[e];
        return;
    }
    // Racc <- R Racc (both upper triangular), through G as scratch.
    for (int e = tid; e < l * l; e += SMALL_THREADS) {
        const int a = e / l, b = e % l;
        double s = 0.0;
        if (b >= a)
            for (int t = a; t <= b; t++) s += W[a * l + t] * P.Racc[t * l + b];
        P.G[e] = s;
    }
    __syncthreads();
    for (int e = tid; e < l * l; e += SMALL_THREADS) P.Racc[e] = P.G[e];
}

hipError_t launch_chol(const LaunchGroup& g, int mode, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * CHOL_LDS_MAX * CHOL_LDS_MAX;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_chol,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_chol, dim3(g.blocks), dim3(SMALL_THREADS), lds, s, g.probs, g.pidx,
                       g.toff, g.count, mode, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// QRCP of M = Racc^T (l x l).  Wave 0 picks the pivot, swaps and builds the
// reflector; then every wave updates its trailing columns (one column per
// wave at a time, rows over lanes) and recomputes their norms over the rows
// below the diagonal for the next pivot choice.  The reflectors are then
// accumulated backwards in place into Qt = H_0 H_1 ... H_{l-1}.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(SMALL_THREADS) void k_qrcp(const Prob* __restrict__ probs,
                                                        const int32_t* __restrict__ pidx,
                                                        const int32_t* __restrict__ toff,
                                                        int cnt) {
    extern __shared__ __align__(16) double sm[];
    __shared__ double s_v[LMAX];
    __shared__ double s_nrm[LMAX];
    __shared__ double s_tau[LMAX];
    __shared__ double s_sign[LMAX];
    __shared__ int s_perm[LMAX];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    const int l = P.l;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = SMALL_THREADS / 64;
    const bool in_lds = l <= QRCP_LDS_MAX;
    double* W = in_lds ? sm : P.Qt;

    for (int e = tid; e < l * l; e += SMALL_THREADS) {
        const int a = e / l, b = e % l;
        W[e] = P.Racc[b * l + a];  // M = R2^T
    }
    for (int c = tid; c < l; c += SMALL_THREADS) s_perm[c] = c;
    __syncthreads();
    for (int c = wave; c < l; c += NW) {
        double ss = 0.0;
        for (int i = lane; i < l; i += 64) ss += W[i * l + c] * W[i * l + c];
        ss = wave_sum(ss);
        if (lane == 0) s_nrm[c] = ss;
    }
    __syncthreads();

    for (int j = 0; j < l; j++) {
        if (wave == 0) {
            // pivot: largest squared norm, lowest index on ties
            double bv = -1.0;
            int bi = l;
            for (int c = j + lane; c < l; c += 64) {
                const double v = s_nrm[c];
                if (v > bv) { bv = v; bi = c; }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(bv, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            const int p = bi;
            if (p != j) {
                for (int i = lane; i < l; i += 64) {
                    const double t = W[i * l + j];
                    W[i * l + j] = W[i * l + p];
                    W[i * l + p] = t;
                }
                if (lane == 0) {
                    const int t = s_perm[j]; s_perm[j] = s_perm[p]; s_perm[p] = t;
                    const double tn = s_nrm[j]; s_nrm[j] = s_nrm[p]; s_nrm[p] = tn;
                }
            }
            // Householder reflector of column j, rows j..l-1
            double ss = 0.0;
            for (int i = j + lane; i < l; i += 64) ss += W[i * l + j] * W[i * l + j];
            ss = wave_sum(ss);
            const double alpha = W[j * l + j];
            const double xnorm = sqrt(ss);
            double tau = 0.0, beta = alpha, scale = 0.0;
            if (xnorm != 0.0) {
                beta = alpha >= 0.0 ? -xnorm : xnorm;
                scale = 1.0 / (alpha - beta);
                tau = (beta - alpha) / beta;
            }
            for (int i = j + lane; i < l; i += 64) {
                double v;
                if (i == j) v = 1.0;
                else {
                    v = W[i * l + j] * scale;
                    if (xnorm != 0.0) W[i * l + j] = v;
                }
                s_v[i] = v;
            }
            if (lane == 0) {
                s_tau[j] = tau;
                W[j * l + j] = beta;
            }
        }
        __syncthreads();
        const double tau = s_tau[j];
        for (int c = j + 1 + wave; c < l; c += NW) {
            double dot = 0.0;
            if (tau != 0.0) {
                for (int i = j + lane; i < l; i += 64) dot += s_v[i] * W[i * l + c];
                dot = wave_sum(dot) * tau;
                for (int i = j + lane; i < l; i += 64) W[i * l + c] -= dot * s_v[i];
            }
            double ss = 0.0;
            for (int i = j + 1 + lane; i < l; i += 64) ss += W[i * l + c] * W[i * l + c];
            ss = wave_sum(ss);
            if (lane == 0) s_nrm[c] = ss;
        }
        __syncthreads();
    }

    // T (upper, T_jj >= 0) and the permutation.
    for (int j = tid; j < l; j += SMALL_THREADS) s_sign[j] = W[j * l + j] < 0.0 ? -1.0 : 1.0;
    __syncthreads();
    for (int e = tid; e < l * l; e += SMALL_THREADS) {
        const int a = e / l, b = e % l;
        P.T[e] = b >= a ? s_sign[a] * W[e] : 0.0;
    }
    for (int j = tid; j < l; j += SMALL_THREADS) P.perm[j] = s_perm[j];
    __syncthreads();

    // Qt = H_0 (H_1 (... H_{l-1} I)), in place.
    for (int j = l - 1; j >= 0; j--) {
        if (wave == 0) {
            for (int i = j + lane; i < l; i += 64) {
                s_v[i] = (i == j) ? 1.0 : W[i * l + j];
                W[i * l + j] = (i == j) ? 1.0 : 0.0;
                if (i > j) W[j * l + i] = 0.0;
            }
        }
        __syncthreads();
        const double tau = s_tau[j];
        if (tau != 0.0) {
            for (int c = j + wave; c < l; c += NW) {
                double dot = 0.0;
                for (int i = j + lane; i < l; i += 64) dot += s_v[i] * W[i * l + c];
                dot = wave_sum(dot) * tau;
                for (int i = j + lane; i < l; i += 64) W[i * l + c] -= dot * s_v[i];
            }
        }
        __syncthreads();
    }
    for (int e = tid; e < l * l; e += SMALL_THREADS) P.Qt[e] = W[e] * s_sign[e % l];
}

hipError_t launch_qrcp(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * QRCP_LDS_MAX * QRCP_LDS_MAX;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_qrcp,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_qrcp, dim3(g.blocks), dim3(SMALL_THREADS), lds, s, g.probs, g.pidx,
                       g.toff, g.count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// U = Q1 Qt (blocks of 32 rows of U) and V = Q2 P (blocks of 64 rows of V).
// Per problem: ceil(m/32) U-blocks followed by ceil(n/64) V-blocks.
// ---------------------------------------------------------------------------
constexpr int UV_ROWS = 32;
constexpr int V_ROWS = 64;

__global__ __launch_bounds__(256) void k_form_uv(const Prob* __restrict__ probs,
                                                 const int32_t* __restrict__ pidx,
                                                 const int32_t* __restrict__ toff, int cnt) {
    extern __shared__ __align__(16) double xs[];  // UV_ROWS x l
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    const int l = P.l;
    const int ub = (int)((P.m + UV_ROWS - 1) / UV_ROWS);
    const int tid = threadIdx.x;
    if (local >= ub) {
        const int64_t r0 = (int64_t)(local - ub) * V_ROWS;
        for (int e = tid; e < V_ROWS * l; e += 256) {
            const int64_t r = r0 + e / l;
            const int c = e % l;
            if (r < P.n) P.V[r * l + c] = P.Q2[r * l + P.perm[c]];
        }
        return;
    }
    const int64_t r0 = (int64_t)local * UV_ROWS;
    const int nrows = (int)min((int64_t)UV_ROWS, P.m - r0);
    for (int e = tid; e < UV_ROWS * l; e += 256) {
        const int rr = e / l;
        xs[e] = rr < nrows ? P.Q1[(r0 + rr) * l + e % l] : 0.0;
    }
    __syncthreads();
    const int cg = tid & 63;
    const int rg = tid >> 6;  // 8 rows per group
    constexpr int NJ = (LMAX + 63) / 64;
    double acc[8][NJ];
#pragma unroll
    for (int r = 0; r < 8; r++)
#pragma unroll
        for (int jj = 0; jj < NJ; jj++) acc[r][jj] = 0.0;
    for (int a = 0; a < l; a++) {
        double qt[NJ];
#pragma unroll
        for (int jj = 0; jj < NJ; jj++) {
            const int c = cg + 64 * jj;
            qt[jj] = c < l ? P.Qt[a * l + c] : 0.0;
        }
#pragma unroll
        for (int r = 0; r < 8; r++) {
            const double q = xs[(rg * 8 + r) * l + a];
#pragma unroll
            for (int jj = 0; jj < NJ; jj++) acc[r][jj] += q * qt[jj];
        }
    }
#pragma unroll
    for (int r = 0; r < 8; r++) {
        const int rr = rg * 8 + r;
        if (rr >= nrows) continue;
#pragma unroll
        for (int jj = 0; jj < NJ; jj++) {
            const int c = cg + 64 * jj;
            if (c < l) P.U[(r0 + rr) * l + c] = acc[r][jj];
        }
    }
}

hipError_t launch_form_uv(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * UV_ROWS * LMAX;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_form_uv,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_form_uv, dim3(g.blocks), dim3(256), lds, s, g.probs, g.pidx, g.toff,
                       g.count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Report.  ||A||_F^2 in 64 fixed partial sums (rep[32 + b]); then
// phase 1/2: ||G - I||_F of the Gram of U / V; phase 3: err_l, err_k from
// ||A - U T V^T||_F^2 = ||A||_F^2 - ||T||_F^2 (T = U^T A V) and the rank-k
// analogue with T[:k, :].
// ---------------------------------------------------------------------------
constexpr int NORM_BLOCKS = 64;

__device__ __forceinline__ double block_sum256(double v, double* red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) s += red[w];
    return s;
}

__global__ __launch_bounds__(256) void k_normA(const Prob* __restrict__ probs,
                                               const int32_t* __restrict__ pidx,
                                               const int32_t* __restrict__ toff, int cnt) {
    __shared__ double red[4];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    double s = 0.0;
    for (int64_t r = local; r < P.m; r += NORM_BLOCKS) {
        for (int64_t c = threadIdx.x; c < P.n; c += 256) {
            const int64_t o = r * P.lda + c;
            double v;
            switch (P.prec) {
                case P_F64: v = reinterpret_cast<const double*>(P.A)[o]; break;
                case P_F32: v = reinterpret_cast<const float*>(P.A)[o]; break;
                case P_BF16: v = __uint_as_float((uint32_t)reinterpret_cast<const uint16_t*>(P.A)[o] << 16); break;
                default: {
                    const uint8_t code = reinterpret_cast<const uint8_t*>(P.A)[o];
                    const int e = (code >> 3) & 15, mt = code & 7;
                    double x = e == 0 ? ldexp((double)mt / 8.0, -6) : ldexp(1.0 + mt / 8.0, e - 7);
                    v = ((code & 0x80) ? -x : x) * (double)P.colscale[c];
                }
            }
            s += v * v;
        }
    }
    s = block_sum256(s, red);
    if (threadIdx.x == 0) P.rep[32 + local] = s;
}

hipError_t launch_normA(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normA, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_report(const Prob* __restrict__ probs,
                                                const int32_t* __restrict__ pidx,
                                                const int32_t* __restrict__ toff, int cnt,
                                                int phase) {
    __shared__ double red[4];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    const int l = P.l;
    if (phase == 1 || phase == 2) {
        double s = 0.0;
        for (int e = threadIdx.x; e < l * l; e += 256) {
            const double d = P.G[e] - ((e / l) == (e % l) ? 1.0 : 0.0);
            s += d * d;
        }
        s = block_sum256(s, red);
        if (threadIdx.x == 0) P.rep[phase + 1] = sqrt(s);
        return;
    }
    double t2 = 0.0, tk2 = 0.0;
    for (int e = threadIdx.x; e < l * l; e += 256) {
        const double v = P.T[e];
        t2 += v * v;
        if (e / l < P.k) tk2 += v * v;
    }
    t2 = block_sum256(t2, red);
    tk2 = block_sum256(tk2, red);
    if (threadIdx.x == 0) {
        double na = 0.0;
        for (int b = 0; b < NORM_BLOCKS; b++) na += P.rep[32 + b];
        P.rep[4] = na;
        P.rep[0] = na > 0.0 ? sqrt(fmax(0.0, 1.0 - t2 / na)) : 0.0;
        P.rep[1] = na > 0.0 ? sqrt(fmax(0.0, 1.0 - tk2 / na)) : 0.0;
    }
}

hipError_t launch_report(const LaunchGroup& g, int phase, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_report, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count,
                       phase);
    return hipGetLastError();
}

__global__ void k_clear_flags(const Prob* __restrict__ probs, const int32_t* __restrict__ pidx,
                              const int32_t* __restrict__ toff, int cnt) {
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    if (threadIdx.x == 0) *P.flags = 0;
}

hipError_t launch_clear_flags(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_clear_flags, dim3(g.blocks), dim3(64), 0, s, g.probs, g.pidx, g.toff,
                       g.count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Format conversion of a stored FP32 matrix (cor_quantize).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_to_bf16(const float* __restrict__ a, int64_t m, int64_t n,
                                                 int64_t lda, uint16_t* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= m * n) return;
    const int64_t r = idx / n, c = idx % n;
    out[idx] = f32_to_bf16(a[r * lda + c]);
}

__global__ __launch_bounds__(256) void k_colscale(const float* __restrict__ a, int64_t m, int64_t n,
                                                  int64_t lda, float* __restrict__ s) {
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    float mx = 0.0f;
    for (int64_t r = 0; r < m; r++) mx = fmaxf(mx, fabsf(a[r * lda + c]));
    s[c] = mx > 0.0f ? mx / 448.0f : 1.0f;
}

__global__ __launch_bounds__(256) void k_to_fp8(const float* __restrict__ a, int64_t m, int64_t n,
                                                int64_t lda, const float* __restrict__ s,
                                                uint8_t* __restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= m * n) return;
    const int64_t r = idx / n, c = idx % n;
    out[idx] = f32_to_e4m3(a[r * lda + c] / s[c]);
}

hipError_t launch_quantize(const float* a32, int64_t m, int64_t n, int64_t lda, int to, void* out,
                           float* colscale, hipStream_t s) {
    const int64_t total = m * n;
    if (total == 0) return hipSuccess;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    if (to == P_BF16) {
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks), dim3(256), 0, s, a32, m, n, lda,
                           reinterpret_cast<uint16_t*>(out));
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_colscale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a32, m, n,
                       lda, colscale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_fp8, dim3(blocks), dim3(256), 0, s, a32, m, n, lda, colscale,
                       reinterpret_cast<uint8_t*>(out));
    return hipGetLastError();
}

}  // namespace cor
