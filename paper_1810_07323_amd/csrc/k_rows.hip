// Row-parallel stages of CoR-UTV around the passes over A:
//   - the Gaussian test matrix (Alg. 3, step 1) from a counter-based stream;
//   - operand copies of the skinny factors in the pass format (transposed);
//   - the fixed-order reduction of split-K partial sums into the FP64 sketch;
//   - CholeskyQR pieces of the orthonormalisation (QR of C1 and C2, Alg. 3):
//     Gram partial sums on FP64 MFMA, their fixed-order reduction, and the
//     row-wise triangular solve Q = Y R^{-1}.
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace cor {

__device__ __forceinline__ const Prob& group_prob(const Prob* probs, const int32_t* pidx,
                                                  const int32_t* toff, int cnt, int& local) {
    const int j = find_group(toff, cnt, blockIdx.x);
    local = blockIdx.x - toff[j];
    return probs[pidx[j]];
}

// ---------------------------------------------------------------------------
// Gaussian test matrix: SplitMix64 outputs (2t, 2t+1) -> Box-Muller pair t.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t idx) {
    uint64_t z = seed + (idx + 1ull) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ void gauss_pair(uint64_t seed, uint64_t t, double& z0, double& z1) {
    const double u1 = (double)((splitmix64_at(seed, 2 * t) >> 11) + 1ull) * 0x1.0p-53;
    const double u2 = (double)(splitmix64_at(seed, 2 * t + 1) >> 11) * 0x1.0p-53;
    const double r = sqrt(-2.0 * log(u1));
    const double th = 6.283185307179586 * u2;
    z0 = r * cos(th);
    z1 = r * sin(th);
}

__global__ __launch_bounds__(256) void k_omega(const Prob* __restrict__ probs,
                                               const int32_t* __restrict__ pidx,
                                               const int32_t* __restrict__ toff, int cnt) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    const int64_t total = P.n * P.l;
    const int64_t t = (int64_t)local * 256 + threadIdx.x;  // pair index
    const int64_t e = 2 * t;
    if (e >= total) return;
    if (P.omega) {
        P.Q2[e] = P.omega[e];
        if (e + 1 < total) P.Q2[e + 1] = P.omega[e + 1];
        return;
    }
    double z0, z1;
    gauss_pair(P.seed, (uint64_t)t, z0, z1);
    P.Q2[e] = z0;
    if (e + 1 < total) P.Q2[e + 1] = z1;
}

__global__ __launch_bounds__(256) void k_omega_raw(uint64_t seed, int64_t total, double* out) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t e = 2 * t;
    if (e >= total) return;
    double z0, z1;
    gauss_pair(seed, (uint64_t)t, z0, z1);
    out[e] = z0;
    if (e + 1 < total) out[e + 1] = z1;
}

hipError_t launch_omega(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_omega, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count);
    return hipGetLastError();
}

hipError_t launch_omega_raw(uint64_t seed, int64_t n, int32_t l, double* out, hipStream_t s) {
    const int64_t total = n * (int64_t)l;
    const int64_t pairs = (total + 1) / 2;
    if (pairs == 0) return hipSuccess;
    hipLaunchKernelGGL(k_omega_raw, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, s, seed,
                       total, out);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operand copy of an FP64 factor F (rows x l, row-major) in the pass format,
// stored transposed: op[c][r], c < lp, r < ld; zero outside rows x l.
// n-side (Omega / Q2): FP8 folds the column scale of A into the rows first.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T conv_op(double v, float scale_inv);
template <> __device__ __forceinline__ double conv_op<double>(double v, float) { return v; }
template <> __device__ __forceinline__ float conv_op<float>(double v, float) { return (float)v; }
template <> __device__ __forceinline__ uint16_t conv_op<uint16_t>(double v, float) { return f32_to_bf16((float)v); }
template <> __device__ __forceinline__ uint8_t conv_op<uint8_t>(double v, float sinv) { return f32_to_e4m3((float)v * sinv); }

template <typename T>
__device__ void make_op_body(const Prob& P, int side, int64_t local) {
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int64_t ld = side == SIDE_M ? P.ldq : P.ldx;
    const double* F = side == SIDE_M ? P.Q1 : P.Q2;
    T* op = reinterpret_cast<T*>(side == SIDE_M ? P.qop : P.xop);
    const float* sc = side == SIDE_M ? P.qscale : P.xscale;
    const int64_t idx = local * 256 + threadIdx.x;
    if (idx >= (int64_t)P.lp * ld) return;
    const int c = (int)(idx / ld);
    const int64_t r = idx % ld;
    T v = T(0);
    if (c < P.l && r < rows) {
        double x = F[r * P.l + c];
        float sinv = 1.0f;
        if constexpr (std::is_same<T, uint8_t>::value) {
            if (side == SIDE_N) x *= (double)P.colscale[r];
            sinv = 1.0f / sc[c];
        }
        v = conv_op<T>(x, sinv);
    }
    op[idx] = v;
}

__global__ __launch_bounds__(256) void k_make_op(const Prob* __restrict__ probs,
                                                 const int32_t* __restrict__ pidx,
                                                 const int32_t* __restrict__ toff, int cnt,
                                                 int side) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    switch (P.prec) {
        case P_F64: make_op_body<double>(P, side, local); break;
        case P_F32: make_op_body<float>(P, side, local); break;
        case P_BF16: make_op_body<uint16_t>(P, side, local); break;
        default: make_op_body<uint8_t>(P, side, local); break;
    }
}

hipError_t launch_make_op(const LaunchGroup& g, int side, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_make_op, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff,
                       g.count, side);
    return hipGetLastError();
}

// FP8 operand scales: s_c = max_r |F'[r][c]| / 448 (1 if zero), F' = F or
// diag(colscale) F on the n-side.  One block per problem.
__global__ __launch_bounds__(256) void k_op_scales(const Prob* __restrict__ probs,
                                                   const int32_t* __restrict__ pidx,
                                                   const int32_t* __restrict__ toff, int cnt,
                                                   int side, int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (P.prec != P_FP8 || iter > P.q) return;
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const double* F = side == SIDE_M ? P.Q1 : P.Q2;
    float* sc = side == SIDE_M ? P.qscale : P.xscale;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int c = wave; c < P.lp; c += 4) {
        float mx = 0.0f;
        if (c < P.l) {
            for (int64_t r = lane; r < rows; r += 64) {
                double x = F[r * P.l + c];
                if (side == SIDE_N) x *= (double)P.colscale[r];
                mx = fmaxf(mx, fabsf((float)x));
            }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, 64));
        if (lane == 0) sc[c] = mx > 0.0f ? mx / 448.0f : 1.0f;
    }
}

hipError_t launch_op_scales(const LaunchGroup& g, int side, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_op_scales, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff,
                       g.count, side, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Split-K reduction: Y[r][c] = sum_s ypart[s][r][c], s in increasing order,
// in FP64; FP8 scale folding (m-side: column scale of X; n-side: column
// scale of A on rows and of Q1 on columns).  Blocks of ROWS_PER_BLOCK rows.
// ---------------------------------------------------------------------------
template <typename Acc>
__device__ void sum_body(const Prob& P, int side, int local) {
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int S = side == SIDE_M ? P.s_ax : P.s_atx;
    const Acc* yp = reinterpret_cast<const Acc*>(P.ypart);
    const int64_t r0 = (int64_t)local * ROWS_PER_BLOCK;
    const int l = P.l, lp = P.lp;
    const bool fp8 = P.prec == P_FP8;
    for (int e = threadIdx.x; e < ROWS_PER_BLOCK * l; e += 256) {
        const int rr = e / l, c = e % l;
        const int64_t r = r0 + rr;
        if (r >= rows) break;
        double acc = 0.0;
        for (int sp = 0; sp < S; sp++) acc += (double)yp[((int64_t)sp * rows + r) * lp + c];
        if (fp8) {
            if (side == SIDE_M) acc *= (double)P.xscale[c];
            else acc *= (double)P.colscale[r] * (double)P.qscale[c];
        }
        P.Y[r * l + c] = acc;
    }
}

__global__ __launch_bounds__(256) void k_sum(const Prob* __restrict__ probs,
                                             const int32_t* __restrict__ pidx,
                                             const int32_t* __restrict__ toff, int cnt, int side,
                                             int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (iter > P.q) return;
    if (P.prec == P_F64) sum_body<double>(P, side, local);
    else sum_body<float>(P, side, local);
}

hipError_t launch_sum(const LaunchGroup& g, int side, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count,
                       side, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram partial sums G_b = Z_b^T Z_b of a row chunk Z_b of an FP64 rows x l
// matrix, on FP64 MFMA 16x16x4.  A block is (row chunk, group of upper
// 16x16 tiles); each wave holds GT_PER_WAVE tile accumulators across the
// whole chunk.  Partials: gpart[chunk][l][l], upper tiles only (entries with
// a <= b are all written).
// ---------------------------------------------------------------------------
constexpr int GT_PER_WAVE = 8;
constexpr int GT_PER_BLOCK = 4 * GT_PER_WAVE;

__device__ __forceinline__ void tile_of(int t, int nt, int& ta, int& tb) {
    // t-th upper tile (ta <= tb) in row-major order over ta.
    int a = 0, rem = t;
    while (rem >= nt - a) { rem -= nt - a; a++; }
    ta = a;
    tb = a + rem;
}

__global__ __launch_bounds__(GRAM_THREADS) void k_gram(const Prob* __restrict__ probs,
                                                      const int32_t* __restrict__ pidx,
                                                      const int32_t* __restrict__ toff, int cnt,
                                                      int side, int src, int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (iter >= 0 && iter > P.q) return;
    const int l = P.l;
    const int nt = P.lp / 16;
    const int ntu = nt * (nt + 1) / 2;
    const int ngroups = (ntu + GT_PER_BLOCK - 1) / GT_PER_BLOCK;
    const int chunk = local / ngroups;
    const int grp = local % ngroups;
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int rb = side == SIDE_M ? P.rb_m : P.rb_n;
    const int64_t r0 = (int64_t)chunk * rb;
    const int64_t r1 = min(rows, r0 + rb);
    const double* Z = src == GSRC_Y ? P.Y : src == GSRC_QA ? P.Qa : src == GSRC_U ? P.U : P.V;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    int ta[GT_PER_WAVE], tb[GT_PER_WAVE];
    bool act[GT_PER_WAVE];
    f64x4 acc[GT_PER_WAVE];
#pragma unroll
    for (int t = 0; t < GT_PER_WAVE; t++) {
        const int tt = grp * GT_PER_BLOCK + wave * GT_PER_WAVE + t;
        act[t] = tt < ntu;
        tile_of(act[t] ? tt : 0, nt, ta[t], tb[t]);
        acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
    for (int64_t kb = r0; kb < r1; kb += 4) {  // uniform trip count across the wave
        const int64_t r = kb + lg;
        const bool rv = r < r1;
        const double* zr = Z + (rv ? r : r0) * l;
#pragma unroll
        for (int t = 0; t < GT_PER_WAVE; t++) {
            if (!act[t]) continue;
            const int ca = ta[t] * 16 + li, cb = tb[t] * 16 + li;
            const double a = (rv && ca < l) ? zr[ca] : 0.0;
            const double b = (rv && cb < l) ? zr[cb] : 0.0;
            acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
        }
    }
    double* out = P.gpart + (int64_t)chunk * l * l;
#pragma unroll
    for (int t = 0; t < GT_PER_WAVE; t++) {
        if (!act[t]) continue;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int ga = ta[t] * 16 + lg + 4 * e;  // f64 MFMA output row
            const int gb = tb[t] * 16 + li;
            if (ga < l && gb < l) out[(int64_t)ga * l + gb] = acc[t][e];
        }
    }
}

hipError_t launch_gram(const LaunchGroup& g, int side, int src, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gram, dim3(g.blocks), dim3(GRAM_THREADS), 0, s, g.probs, g.pidx, g.toff,
                       g.count, side, src, iter);
    return hipGetLastError();
}

// G[a][b] = G[b][a] = sum over chunks (increasing) of gpart[chunk][min][max].
__global__ __launch_bounds__(256) void k_gram_reduce(const Prob* __restrict__ probs,
                                                     const int32_t* __restrict__ pidx,
                                                     const int32_t* __restrict__ toff, int cnt,
                                                     int side, int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (iter >= 0 && iter > P.q) return;
    const int l = P.l;
    const int e = local * 256 + threadIdx.x;
    if (e >= l * l) return;
    const int a = e / l, b = e % l;
    const int lo = min(a, b), hi = max(a, b);
    const int nb = side == SIDE_M ? P.gb_m : P.gb_n;
    double s = 0.0;
    for (int c = 0; c < nb; c++) s += P.gpart[(int64_t)c * l * l + (int64_t)lo * l + hi];
    P.G[e] = s;
    if (!isfinite(s)) atomicOr(P.flags, FLAG_NONFINITE);
}

hipError_t launch_gram_reduce(const LaunchGroup& g, int side, int nblk, int iter, hipStream_t s) {
    (void)nblk;
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gram_reduce, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff,
                       g.count, side, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row-wise forward substitution  X R = Z  (R upper, l x l, FP64):
//   X[r][c] = (Z[r][c] - sum_{a<c} X[r][a] R[a][c]) / R[c][c].
// Eight lanes share a row; lane k owns the columns a = k (mod 8) of the dot
// products, so it only ever reads back values it wrote itself.  Rows are
// staged in LDS; the result is written coalesced, optionally with the
// transposed operand copy in the pass format.
// ---------------------------------------------------------------------------
constexpr int SOLVE_ROWS = 32;
constexpr int SOLVE_PANEL = 16;  // columns of R staged in LDS at a time

template <typename T>
__device__ void write_op_rows(const Prob& P, int side, int64_t r0, int nrows, const double* xs) {
    const int l = P.l;
    T* op = reinterpret_cast<T*>(side == SIDE_M ? P.qop : P.xop);
    const int64_t ld = side == SIDE_M ? P.ldq : P.ldx;
    for (int e = threadIdx.x; e < l * SOLVE_ROWS; e += 256) {
        const int c = e / SOLVE_ROWS, rr = e % SOLVE_ROWS;
        if (rr < nrows) op[(int64_t)c * ld + r0 + rr] = conv_op<T>(xs[rr * l + c], 1.0f);
    }
}

__global__ __launch_bounds__(256) void k_solve(const Prob* __restrict__ probs,
                                               const int32_t* __restrict__ pidx,
                                               const int32_t* __restrict__ toff, int cnt,
                                               int side, int mode, int iter) {
    extern __shared__ __align__(16) double lds[];
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (iter > P.q) return;
    const int l = P.l;
    double* xs = lds;                         // SOLVE_ROWS x l
    double* rp = lds + SOLVE_ROWS * l;        // SOLVE_PANEL x l : rp[cc][a] = R[a][c0 + cc]
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int64_t r0 = (int64_t)local * SOLVE_ROWS;
    const int nrows = (int)min((int64_t)SOLVE_ROWS, rows - r0);
    const double* Z = mode == SOLVE_QA_TO_Q ? P.Qa : P.Y;
    double* D = mode == SOLVE_Y_TO_QA ? P.Qa : (side == SIDE_M ? P.Q1 : P.Q2);
    const double* __restrict__ R = P.R;

    for (int e = threadIdx.x; e < SOLVE_ROWS * l; e += 256) {
        const int rr = e / l;
        xs[e] = rr < nrows ? Z[(r0 + rr) * l + (e % l)] : 0.0;
    }

    const int rr = threadIdx.x >> 3;  // row within the block
    const int k = threadIdx.x & 7;    // lane within the row group
    double* x = xs + rr * l;
    for (int c0 = 0; c0 < l; c0 += SOLVE_PANEL) {
        const int pc = min(SOLVE_PANEL, l - c0);
        __syncthreads();  // previous panel fully used (and xs loaded)
        for (int e = threadIdx.x; e < SOLVE_PANEL * l; e += 256) {
            const int cc = e / l, a = e % l;
            rp[e] = (cc < pc && a <= c0 + cc) ? R[(int64_t)a * l + c0 + cc] : 0.0;
        }
        __syncthreads();
        for (int cc = 0; cc < pc; cc++) {
            const int c = c0 + cc;
            const double* rc = rp + cc * l;
            double part = 0.0;
            for (int a = k; a < c; a += 8) part += x[a] * rc[a];
            part += __shfl_xor(part, 1, 64);
            part += __shfl_xor(part, 2, 64);
            part += __shfl_xor(part, 4, 64);
            const double zc = x[c];
            __builtin_amdgcn_wave_barrier();
            const double xc = (zc - part) / rc[c];
            if ((c & 7) == k) x[c] = xc;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SOLVE_ROWS * l; e += 256) {
        const int r = e / l;
        if (r < nrows) D[(r0 + r) * l + (e % l)] = xs[e];
    }
    if (mode != SOLVE_Y_TO_QA && P.prec != P_FP8) {
        switch (P.prec) {
            case P_F64: write_op_rows<double>(P, side, r0, nrows, xs); break;
            case P_F32: write_op_rows<float>(P, side, r0, nrows, xs); break;
            default: write_op_rows<uint16_t>(P, side, r0, nrows, xs); break;
        }
    }
}

hipError_t launch_solve(const LaunchGroup& g, int side, int mode, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * (SOLVE_ROWS + SOLVE_PANEL) * LMAX;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_solve,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_solve, dim3(g.blocks), dim3(256), lds, s, g.probs, g.pidx, g.toff,
                       g.count, side, mode, iter);
    return hipGetLastError();
}

}  // namespace cor
