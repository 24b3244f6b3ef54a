// Row-parallel stages of CoR-UTV around the passes over A:
//   - the Gaussian test matrix (Alg. 3, step 1) from a counter-based stream;
//   - operand copies of the skinny factors in the pass format (transposed);
//   - the fixed-order reduction of split-K partial sums into the FP64 sketch;
//   - CholeskyQR pieces of the orthonormalisation (QR of C1 and C2, Alg. 3):
//     Gram partial sums on FP64 MFMA, their fixed-order reduction, and the
//     products Q = Y R^{-1}; the assembly U = Q1 Qt and V = Q2 P.
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
    // the first stage of a decomposition: its flag word starts cleared
    if (local == 0 && threadIdx.x == 0) *P.flags = 0;
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

// Zero fill of a device byte range (16-byte words; `bytes` a multiple of 16,
// `p` 16-byte aligned): the workspace clear of plans in caller-provided memory.
__global__ __launch_bounds__(256) void k_zero16(uint4* __restrict__ p, int64_t words) {
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < words; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t words = (int64_t)(bytes / 16);
    if (words <= 0) return hipSuccess;
    const int64_t want = (words + 255) / 256;
    const unsigned blocks = (unsigned)(want < 2048 ? want : 2048);
    hipLaunchKernelGGL(k_zero16, dim3(blocks), dim3(256), 0, s, reinterpret_cast<uint4*>(p), words);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Operand copy of an FP64 factor F (rows x l, row-major) in the pass format,
// stored transposed: op[c][r], c < lp, r < ld; zero outside rows x l.
// n-side (Omega / Q2): FP8 folds the column scale of A into the rows first.
// A block transposes one tile through LDS, so that both the reads of F and
// the writes of op are contiguous runs.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T conv_op(double v, float scale_inv);
template <> __device__ __forceinline__ double conv_op<double>(double v, float) { return v; }
template <> __device__ __forceinline__ float conv_op<float>(double v, float) { return (float)v; }
template <> __device__ __forceinline__ uint16_t conv_op<uint16_t>(double v, float) { return f32_to_bf16((float)v); }
template <> __device__ __forceinline__ uint8_t conv_op<uint8_t>(double v, float sinv) { return f32_to_e4m3((float)v * sinv); }

template <typename T>
__device__ void make_op_body(const Prob& P, int side, int64_t local, double (*tile)[MO_ROWS + 1]) {
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int64_t ld = side == SIDE_M ? P.ldq : P.ldx;
    const double* F = side == SIDE_M ? P.Q1 : P.Q2;
    T* op = reinterpret_cast<T*>(side == SIDE_M ? P.qop : P.xop);
    const float* sc = side == SIDE_M ? P.qscale : P.xscale;
    const int l = P.l;
    const int64_t nrt = (ld + MO_ROWS - 1) / MO_ROWS;
    const int64_t r0 = (local % nrt) * MO_ROWS;
    const int c0 = (int)(local / nrt) * MO_COLS;
    const int tid = threadIdx.x;
    // read MO_ROWS rows x MO_COLS columns of F, each row segment contiguous
#pragma unroll
    for (int p = 0; p < MO_ROWS * MO_COLS / 256; p++) {
        const int rr = p * (256 / MO_COLS) + tid / MO_COLS, cc = tid % MO_COLS;
        const int64_t r = r0 + rr;
        const int c = c0 + cc;
        tile[cc][rr] = (r < rows && c < l) ? F[r * l + c] : 0.0;
    }
    __syncthreads();
    // write them transposed: op[c][r], each column segment contiguous
#pragma unroll
    for (int p = 0; p < MO_ROWS * MO_COLS / 256; p++) {
        const int cc = p * (256 / MO_ROWS) + tid / MO_ROWS, rr = tid % MO_ROWS;
        const int64_t r = r0 + rr;
        const int c = c0 + cc;
        if (r >= ld) continue;
        T v = T(0);
        if (c < l && r < rows) {
            double x = tile[cc][rr];
            float sinv = 1.0f;
            if constexpr (std::is_same<T, uint8_t>::value) {
                if (side == SIDE_N) x *= (double)P.colscale[r];
                sinv = 1.0f / sc[c];
            }
            v = conv_op<T>(x, sinv);
        }
        op[(int64_t)c * ld + r] = v;
    }
}

__global__ __launch_bounds__(256) void k_make_op(const Prob* __restrict__ probs,
                                                 const int32_t* __restrict__ pidx,
                                                 const int32_t* __restrict__ toff, int cnt,
                                                 int side) {
    __shared__ double tile[MO_COLS][MO_ROWS + 1];
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    switch (P.prec) {
        case P_F64: make_op_body<double>(P, side, local, tile); break;
        case P_F32: make_op_body<float>(P, side, local, tile); break;
        case P_BF16: make_op_body<uint16_t>(P, side, local, tile); break;
        default: make_op_body<uint8_t>(P, side, local, tile); break;
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
// FP8 operand scales of an FP64 factor F (rows x l; n-side rows scaled by the
// column scales of A first): s_c = max_r |F_rc| / 448 (1 for a zero column).
// Stage 1: a block per row chunk writes the chunk's column maxima, one thread
// per column (the rows are read as contiguous runs); stage 2: a block per
// problem takes the maximum over the chunks.  Maxima are exact, so the result
// does not depend on the chunking.
__global__ __launch_bounds__(256) void k_op_colmax(const Prob* __restrict__ probs,
                                                   const int32_t* __restrict__ pidx,
                                                   const int32_t* __restrict__ toff, int cnt,
                                                   int side, int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (P.prec != P_FP8 || iter > P.q) return;
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int nch = side == SIDE_M ? P.sch_m : P.sch_n;
    const double* F = side == SIDE_M ? P.Q1 : P.Q2;
    const int64_t per = (rows + nch - 1) / nch;
    const int64_t r0 = (int64_t)local * per;
    const int64_t r1 = r0 + per < rows ? r0 + per : rows;
    for (int c = threadIdx.x; c < P.lp; c += 256) {
        float mx = 0.0f;
        if (c < P.l) {
            for (int64_t r = r0; r < r1; r++) {
                double x = F[r * P.l + c];
                if (side == SIDE_N) x *= (double)P.colscale[r];
                mx = fmaxf(mx, fabsf((float)x));
            }
        }
        P.scpart[(int64_t)local * P.lp + c] = mx;
    }
}

__global__ __launch_bounds__(256) void k_op_scales(const Prob* __restrict__ probs,
                                                   const int32_t* __restrict__ pidx,
                                                   const int32_t* __restrict__ toff, int cnt,
                                                   int side, int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (P.prec != P_FP8 || iter > P.q) return;
    const int nch = side == SIDE_M ? P.sch_m : P.sch_n;
    float* sc = side == SIDE_M ? P.qscale : P.xscale;
    for (int c = threadIdx.x; c < P.lp; c += 256) {
        float mx = 0.0f;
        for (int ch = 0; ch < nch; ch++) mx = fmaxf(mx, P.scpart[(int64_t)ch * P.lp + c]);
        sc[c] = mx > 0.0f ? mx / 448.0f : 1.0f;
    }
}

hipError_t launch_op_scales(const LaunchGroup& chunks, const LaunchGroup& one, int side, int iter,
                            hipStream_t s) {
    if (chunks.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_op_colmax, dim3(chunks.blocks), dim3(256), 0, s, chunks.probs,
                       chunks.pidx, chunks.toff, chunks.count, side, iter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_op_scales, dim3(one.blocks), dim3(256), 0, s, one.probs, one.pidx,
                       one.toff, one.count, side, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Split-K reduction: Y[r][c] = sum_s ypart[s][r][c], s in increasing order,
// in FP64; FP8 scale folding (m-side: column scale of X; n-side: column
// scale of A on rows and of Q1 on columns).  One thread per 4 columns of a
// row (16-byte loads of the FP32 partials).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sum(const Prob* __restrict__ probs,
                                             const int32_t* __restrict__ pidx,
                                             const int32_t* __restrict__ toff, int cnt, int side,
                                             int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (iter > P.q) return;
    if (iter < 0 && P.mmode != M_EXPLICIT) return;  // the pass A Q2 of eq. (14)
    if (side == SIDE_F && (!P.fused || iter >= P.q)) return;
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int S = side == SIDE_M ? P.s_ax : side == SIDE_N ? P.s_atx : P.s_f;
    const int l = P.l, lp = P.lp, nq = lp / 4;
    const int64_t idx = (int64_t)local * 256 + threadIdx.x;
    const int64_t r = idx / nq;
    const int c0 = (int)(idx % nq) * 4;
    if (r >= rows || c0 >= l) return;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    if (P.prec == P_F64) {
        const double* yp = reinterpret_cast<const double*>(P.ypart);
#pragma unroll 4
        for (int sp = 0; sp < S; sp++) {
            const double* p = yp + ((int64_t)sp * rows + r) * lp + c0;
            const double2 u = *reinterpret_cast<const double2*>(p);
            const double2 v = *reinterpret_cast<const double2*>(p + 2);
            acc[0] += u.x; acc[1] += u.y; acc[2] += v.x; acc[3] += v.y;
        }
    } else {
        const float* yp = reinterpret_cast<const float*>(P.ypart);
#pragma unroll 8
        for (int sp = 0; sp < S; sp++) {
            const float4 u = *reinterpret_cast<const float4*>(yp + ((int64_t)sp * rows + r) * lp + c0);
            acc[0] += (double)u.x; acc[1] += (double)u.y; acc[2] += (double)u.z; acc[3] += (double)u.w;
        }
    }
    if (P.prec == P_FP8) {
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int c = min(c0 + e, l - 1);
            acc[e] *= side == SIDE_M ? (double)P.xscale[c]
                                     : (double)P.colscale[r] * (double)P.qscale[c];
        }
    }
    double* y = P.Y + r * l + c0;
    if ((l & 1) == 0 && c0 + 4 <= l) {
        // even l: the four entries are two aligned 16-byte stores
        reinterpret_cast<double2*>(y)[0] = make_double2(acc[0], acc[1]);
        reinterpret_cast<double2*>(y)[1] = make_double2(acc[2], acc[3]);
        return;
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
        if (c0 + e >= l) break;
        y[e] = acc[e];
    }
}

hipError_t launch_sum(const LaunchGroup& g, int side, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count,
                       side, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gram partial sums G_b = Z_b^T Z_b of a row chunk Z_b of an FP64 rows x l
// matrix, on FP64 MFMA 16x16x4.  A block is (row chunk, one upper 2 x 2
// group of 16x16 tiles); its four waves take consecutive quarters of the
// chunk's rows and stream them from memory straight into MFMA operands (16
// lanes read 128 contiguous bytes of a row): two column fragments of each
// side feed the four tiles' MFMAs, so every operand loaded serves two MFMAs
// (one tile per block: one MFMA per operand, and the L2 traffic was twice
// as high).  Four K steps per batch with the next batch's loads in flight;
// the four partial tiles are added in LDS in wave order (a fixed summation
// order).  Partials: gpart[chunk][l][l], upper tiles only (every entry with
// a <= b is written).  The grid is chunks x tile groups blocks.
// ---------------------------------------------------------------------------
// A zero in global memory: operands outside a matrix are loaded from here (an
// address select instead of a branch or a mask on the loaded value).  Never
// written.
__device__ double g_zero_word[2] = {0.0, 0.0};

static_assert(GRAM_THREADS == 256, "four waves per Gram tile group");

__device__ __forceinline__ void tile_of(int t, int nt, int& ta, int& tb) {
    // t-th upper tile (ta <= tb) of an nt x nt grid in row-major order over ta.
    int a = 0, rem = t;
    while (rem >= nt - a) { rem -= nt - a; a++; }
    ta = a;
    tb = a + rem;
}

template <int SRC>
__global__ __launch_bounds__(GRAM_THREADS) void k_gram(const Prob* __restrict__ probs,
                                                      const int32_t* __restrict__ pidx,
                                                      const int32_t* __restrict__ toff, int cnt,
                                                      int side, int iter) {
    __shared__ double part[3][4][4][64];  // waves 1-3 x tiles x MFMA entries
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    constexpr bool CROSS = SRC == GSRC_XM || SRC == GSRC_XA;
    if (iter >= 0 && iter > P.q) return;
    if (SRC == GSRC_QA && !second_pass(P, iter)) return;
    if (CROSS && P.mmode != (SRC == GSRC_XM ? M_EXPLICIT : M_APPROX)) return;
    if (SRC == GSRC_XY && (!P.fused || iter >= P.q)) return;
    const int l = P.l, lp = P.lp;
    const int nt = lp / 16;
    const int ns = (nt + 1) / 2;  // groups of 2 x 2 tiles per side
    // symmetric Grams: the upper groups; cross products Z1^T Z2: every group
    const int ntu = CROSS ? ns * ns : ns * (ns + 1) / 2;
    const int gb = side == SIDE_M ? P.gb_m : P.gb_n;
    // Blocks are handed to the eight XCDs in turn (block b to XCD b mod 8),
    // each with its own L2: with a multiple of 8 chunks, chunk c's tiles all
    // go to blocks b = c (mod 8), so every row of Z is fetched into one L2.
    int chunk, tt;
    if (gb % 8 == 0) {
        const int i = local >> 3;
        chunk = (local & 7) + 8 * (i / ntu);
        tt = i - (i / ntu) * ntu;
    } else {
        chunk = local / ntu;
        tt = local - chunk * ntu;
    }
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int rb = side == SIDE_M ? P.rb_m : P.rb_n;
    const int64_t c0 = (int64_t)chunk * rb;
    const int64_t c1 = min(rows, c0 + rb);
    const double* __restrict__ Z = SRC == GSRC_Y ? P.Y : SRC == GSRC_QA ? P.Qa : SRC == GSRC_U ? P.U
                                 : SRC == GSRC_V ? P.V : SRC == GSRC_XM ? P.Q1 : P.Q2;
    // second operand: Z itself, or A Q2 (in Y) for M = Q1^T A Q2, or the last
    // power step's input X for Q2^T X, or A^T A X (in Y) for X^T A^T A X
    const double* __restrict__ Z2 =
        (SRC == GSRC_XM || SRC == GSRC_XY) ? P.Y : SRC == GSRC_XA ? P.Xk : Z;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    // rows of this wave: quarter `wave` of the chunk (whole K steps of 4 rows)
    const int64_t qr = (((c1 - c0) + 3) / 4 + 3) / 4 * 4;
    const int64_t r0 = c0 + wave * qr;
    const int64_t r1 = min(c1, r0 + qr);
    int sa, sb;
    if (CROSS) {
        sa = tt / ns;
        sb = tt - sa * ns;
    } else {
        tile_of(tt, ns, sa, sb);
    }
    // tiles (2 sa + i, 2 sb + j); of a diagonal group of a symmetric Gram the
    // tile below the diagonal is skipped, as are tiles past the last one
    auto live = [&](int i, int j) {
        return 2 * sa + i < nt && 2 * sb + j < nt && (CROSS || sa != sb || i <= j);
    };
    // MFMA K slot g of step s is row rs + 4 s + g; U steps per batch, the next
    // batch's loads in flight while this batch's MFMAs run.
    constexpr int U = 2;
    f64x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    double xa[U][2], xb[U][2], ya[U][2], yb[U][2];
    // Loads are unconditional: columns past l are read at column l - 1 (their
    // tile entries are never written); rows past the wave's range are read
    // from a zero word.  Straight-line code lets the compiler wait for the
    // older batch while the newer one is in flight.
    int cac[2], cbc[2];
#pragma unroll
    for (int i = 0; i < 2; i++) {
        cac[i] = min(16 * (2 * sa + i) + li, l - 1);
        cbc[i] = min(16 * (2 * sb + i) + li, l - 1);
    }
    gdouble* Zg = as_global(Z);
    gdouble* Z2g = as_global(Z2);
    gdouble* zw = as_global(g_zero_word);
    auto load = [&](int64_t rs, double (&va)[U][2], double (&vb)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int64_t r = rs + 4 * u + lg;
            const bool okr = r < r1;
#pragma unroll
            for (int i = 0; i < 2; i++) {
                va[u][i] = *(okr ? Zg + r * l + cac[i] : zw);
                vb[u][i] = *(okr ? Z2g + r * l + cbc[i] : zw);
            }
        }
    };
    auto step = [&](const double (&va)[U][2], const double (&vb)[U][2]) {
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int i = 0; i < 2; i++)
#pragma unroll
                for (int j = 0; j < 2; j++)
                    if (live(i, j)) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(va[u][i], vb[u][j], acc[i][j], 0, 0, 0);
    };
    load(r0, xa, xb);
    for (int64_t rs = r0; rs < r1; rs += 8 * U) {
        load(rs + 4 * U, ya, yb);
        step(xa, xb);
        load(rs + 8 * U, xa, xb);
        step(ya, yb);
    }
    if (wave > 0)
#pragma unroll
        for (int i = 0; i < 2; i++)
#pragma unroll
            for (int j = 0; j < 2; j++)
#pragma unroll
                for (int e = 0; e < 4; e++) part[wave - 1][2 * i + j][e][lane] = acc[i][j][e];
    __syncthreads();
    if (wave != 0) return;
    double* out = P.gpart + (int64_t)chunk * l * l;
#pragma unroll
    for (int i = 0; i < 2; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            if (!live(i, j)) continue;
            const int cb = 16 * (2 * sb + j) + li;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int q = 2 * i + j;
                const double v = ((acc[i][j][e] + part[0][q][e][lane]) + part[1][q][e][lane]) + part[2][q][e][lane];
                const int ga = 16 * (2 * sa + i) + lg + 4 * e;  // f64 MFMA output row
                if (ga < l && cb < l) out[(int64_t)ga * l + cb] = v;
            }
        }
}

template <int SRC>
static hipError_t launch_gram_t(const LaunchGroup& g, int side, int iter, hipStream_t s) {
    hipLaunchKernelGGL(k_gram<SRC>, dim3(g.blocks), dim3(GRAM_THREADS), 0, s, g.probs, g.pidx,
                       g.toff, g.count, side, iter);
    return hipGetLastError();
}

hipError_t launch_gram(const LaunchGroup& g, int side, int src, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    switch (src) {
        case GSRC_Y: return launch_gram_t<GSRC_Y>(g, side, iter, s);
        case GSRC_QA: return launch_gram_t<GSRC_QA>(g, side, iter, s);
        case GSRC_U: return launch_gram_t<GSRC_U>(g, side, iter, s);
        case GSRC_V: return launch_gram_t<GSRC_V>(g, side, iter, s);
        case GSRC_XM: return launch_gram_t<GSRC_XM>(g, side, iter, s);
        case GSRC_XA: return launch_gram_t<GSRC_XA>(g, side, iter, s);
        case GSRC_XY: return launch_gram_t<GSRC_XY>(g, side, iter, s);
    }
    return hipErrorInvalidValue;
}

// Cross products Z1^T Z2 (every entry, no mirroring) from the partial sums,
// in the same fixed order as k_gram_reduce.  M = Q1^T (A Q2) is stored
// transposed into Mx (Mx[b][a] = M[a][b], the layout in which the QRCP reads
// R2 for M = R2^T); Q2^T X goes to G as it is.
__global__ __launch_bounds__(256) void k_xreduce(const Prob* __restrict__ probs,
                                                 const int32_t* __restrict__ pidx,
                                                 const int32_t* __restrict__ toff, int cnt,
                                                 int src) {
    __shared__ double part[4][64];
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (P.mmode != (src == GSRC_XM ? M_EXPLICIT : M_APPROX)) return;
    const int l = P.l;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = local * 64 + lane;
    const int nb = src == GSRC_XM ? P.gb_m : P.gb_n;
    const bool in = e < l * l;
    double s = 0.0;
    if (in) {
        const int64_t ll = (int64_t)l * l;
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int c = wave;
        for (; c + 12 < nb; c += 16) {
            s += P.gpart[c * ll + e];
            s1 += P.gpart[(c + 4) * ll + e];
            s2 += P.gpart[(c + 8) * ll + e];
            s3 += P.gpart[(c + 12) * ll + e];
        }
        for (; c < nb; c += 4) s += P.gpart[c * ll + e];
        s = (s + s1) + (s2 + s3);
    }
    part[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && in) {
        const double g = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        const int a = e / l, b = e - (e / l) * l;
        if (src == GSRC_XM) P.Mx[(int64_t)b * l + a] = g;
        else P.G[e] = g;
        if (!isfinite(g)) atomicOr(P.flags, FLAG_NONFINITE);
    }
}

hipError_t launch_xreduce(const LaunchGroup& g, int src, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_xreduce, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff,
                       g.count, src);
    return hipGetLastError();
}

// The last power step's input X (Q2 of the previous step, or Omega) kept
// for eq. (18) before the step's n-side orthonormalisation overwrites it.
__global__ __launch_bounds__(256) void k_keep_x(const Prob* __restrict__ probs,
                                                const int32_t* __restrict__ pidx,
                                                const int32_t* __restrict__ toff, int cnt,
                                                int iter) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (P.mmode != M_APPROX || iter != P.q) return;
    const int64_t e = (int64_t)local * 256 + threadIdx.x;
    if (e < P.n * P.l) P.Xk[e] = P.Q2[e];
}

hipError_t launch_keep_x(const LaunchGroup& g, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_keep_x, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff,
                       g.count, iter);
    return hipGetLastError();
}

// G[a][b] = G[b][a] = sum over chunks of gpart[chunk][min][max].  A block
// covers 64 entries; its four waves add chunks c = w (mod 4) in increasing
// order and the four parts are added in wave order: a fixed summation order.
__global__ __launch_bounds__(256) void k_gram_reduce(const Prob* __restrict__ probs,
                                                     const int32_t* __restrict__ pidx,
                                                     const int32_t* __restrict__ toff, int cnt,
                                                     int side, int second, int iter) {
    __shared__ double part[4][64];
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (iter >= 0 && iter > P.q) return;
    if (second && !second_pass(P, iter)) return;
    const int l = P.l;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int e = local * 64 + lane;
    const int nb = side == SIDE_M ? P.gb_m : P.gb_n;
    double s = 0.0;
    // upper entries only (contiguous reads of the partials); each is also
    // written to its mirror position
    const int a = e / l, b = e - (e / l) * l;
    const bool up = e < l * l && a <= b;
    if (up) {
        const int64_t o = (int64_t)a * l + b;
        const int64_t ll = (int64_t)l * l;
        double s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int c = wave;
        for (; c + 12 < nb; c += 16) {
            s += P.gpart[c * ll + o];
            s1 += P.gpart[(c + 4) * ll + o];
            s2 += P.gpart[(c + 8) * ll + o];
            s3 += P.gpart[(c + 12) * ll + o];
        }
        for (; c < nb; c += 4) s += P.gpart[c * ll + o];
        s = (s + s1) + (s2 + s3);
    }
    part[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && up) {
        const double g = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
        P.G[e] = g;
        if (a != b) P.G[(int64_t)b * l + a] = g;
        if (!isfinite(g)) atomicOr(P.flags, FLAG_NONFINITE);
    }
}

hipError_t launch_gram_reduce(const LaunchGroup& g, int side, int second, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gram_reduce, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff,
                       g.count, side, second, iter);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dst = src S for a block of AP_ROWS = 16 rows, S an l x l FP64 matrix
// (R^{-1} of a CholeskyQR pass, or Qs for U = Q1 Qs), on the FP64 MFMA
// (16x16x4).  Wave w owns column tiles w, w + 4, w + 8, ...; small blocks
// give several waves per SIMD, so one wave's load latency hides behind
// another's MFMAs (64-row blocks with four row tiles per wave measured
// slower).  K runs in blocks of 16, MFMA step u of block kb taking
// K = 16 kb + 4 u + g in lane group g: both operands stream from memory into
// registers (S is small and stays in cache), half a K block per batch with
// the next batch's loads in flight.  R^{-1} is upper triangular (its lower part
// is stored as exact zeros), so column tile c only needs K blocks 0 .. c:
// the R^{-1} stages skip the rest, about half of the MFMAs and of the reads
// of S, and the interleaved tiles give the four waves similar shares.  The
// finished 16 x l tile goes through LDS so that dst (row-major) and the
// transposed operand copy in the pass format are both written with
// contiguous runs.  H = column tiles per wave, ceil(nt / 4) (compile-time bound of the
// accumulator array).
// The stage (source, destination) is a template parameter: a run-time switch
// over these pointers was mis-compiled by the gfx950 backend (the default
// branch kept the source of another case).
// ---------------------------------------------------------------------------
constexpr int AP_ROWS = APPLY_ROWS;
static_assert(AP_ROWS == 16, "16-row blocks");

template <typename T>
__device__ void write_op_rows(const Prob& P, int side, int64_t r0, int nrows, const double* xs,
                              int ldx) {
    // op[c][r0 + rr] for c < l, rr < nrows: four columns per wave pass, lane & 15 = row
    static_assert(AP_ROWS == 16, "one row per lane of a 16-lane group");
    const int l = P.l;
    T* op = reinterpret_cast<T*>(side == SIDE_M ? P.qop : P.xop);
    const int64_t ld = side == SIDE_M ? P.ldq : P.ldx;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int rr = lane & 15;
    for (int c = 4 * wave + (lane >> 4); c < l; c += 16)
        if (rr < nrows) op[(int64_t)c * ld + r0 + rr] = conv_op<T>(xs[rr * ldx + c], 1.0f);
}

template <int MODE, int H>
__global__ __launch_bounds__(256, H <= 4 ? 5 : 1) void k_apply(const Prob* __restrict__ probs,
                                               const int32_t* __restrict__ pidx,
                                               const int32_t* __restrict__ toff, int cnt,
                                               int side, int iter) {
    extern __shared__ __align__(16) double lds[];  // 16 x lp output tile
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    if (iter >= 0 && iter > P.q) return;
    if (MODE == AP_Y_RINV_Y && (!P.fused || iter >= P.q)) return;
    const bool two = MODE != AP_Q1_QS_U && MODE != AP_Y_RINV_Y && second_pass(P, iter);
    if (MODE == AP_QA_RINV_Q && !two) return;
    const int l = P.l, lp = P.lp;
    const int nt = lp / 16;
    const int64_t rows = side == SIDE_M ? P.m : P.n;
    const int64_t r0 = (int64_t)local * AP_ROWS;
    const int nrows = (int)min((int64_t)AP_ROWS, rows - r0);
    const double* __restrict__ src = MODE == AP_Q1_QS_U ? P.Q1 : (MODE == AP_QA_RINV_Q) ? P.Qa : P.Y;
    const double* __restrict__ S = MODE == AP_Q1_QS_U ? P.G : P.Rinv;
    // First pass: into Qa when a second pass follows, else straight into Q
    // (and its operand copy for the next pass).  U = Q1 Qs: into U only.
    // The fused power step's Y R1^{-1} stays in Y (a block reads all of its
    // rows before it writes them back).
    double* const qdst = MODE == AP_Q1_QS_U ? P.U : side == SIDE_M ? P.Q1 : P.Q2;
    double* const dst = (MODE == AP_Y_RINV_QA && two) ? P.Qa : MODE == AP_Y_RINV_Y ? P.Y : qdst;
    const bool op = MODE != AP_Q1_QS_U && MODE != AP_Y_RINV_Y && !(MODE == AP_Y_RINV_QA && two);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int nct = nt > wave ? (nt - wave + 3) / 4 : 0;  // column tiles of this wave (may be 0)
    // K blocks this wave visits: up to its last column tile when S = R^{-1}
    // (upper triangular), all of them for U = Q1 Qs
    constexpr bool TRI = MODE != AP_Q1_QS_U;
    const int nkb = nct > 0 ? (TRI ? wave + 4 * (nct - 1) + 1 : nt) : 0;
    const int64_t arow = r0 + li;  // row of src this lane feeds
    const double* __restrict__ arp = src + min(arow, rows - 1) * l;  // clamped: loads are unconditional

    f64x4 acc[H];
#pragma unroll
    for (int t = 0; t < H; t++) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
    // Batches of U MFMA steps (4 K each), BPK = 4 / U batches per K block.
    // Two steps per batch keep the kernel at 5 waves per SIMD, so that the
    // 1250 blocks of a 20000-row apply run in one round of the CU slots (four
    // steps per batch: 3 waves, 1.6 rounds).
    constexpr int U = 2, BPK = 4 / U;
    double a0[U], a1[U], b0[U][H], b1[U][H];
#pragma unroll
    for (int u = 0; u < U; u++)
#pragma unroll
        for (int t = 0; t < H; t++) b0[u][t] = b1[u][t] = 0.0;
    // Operands past the matrices come from clamped addresses (junk rows and
    // columns of the tile are never written) except the K slots past l, whose
    // A operand is read from a zero word.  Tile t of the wave (column tile
    // wave + 4 t) takes part in K block kb when t < nct and, for triangular
    // S, kb <= wave + 4 t: a wave-uniform test, so loads and MFMAs of the
    // skipped blocks are branched over, not masked.
    gdouble* ag = as_global(arp);
    gdouble* Sg = as_global(S);
    gdouble* zw = as_global(g_zero_word);
    int cc[H];
#pragma unroll
    for (int t = 0; t < H; t++) cc[t] = min(16 * (wave + 4 * t) + li, l - 1);
    auto part = [&](int kb, int t) { return t < nct && (!TRI || kb <= wave + 4 * t); };
    const int nbat = nkb * BPK;
    auto load = [&](int bi, double (&a)[U], double (&b)[U][H]) {
        const int kb = bi / BPK;
#pragma unroll
        for (int u = 0; u < U; u++) {
            const int k = 16 * kb + 4 * ((bi % BPK) * U + u) + lg;
            a[u] = *((bi < nbat && k < l) ? ag + k : zw);
            gdouble* srow = Sg + (int64_t)min(k, l - 1) * l;
#pragma unroll
            for (int t = 0; t < H; t++)
                if (part(kb, t)) b[u][t] = srow[cc[t]];
        }
    };
    auto step = [&](int bi, const double (&a)[U], const double (&b)[U][H]) {
        const int kb = bi / BPK;
#pragma unroll
        for (int u = 0; u < U; u++)
#pragma unroll
            for (int t = 0; t < H; t++)
                if (bi < nbat && part(kb, t))
                    acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u][t], acc[t], 0, 0, 0);
    };
    // Two register buffers in turn: the compiler waits for the older batch
    // while the newer one is in flight.
    load(0, a0, b0);
    for (int bi = 0; bi < nbat; bi += 2) {
        load(bi + 1, a1, b1);
        step(bi, a0, b0);
        load(bi + 2, a0, b0);
        step(bi + 1, a1, b1);
    }
    // f64 MFMA output: lane (i, g), entry e -> row g + 4e, column i of the tile.
    double* xs = lds;  // 16 x lp
#pragma unroll
    for (int t = 0; t < H; t++)
        if (t < nct)
#pragma unroll
            for (int e = 0; e < 4; e++)
                xs[(lg + 4 * e) * lp + 16 * (wave + 4 * t) + li] = acc[t][e];
    __syncthreads();
    if (MODE == AP_Y_RINV_QA && two) {
        // First factor of the final orthonormalisation.  Rank-deficient
        // sketch (rank below l, e.g. rank(A) < l): column j whose Cholesky
        // pivot was clamped (marker tau[j] = 1) spans no direction of Y; it
        // becomes a Gaussian column of norm about 1 (its own counter-based
        // stream) and row j of the accumulated R is zeroed, so the second
        // pass makes Q orthonormal while Q R still reproduces Y.  A full-rank
        // sketch leaves everything untouched.
        const uint64_t stream =
            P.seed ^ (side == SIDE_M ? 0x6A09E667F3BCC908ull : 0xBB67AE8584CAA73Bull);
        const double sc = 1.0 / sqrt((double)rows);
        constexpr int NQ = (LMAX + 63) / 64;  // columns per lane
        bool def[NQ];
#pragma unroll
        for (int q = 0; q < NQ; q++) def[q] = lane + 64 * q < l && P.tau[lane + 64 * q] != 0.0;
        for (int r = wave; r < nrows; r += 4)
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                const int c = lane + 64 * q;
                if (c >= l) break;
                double v = xs[r * lp + c];
                if (def[q]) {
                    double z0, z1;
                    gauss_pair(stream, (uint64_t)((r0 + r) * l + c), z0, z1);
                    v = z0 * sc;
                }
                dst[(r0 + r) * l + c] = v;
            }
        if (local == 0)
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                // rows j = 64 q + bit of the clamped pivots, wave j % 4 each
                unsigned long long mk = __ballot(def[q]);
                while (mk) {
                    const int j = 64 * q + __ffsll((long long)mk) - 1;
                    mk &= mk - 1;
                    if ((j & 3) == wave)
                        for (int c = lane; c < l; c += 64) P.Racc[j * l + c] = 0.0;
                }
            }
        return;
    }
    for (int r = wave; r < nrows; r += 4)
        for (int c = lane; c < l; c += 64) dst[(r0 + r) * l + c] = xs[r * lp + c];
    if (op && P.prec != P_FP8) {
        switch (P.prec) {
            case P_F64: write_op_rows<double>(P, side, r0, nrows, xs, lp); break;
            case P_F32: write_op_rows<float>(P, side, r0, nrows, xs, lp); break;
            default: write_op_rows<uint16_t>(P, side, r0, nrows, xs, lp); break;
        }
    }
}

template <int MODE, int H>
static hipError_t launch_apply_t(const LaunchGroup& g, int side, int lmax, int iter,
                                 hipStream_t s) {
    const int lp = (lmax + 15) / 16 * 16;
    const size_t lds = sizeof(double) * (size_t)AP_ROWS * lp;
    hipLaunchKernelGGL((k_apply<MODE, H>), dim3(g.blocks), dim3(256), lds, s, g.probs, g.pidx,
                       g.toff, g.count, side, iter);
    return hipGetLastError();
}

template <int MODE>
static hipError_t launch_apply_m(const LaunchGroup& g, int side, int lmax, int iter,
                                 hipStream_t s) {
    const int nt = (lmax + 15) / 16;
    const int qn = (nt + 3) / 4;
    if (qn <= 1) return launch_apply_t<MODE, 1>(g, side, lmax, iter, s);
    if (qn <= 2) return launch_apply_t<MODE, 2>(g, side, lmax, iter, s);
    if (qn <= 3) return launch_apply_t<MODE, 3>(g, side, lmax, iter, s);
    if (qn <= 4) return launch_apply_t<MODE, 4>(g, side, lmax, iter, s);
    return launch_apply_t<MODE, 5>(g, side, lmax, iter, s);
}

hipError_t launch_apply(const LaunchGroup& g, int side, int mode, int lmax, int iter,
                        hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    switch (mode) {
        case AP_Y_RINV_QA: return launch_apply_m<AP_Y_RINV_QA>(g, side, lmax, iter, s);
        case AP_QA_RINV_Q: return launch_apply_m<AP_QA_RINV_Q>(g, side, lmax, iter, s);
        case AP_Y_RINV_Q: return launch_apply_m<AP_Y_RINV_Q>(g, side, lmax, iter, s);
        case AP_Q1_QS_U: return launch_apply_m<AP_Q1_QS_U>(g, side, lmax, iter, s);
        case AP_Y_RINV_Y: return launch_apply_m<AP_Y_RINV_Y>(g, side, lmax, iter, s);
    }
    return hipErrorInvalidValue;
}

// V = Q2 P: V[r][c] = Q2[r][perm[c]].
__global__ __launch_bounds__(256) void k_gather_v(const Prob* __restrict__ probs,
                                                  const int32_t* __restrict__ pidx,
                                                  const int32_t* __restrict__ toff, int cnt) {
    int local;
    const Prob& P = group_prob(probs, pidx, toff, cnt, local);
    const int l = P.l;
    const int64_t e = (int64_t)local * 256 + threadIdx.x;
    if (e >= P.n * l) return;
    const int64_t r = e / l;
    const int c = (int)(e % l);
    P.V[e] = P.Q2[r * l + P.perm[c]];
}

hipError_t launch_gather_v(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_v, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count);
    return hipGetLastError();
}

}  // namespace cor
