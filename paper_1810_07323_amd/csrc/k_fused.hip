// Fused power step: A^T (A X) in one read of A (the loop of Alg. 3 as
// printed, C2 = A^T (A C2), for the iterations before the final pair).
//
// A block (8 waves) owns a contiguous range of kc_f rows of A (one of s_f
// row splits).  Its n x lp partial sum P of A^T (A X) lives in registers as
// MFMA accumulators: the 16 x 16 tiles of P are dealt to the waves in turn
// (tile t to wave t mod 8, TPW tiles per wave at most).  The rows are walked
// in chunks of 8 (rows 8 .. 15 of the MFMA row tile are zero, which keeps
// the next chunk's loads in few registers):
//   0. the chunk (8 x n) is in LDS; the loads of the next chunk are issued
//      into registers before any of the work below, so that they are in
//      flight while it runs, and stored to LDS after it;
//   1. Y1 = chunk X (8 x lp) on the MFMA (FP32 16x16x4 with FP32
//      accumulation, or FP64 16x16x4): the eight waves take consecutive
//      slices of K = n, lane group g the K slots k0 + 4 g + s of each
//      16-wide step; X streams from the cache (it is n x lp, shared by all);
//   2. the eight partial blocks are added in LDS in wave order;
//   3. P += chunk^T Y1: every tile of P takes K = 8 (two MFMAs), both
//      operands from LDS.
// Every element of A is read from HBM once per step.  The partial sums go to
// ypart[split][n][lp]; k_sum adds the splits in a fixed order into the FP64
// n x l matrix Y = A^T A X.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace cor {

constexpr int ATA_THREADS = 512;
constexpr int ATA_R = 8;  // rows of A per chunk (the upper half of a 16-row MFMA tile)

__device__ __forceinline__ const Prob& ata_prob(const Prob* __restrict__ probs,
                                                const int32_t* __restrict__ pidx,
                                                const int32_t* __restrict__ toff, int cnt,
                                                int& local) {
    const int j = find_group(toff, cnt, (int)blockIdx.x);
    local = (int)blockIdx.x - toff[j];
    return probs[pidx[j]];
}

// Row stride (elements) of the chunk in LDS: n rounded up to 4, plus 4, so
// that the rows of an MFMA operand fall on different banks.
__host__ __device__ inline int64_t ata_stride(int64_t n) { return (n + 3) / 4 * 4 + 4; }

// LDS bytes of one block: the chunk, the eight partial Y1 blocks and Y1
// (16-row MFMA blocks).
__host__ __device__ inline int64_t ata_lds(int64_t n, int lp, int sz) {
    return (ATA_R * ata_stride(n) + 9 * 16 * (int64_t)lp) * sz;
}

template <int PREC, int NT, int TPW, int CPT>
__global__ __launch_bounds__(ATA_THREADS) void k_ata(const Prob* __restrict__ probs,
                                                     const int32_t* __restrict__ pidx,
                                                     const int32_t* __restrict__ toff, int cnt,
                                                     int iter) {
    static_assert(PREC == P_F32 || PREC == P_F64, "FP32 or FP64 passes");
    typedef typename PrecT<PREC>::T T;  // pass format = accumulation format here
    typedef typename std::conditional<PREC == P_F64, f64x4, f32x4>::type AccV;
    extern __shared__ __align__(16) unsigned char smem[];
    int local;
    const Prob& P = ata_prob(probs, pidx, toff, cnt, local);
    if (!P.fused || iter >= P.q) return;
    constexpr int LP = 16 * NT;
    if (P.lp != LP) return;  // a launch serves one column-tile class
    const int64_t m = P.m, n = P.n, lda = P.lda, ldx = P.ldx;
    const int64_t st = ata_stride(n);
    T* __restrict__ As = reinterpret_cast<T*>(smem);  // [8][st] chunk of A
    T* __restrict__ Yp = As + ATA_R * st;              // [8][16][LP] partial Y1
    T* __restrict__ Ys = Yp + 8 * 16 * LP;             // [16][LP] Y1 of the chunk
    const T* __restrict__ A = reinterpret_cast<const T*>(P.A);
    const T* __restrict__ X = reinterpret_cast<const T*>(P.xop);  // [LP][ldx]: row c = column c
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int64_t rb = (int64_t)local * P.kc_f;
    const int64_t re = min(m, rb + P.kc_f);
    const int64_t ntile = ((n + 15) / 16) * NT;

    // chunk loads: columns c = tid + 512 j of each of the 8 rows (the row
    // address is the same for the whole block, the column offset per thread)
    T pre[ATA_R][CPT];
    const int ni = (int)n;  // n <= ATA_NMAX32
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int r = 0; r < ATA_R; r++) {
            const bool rok = r0 + r < re;
            const T* __restrict__ rowp = A + min(r0 + r, m - 1) * lda;
#pragma unroll
            for (int j = 0; j < CPT; j++) {
                const int c = tid + ATA_THREADS * j;
                pre[r][j] = (rok && c < ni) ? rowp[c] : T(0);
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int r = 0; r < ATA_R; r++)
#pragma unroll
            for (int j = 0; j < CPT; j++) {
                const int c = tid + ATA_THREADS * j;
                if (c < ni) As[r * st + c] = pre[r][j];
            }
    };

    AccV pacc[TPW];
#pragma unroll
    for (int t = 0; t < TPW; t++)
#pragma unroll
        for (int e = 0; e < 4; e++) pacc[t][e] = T(0);
    // K slice of this wave in step 1
    const int64_t kw = ((n + 7) / 8 + 15) / 16 * 16;
    const int64_t kb = wave * kw, ke = min(n, kb + kw);

    fetch(rb);
    for (int64_t r0 = rb; r0 < re; r0 += ATA_R) {
        stash();
        __syncthreads();
        if (r0 + ATA_R < re) fetch(r0 + ATA_R);  // in flight during the work below
        // 1. partial Y1 over this wave's K slice
        AccV acc[NT];
#pragma unroll
        for (int c = 0; c < NT; c++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[c][e] = T(0);
        for (int64_t k0 = kb; k0 < ke; k0 += 16) {
            const int64_t kq = k0 + 4 * lg;
            T a[4], b[NT][4];
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int64_t k = kq + e;
                const bool ok = k < ke;
                a[e] = (ok && li < ATA_R) ? As[li * st + k] : T(0);
#pragma unroll
                for (int c = 0; c < NT; c++)
                    b[c][e] = ok ? X[(int64_t)(16 * c + li) * ldx + k] : T(0);
            }
#pragma unroll
            for (int e = 0; e < 4; e++)
#pragma unroll
                for (int c = 0; c < NT; c++) {
                    if constexpr (PREC == P_F32)
                        acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[c][e], acc[c], 0, 0, 0);
                    else
                        acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e], b[c][e], acc[c], 0, 0, 0);
                }
        }
        // f32 form: (row 4g + e, col i); f64 form: (row g + 4e, col i)
#pragma unroll
        for (int c = 0; c < NT; c++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = PREC == P_F64 ? lg + 4 * e : 4 * lg + e;
                Yp[(wave * 16 + row) * LP + 16 * c + li] = acc[c][e];
            }
        __syncthreads();
        // 2. Y1 = sum of the eight partials in wave order
        for (int e = tid; e < 16 * LP; e += ATA_THREADS) {
            T s = Yp[e];
#pragma unroll
            for (int w = 1; w < 8; w++) s += Yp[w * 16 * LP + e];
            Ys[e] = s;
        }
        __syncthreads();
        // 3. P += chunk^T Y1 (K = 8 rows: two MFMA steps per tile)
#pragma unroll
        for (int t = 0; t < TPW; t++) {
            const int64_t tt = wave + 8 * (int64_t)t;
            if (tt < ntile) {
                const int64_t jt = tt / NT;
                const int ct = (int)(tt - jt * NT);
                const int64_t j = 16 * jt + li;
                const bool jok = j < n;
#pragma unroll
                for (int kk = 0; kk < ATA_R; kk += 4) {
                    const T av = jok ? As[(kk + lg) * st + j] : T(0);
                    const T bv = Ys[(kk + lg) * LP + 16 * ct + li];
                    if constexpr (PREC == P_F32)
                        pacc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, pacc[t], 0, 0, 0);
                    else
                        pacc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, pacc[t], 0, 0, 0);
                }
            }
        }
        __syncthreads();  // the chunk and Y1 are rewritten by the next step
    }
    // the split's partial sums
    T* __restrict__ out = reinterpret_cast<T*>(P.ypart) + (int64_t)local * n * LP;
#pragma unroll
    for (int t = 0; t < TPW; t++) {
        const int64_t tt = wave + 8 * (int64_t)t;
        if (tt < ntile) {
            const int64_t jt = tt / NT;
            const int ct = (int)(tt - jt * NT);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int64_t pr = 16 * jt + (PREC == P_F64 ? lg + 4 * e : 4 * lg + e);
                if (pr < n) out[pr * LP + 16 * ct + li] = pacc[t][e];
            }
        }
    }
}

// Compile-time bounds: TPW tiles of P per wave, CPT columns of a chunk row
// per thread (n <= ATA_NMAX for the format).
template <int PREC, int NT, int TPW>
static hipError_t launch_ata_t(const LaunchGroup& g, size_t lds, int iter, hipStream_t s) {
    constexpr int CPT = ((PREC == P_F64 ? ATA_NMAX64 : ATA_NMAX32) + ATA_THREADS - 1) /
                        ATA_THREADS;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_ata<PREC, NT, TPW, CPT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, ATA_LDS);
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((k_ata<PREC, NT, TPW, CPT>), dim3(g.blocks), dim3(ATA_THREADS), lds, s,
                       g.probs, g.pidx, g.toff, g.count, iter);
    return hipGetLastError();
}

// Instances without register spills only: tiles per wave up to
// ata_max_tiles_per_wave.
template <int PREC, int NT>
static hipError_t launch_ata_n(const LaunchGroup& g, int tpw, size_t lds, int iter,
                               hipStream_t s) {
    if (tpw <= 4) return launch_ata_t<PREC, NT, 4>(g, lds, iter, s);
    if (tpw <= 8) return launch_ata_t<PREC, NT, 8>(g, lds, iter, s);
    if constexpr (PREC == P_F32 || NT <= 2)
        if (tpw <= 12) return launch_ata_t<PREC, NT, 12>(g, lds, iter, s);
    if constexpr (PREC == P_F32)
        if (tpw <= 16) return launch_ata_t<PREC, NT, 16>(g, lds, iter, s);
    if constexpr (PREC == P_F32 && NT <= 2)
        if (tpw <= 24) return launch_ata_t<PREC, NT, 24>(g, lds, iter, s);
    return hipErrorInvalidValue;
}

int ata_tiles_per_wave(int64_t n, int lp) { return (int)((((n + 15) / 16) * (lp / 16) + 7) / 8); }

int ata_max_tiles_per_wave(int prec, int lp) {
    const int nt = lp / 16;
    if (prec == P_F32) return nt <= 2 ? 24 : 16;
    return nt <= 2 ? 12 : 8;
}

size_t ata_lds_bytes(int64_t n, int lp, int prec) {
    return (size_t)ata_lds(n, lp, prec == P_F64 ? 8 : 4);
}

hipError_t launch_ata(int prec, int nt, int tpw, size_t lds, const LaunchGroup& g, int iter,
                      hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
#define ATA_CASE(PR, N) \
    if (prec == PR && nt == N) return launch_ata_n<PR, N>(g, tpw, lds, iter, s);
    ATA_CASE(P_F32, 1) ATA_CASE(P_F32, 2) ATA_CASE(P_F32, 3) ATA_CASE(P_F32, 4)
    ATA_CASE(P_F64, 1) ATA_CASE(P_F64, 2) ATA_CASE(P_F64, 3) ATA_CASE(P_F64, 4)
#undef ATA_CASE
    return hipErrorInvalidValue;
}

}  // namespace cor
