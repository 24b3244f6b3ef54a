// Shared device-side definitions of the CoR-UTV library (gfx950).
//
// Every kernel works on a list of problem descriptors (Prob) that live in
// device memory.  A launch covers one stage of the method for a group of
// problems: block b belongs to problem pidx[j] where toff[j] <= b < toff[j+1]
// (toff is an exclusive prefix sum of per-problem block counts).  A single
// decomposition is the group of one.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cor {

enum Prec : int32_t { P_F64 = 0, P_F32 = 1, P_BF16 = 2, P_FP8 = 3 };

constexpr int LMAX = 264;   // largest l = k + p supported
constexpr int LPMAX = 272;  // LMAX padded to a multiple of 16
constexpr int NTMAX = 17;   // LPMAX / 16
constexpr int SCALE_CHUNKS = 64;  // most row chunks of an FP8 operand-scale reduction

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// Flags (device word per problem; mirrored by COR_FLAG_* of the public header).
constexpr int32_t FLAG_RANK_DEF = 2;
constexpr int32_t FLAG_NONFINITE = 4;
constexpr int32_t FLAG_SYNC_TIMEOUT = 8;

// One decomposition: inputs, workspace and outputs (all device pointers).
struct Prob {
    const void* A;          // m x n, row-major, leading dimension lda, format prec
    const float* colscale;  // FP8: n column scales of A
    int64_t m, n, lda;
    int32_t k, l, lp, q;    // l = k + p, lp = l rounded up to 16
    int32_t prec, cholqr2_all, report, avec;  // avec: A rows 16-byte aligned

    // Operand copies of the skinny factors, stored transposed: [lp][ld]
    // (row c holds column c of the factor), in the pass format.
    void* xop;   // n-side: Omega, then Q2
    void* qop;   // m-side: Q1
    int64_t ldx, ldq;
    float* xscale;  // FP8: per-column scales of xop (lp)
    float* qscale;  // FP8: per-column scales of qop (lp)

    // Split-K partial sums of a pass over A: [splits][rows][lp], FP32 (FP64
    // in F64 mode).
    void* ypart;
    int32_t s_ax, s_atx;      // number of K splits of A*X and A^T*X
    int64_t kc_ax, kc_atx;    // K range of one split (multiple of the K tile)

    // FP64 work arrays.
    double* Y;    // max(m, n) x l  : reduced sketch
    double* Qa;   // max(m, n) x l  : first CholeskyQR factor
    double* Q1;   // m x l
    double* Q2;   // n x l (Omega in FP64 before the first pass)
    double* gpart;  // Gram partial sums: [blocks][l][l]
    int32_t rb_m, rb_n;  // rows per Gram block on the m- and n-side
    int32_t gb_m, gb_n;  // number of Gram blocks on each side
    double* G;     // l x l reduced Gram
    double* R;     // l x l current Cholesky factor (upper)
    double* Rinv;  // l x l its inverse (upper)
    double* Racc;  // l x l R of the first CholeskyQR pass
    double* R2;    // l x l R factor of the last Y2 = A^T Q1 (M = R2^T)
    double* Qt;    // l x l reflectors of the QRCP (row j = v_j)
    double* tau;   // 2 LMAX: tau[j] of the reflectors, then the column signs of T
    double* rep;   // 16 doubles of report scratch
    int32_t* flags;
    // FP8: per-chunk column maxima of the factor an operand copy is made from
    // ([chunks][lp]) and the row chunks of each side.
    float* scpart;
    int32_t sch_m, sch_n;

    // Outputs.
    double* U;
    double* T;
    double* V;
    int32_t* perm;  // l (always written; the caller's pointer or workspace)

    const double* omega;  // optional caller test matrix (n x l FP64)
    uint64_t seed;

    // Compression (eq. (14) / eq. (18)) and orientation options.
    int32_t mmode;       // M_R2T, M_EXPLICIT or M_APPROX
    int32_t ulv;         // 1: this is the URV of A^T behind a ULV request
    const double* msrc;  // l x l, msrc[c][i] = M[i][c]: R2 (M = R2^T) or Mx
    double* Mx;          // l x l: M^T from the explicit product or eq. (18)
    double* R1;          // l x l: R factor of the last Y1 (eq. (18))
    double* Xk;          // n x l: the last power step's input X (eq. (18))
    double* Tout;        // ULV: the caller's T, written as the transpose of T
    const void* ulv_src; // ULV: the caller's A (m_caller = n rows, leading dimension ulv_lda)
    int64_t ulv_lda;

    // Fused power step (A^T (A X) in one read of A) for the iterations < q:
    // s_f row splits of kc_f rows (a multiple of 128) each, partials in ypart.
    int32_t fused, s_f;
    int64_t kc_f;
};

// Compression of A to the l x l core.
enum MMode : int32_t {
    M_R2T = 0,       // M = Q1^T A Q2 = R2^T, no pass over A
    M_EXPLICIT = 1,  // M = Q1^T (A Q2), one more pass over A (eq. (14) as printed)
    M_APPROX = 2     // M = Q1^T Y1 (Q2^T X)^+ = R1 (Q2^T X)^-1 (eq. (18))
};

// Whether the orthonormalisation of this iteration takes the second
// CholeskyQR pass: always for the final pair (iteration q), and inside the
// power loop only when asked for.  iter < 0 marks calls outside the loop.
__device__ __forceinline__ bool second_pass(const Prob& P, int iter) {
    return iter < 0 || iter == P.q || P.cholqr2_all != 0;
}

// U = Q1 Qt diag(sign) through the l x l product Qs and one MFMA product
// (large l, or more row blocks of Q1 than the GPU holds at once), else by the
// reflectors applied straight to the rows of Q1.  Per problem, so that a
// problem's arithmetic does not depend on what it is batched with.
__host__ __device__ inline bool u_via_qs(int64_t m, int l) { return l > 128 || m > 16384; }

__device__ __forceinline__ int find_group(const int32_t* __restrict__ toff, int cnt, int b) {
    int lo = 0, hi = cnt - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (toff[mid] <= b) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int P> struct PrecT;
template <> struct PrecT<P_F64> { typedef double T; typedef double Acc; static constexpr int SZ = 8; };
template <> struct PrecT<P_F32> { typedef float T; typedef float Acc; static constexpr int SZ = 4; };
template <> struct PrecT<P_BF16> { typedef uint16_t T; typedef float Acc; static constexpr int SZ = 2; };
template <> struct PrecT<P_FP8> { typedef uint8_t T; typedef float Acc; static constexpr int SZ = 1; };

// Global-memory view of a device pointer: loads through it are global (not
// flat) instructions, which the compiler counts without involving LDS.
typedef const __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) double gdouble_rw;
__device__ __forceinline__ gdouble* as_global(const double* p) { return (gdouble*)p; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// DPP lane moves of a double (two 32-bit halves); CTRL is a DPP control word.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum over each aligned group of 8 lanes, result in every lane of the group:
// swap neighbours (quad_perm 1,0,3,2), swap pairs (quad_perm 2,3,0,1), then
// mirror each half-row of 8 (row_half_mirror), which pairs the two quads.
__device__ __forceinline__ double sum8_dpp(double v) {
    v += dpp_mov<0xB1>(v);
    v += dpp_mov<0x4E>(v);
    v += dpp_mov<0x141>(v);
    return v;
}
// Sum over each 16-lane row (the 8-lane sums, then the mirrored half).
__device__ __forceinline__ double sum16_dpp(double v) {
    v = sum8_dpp(v);
    v += dpp_mov<0x140>(v);
    return v;
}

// Binary32 -> bfloat16, round to nearest even (NaN kept quiet).
__device__ __forceinline__ uint16_t f32_to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// Binary32 -> OCP E4M3FN code, round to nearest even, saturating to +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3(float x) {
    uint32_t b = __float_as_uint(x);
    uint8_t sign = (uint8_t)((b >> 24) & 0x80u);
    float a = fabsf(x);
    if (a != a) return 0x7F;
    if (a >= 448.0f) return sign | 0x7E;
    // Normal range of E4M3 starts at 2^-6; below it the spacing is 2^-9.
    if (a < 0.015625f) {
        // subnormal: value = m * 2^-9, m in [0, 8]; m = 8 is the smallest normal (code 0x08)
        float t = a * 512.0f;                 // exact scaling by a power of two
        float r = rintf(t);                   // round half to even
        return sign | (uint8_t)r;
    }
    int e;
    float f = frexpf(a, &e);                  // a = f * 2^e, f in [0.5, 1)
    // mantissa with 3 fraction bits: a = (1 + m/8) 2^(e-1)
    float t = f * 16.0f;                      // in [8, 16)
    float r = rintf(t);                       // round half to even on the 3-bit mantissa
    int ee = e - 1 + 7;                       // biased exponent
    int mm = (int)r - 8;
    if (mm == 8) { mm = 0; ee += 1; }
    if (ee > 15 || (ee == 15 && mm == 7)) return sign | 0x7E;
    return sign | (uint8_t)((ee << 3) | mm);
}

}  // namespace cor
