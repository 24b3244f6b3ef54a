// l x l stages of CoR-UTV and the assembly of the factors.
//   - Cholesky of the Gram matrix (CholeskyQR of C1, C2 in Alg. 3) and the
//     accumulated R factor of the orthonormalisation;
//   - the column-pivoted QR of the compressed matrix M = Q1^T A Q2 = R2^T,
//     eq. (15): Businger-Golub pivoting on exactly recomputed trailing
//     column norms (lowest index on ties), Householder reflections, T_jj >= 0;
//   - U = Q1 Qt and V = Q2 P of eq. (16);
//   - the accuracy report and the stand-alone format conversion.
#include "common.h"
#include "kernels.h"

#include <algorithm>
#include <utility>

namespace cor {

constexpr int QRT_LMAX = 128;      // register-resident QRCP: up to 8 lanes per column
constexpr int QRT_THREADS = 8 * QRT_LMAX;
constexpr int QHY_RR = 36;     // registers + LDS QRCP: register rows per lane,
constexpr int QHY_LMAX = 224;  // largest l (LDS rows per lane <= 20: 143 KB)
constexpr int QHY_LR = (QHY_LMAX + 3) / 4 - QHY_RR;

__device__ __forceinline__ const Prob& group_prob2(const Prob* probs, const int32_t* pidx,
                                                   const int32_t* toff, int cnt, int& local) {
    const int j = find_group(toff, cnt, blockIdx.x);
    local = blockIdx.x - toff[j];
    return probs[pidx[j]];
}

// ---------------------------------------------------------------------------
// Cholesky and inverse in one sweep over an n x n block (n <= 128), with the
// work matrix held in FP64 MFMA accumulator tiles.
//
// Symmetric Gaussian elimination on [G | I], sixteen columns at a time.  The
// upper triangle of the np x np work matrix X (np = n rounded up to 16) holds
// the Schur complement, the strict lower triangle accumulates E = L^{-1}
// (G = L D L^T, L unit lower).  Row j is final once its column block has been
// eliminated and then holds v_j (row j of the Schur complement at step j) and
// E[j][0..j), so that
//   R    = D^{1/2} L^T   : R[j][b]    = v_j[b] / sqrt(d_j)          (b >= j)
//   R^-1 = L^{-T} D^-1/2 : R^-1[b][j] = E[j][b] / sqrt(d_j)         (b <  j)
// X is cut into 16 x 16 tiles kept in the registers of the work-group in the
// layout of the f64 16x16x4 MFMA result (lane 16 g + i, register r holds row
// g + 4 r, column i).  Diagonal tile t sits in slot 0 of wave t.  Per tile
// column K:
//   A. the wave owning diagonal tile K factors it, X_KK = L_K D_K L_K^T, in
//      registers: lane a holds row a, pivot step j takes row j from lane j by
//      lane reads, and the sixteen dependent steps need no LDS and no barrier;
//      it publishes the rows v (upper part) and L_K^{-1} (lower part) and 1/d;
//   B. every other tile of tile row K becomes L_K^{-1} X_KQ (four MFMAs with
//      K = 4), and the tile row is published;
//   C. every tile with rows below tile row K subtracts
//      sum_k (v_k[a] / d_k) w_k[b] over the sixteen rows k of the tile row
//      (four MFMAs), w = v in the upper triangle and the E rows in the lower
//      one (L_K^{-1}, 1 on the diagonal and 0 right of it, for tile column K).
// The owner of the next diagonal tile updates it first and factors it while
// the other tiles are updated, so the serial path per tile column is the
// 16 x 16 factor and two four-MFMA products.  Two barriers per tile column.
// A pivot d_j <= tol (l 2^-52 max_i G_ii) is clamped to tol (numerically
// rank-deficient sketch) and flagged; padding rows get a pivot above tol.
// ---------------------------------------------------------------------------
constexpr int CRT_THREADS = 1024;
constexpr int CRT_LMAX = 128;
constexpr int CH_SLOTS = 4;  // 16 x 16 tiles per wave (64 tiles on 16 waves)
// Row stride of the published tile row: rows g and g + 1 of an MFMA operand
// read fall into different halves of the LDS banks.
constexpr int CH_WLD = CRT_LMAX + 16;

// 1/d from the hardware estimate and two Newton steps y <- y + y (1 - d y).
__device__ __forceinline__ double recip_nr(double d) {
    double y = __builtin_amdgcn_rcp(d);
#pragma unroll
    for (int it = 0; it < 2; it++) y = fma(y, fma(-d, y, 1.0), y);
    return y;
}

// 1/d with one third-order correction of the hardware estimate y0 (relative
// error e of order 2^-23): y0 (1 + e + e^2) has relative error e^3.
__device__ __forceinline__ double recip3(double d) {
    const double y = __builtin_amdgcn_rcp(d);
    const double e = fma(-d, y, 1.0);
    return fma(y, fma(e, e, e), y);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// LDS operations of one wave complete in order: this orders a wave's own
// LDS writes before its later reads.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct CholShared {
    double w[16][CH_WLD];  // tile row K after B (rows 16 K .. 16 K + 15)
    double dt[2][16][17];  // factored diagonal tile by parity of K: v, L_K^{-1}
    double inv[2][16];     // 1 / d of tile column K, by parity of K
    double d[CRT_LMAX];    // pivots
    double sq[CRT_LMAX];   // sqrt(d)
    double rs[CRT_LMAX];   // 1 / sqrt(d)
    double dm[CRT_LMAX];   // 1 where the pivot was clamped, else 0
    int clamped;
};

// Lane J of each 16-lane row of the wave, to every lane of that row (DPP
// row_newbcast: one 64-bit VGPR move, no trip through scalar registers).
template <int J> __device__ __forceinline__ double row_bcast(double v) {
    return __longlong_as_double(__builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + J, 0xF, 0xF, false));
}

// Value v of lane `src` of the wave (any lane; all lanes must be active).
__device__ __forceinline__ double lane_fetch(double v, int src) {
    const int lo = __builtin_amdgcn_ds_bpermute(src << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Pivot step J of chol_factor16.  Lane (g, a) of the wave holds columns
// 4 g .. 4 g + 3 of row a in t[0..3].  The pivot row's four values for those
// columns come from lane J of the lane's own 16-lane row (DPP broadcast), the
// pivot from lane (J / 4, J), and the lane's own entry in column J from lane
// (J / 4, a).  Every lane runs the step (the broadcasts read other lanes,
// which must be active); rows at or above the pivot take m = 0, which leaves
// them unchanged.
template <int J>
__device__ __forceinline__ void chol_pivot16(double (&t)[4], int g, int a, int K, int n, double tol,
                                             double& myd, double& myy, bool& myck) {
    constexpr int JG = J >> 2, JQ = J & 3;
    const double raw = readlane_d(t[JQ], 16 * JG + J);
    const double colj = lane_fetch(t[JQ], 16 * JG + a);
    const double d = fmax(raw, tol);
    const bool ck = !(raw > tol) && 16 * K + J < n;
    const double y = recip3(d);
    if (a == J) {
        myd = d;
        myy = y;
        myck = ck;
    }
    const bool below = a > J;
    const double m = below ? colj * y : 0.0;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const double u = fma(-m, row_bcast<J>(t[q]), t[q]);
        // column J itself (lane group J / 4, slot J % 4) becomes -m below the pivot
        t[q] = (q == JQ && g == JG) ? (below ? -m : t[q]) : u;
    }
}

template <int... J>
__device__ __forceinline__ void chol_pivots16(double (&t)[4], int g, int a, int K, int n, double tol,
                                              double& myd, double& myy, bool& myck,
                                              std::integer_sequence<int, J...>) {
    (chol_pivot16<J>(t, g, a, K, n, tol, myd, myy, myck), ...);
}

// A: factor diagonal tile K (x: upper triangle = Schur complement, strict
// lower triangle zero).  Row a of the symmetric block is spread over the four
// lane groups (lane (g, a): columns 4 g .. 4 g + 3); entries left of the
// diagonal turn into the E row as their pivot step passes (t = -m), so a
// pivot step is the same FMA t_c -= m t_j[c] for every column c != j in every
// row below the pivot, four per lane.  Row j reaches the lanes by DPP
// broadcasts within each 16-lane row, column j by one cross-row permute.
// (With every lane holding a whole row, 16 FMAs and 16 broadcasts per lane and
// step, a tile took 2.9 us; 32 scalar read-lanes per step instead of the
// broadcasts, 3.2 us.)
__device__ __forceinline__ void chol_factor16(f64x4& x, int K, int n, double tol, int g, int i,
                                              CholShared& sh) {
    const int lane = threadIdx.x & 63, a = lane & 15;
    double (*dt)[17] = sh.dt[K & 1];
#pragma unroll
    for (int r = 0; r < 4; r++) dt[4 * r + g][i] = x[r];
    wave_lds_sync();
    double t[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const int c = 4 * g + q;
        t[q] = c >= a ? dt[a][c] : dt[c][a];
    }
    double myd = 0.0, myy = 0.0;
    bool myck = false;
    chol_pivots16(t, g, a, K, n, tol, myd, myy, myck, std::make_integer_sequence<int, 16>{});
    wave_lds_sync();  // every lane has read dt before it is overwritten
#pragma unroll
    for (int q = 0; q < 4; q++) dt[a][4 * g + q] = t[q];
    if (lane < 16) {
        sh.inv[K & 1][a] = myy;
        sh.d[16 * K + a] = myd;
        sh.dm[16 * K + a] = myck ? 1.0 : 0.0;
        if (myck) sh.clamped = 1;
    }
    wave_lds_sync();
#pragma unroll
    for (int r = 0; r < 4; r++) x[r] = dt[4 * r + g][i];
}

// The lane index read afresh at every call: the compiler would otherwise keep
// the LDS addresses of every tile alive across the loop over tile columns.
__device__ __forceinline__ int fresh_lane() {
    int lane;
    asm volatile("v_mov_b32 %0, %1" : "=v"(lane) : "v"((int)threadIdx.x));
    return lane & 63;
}

// B: tile (K, Q) <- L_K^{-1} X_KQ, published to the tile row.
__device__ __forceinline__ void chol_row_tile(f64x4& x, int Q, int K, CholShared& sh) {
    const int lane = fresh_lane(), g = lane >> 4, i = lane & 15;
    const double (*dt)[17] = sh.dt[K & 1];
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < 4; s++) {
        const int c = 4 * s + g;  // A[i][c] = L_K^{-1}[i][c]; B = rows 4 s .. 4 s + 3 of x
        const double la = c < i ? dt[i][c] : (c == i ? 1.0 : 0.0);
        acc = mfma_f64(la, x[s], acc);
    }
    x = acc;
#pragma unroll
    for (int r = 0; r < 4; r++) sh.w[4 * r + g][16 * Q + i] = x[r];
}

// C: tile (P, Q) below tile row K subtracts sum_k (v_k[a] / d_k) w_k[b].
__device__ __forceinline__ void chol_update_tile(f64x4& x, int P, int Q, int K,
                                                 const CholShared& sh) {
    const int lane = fresh_lane(), g = lane >> 4, i = lane & 15;
    const double* inv = sh.inv[K & 1];
    const double (*dt)[17] = sh.dt[K & 1];
    if (Q == P) {
        // diagonal tile: the upper triangle only (the lower one is E, still zero)
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int k = 4 * s + g;
            acc = mfma_f64(sh.w[k][16 * P + i] * inv[k], sh.w[k][16 * Q + i], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; r++) x[r] -= i >= g + 4 * r ? acc[r] : 0.0;
    } else {
#pragma unroll
        for (int s = 0; s < 4; s++) {
            const int k = 4 * s + g;
            const double ma = sh.w[k][16 * P + i] * inv[k];
            const double wb = Q == K ? (i < k ? dt[k][i] : (i == k ? 1.0 : 0.0))
                                     : sh.w[k][16 * Q + i];
            x = mfma_f64(-ma, wb, x);
        }
    }
}

// Factor the n x n block (n <= 128) whose upper triangle is Gs (leading
// dimension ld): R and R^{-1} of the block into Rout and Rinv (same leading
// dimension), and R also into Rcopy unless it is null; pivots clamped at
// *tolp, an LDS word that the caller may still be writing when it calls (it
// is read after the first barrier, so the tile loads overlap its
// computation); mark[a] = 1 where pivot a was clamped, else 0.  Every thread
// of the work-group calls it; the work-group has at least max(Tn, Tn^2 / 4)
// waves, Tn = ceil(n / 16).
__device__ __forceinline__ void chol_block(const double* __restrict__ Gs, int n,
                                           double* __restrict__ Rout, double* __restrict__ Rinv,
                                           double* __restrict__ Rcopy, int ld,
                                           const double* tolp, int* clamped,
                                           double* __restrict__ mark) {
    __shared__ CholShared sh;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform: tile numbers in SGPRs
    const int W = blockDim.x >> 6;
    const int g = lane >> 4, i = lane & 15;
    const int Tn = (n + 15) >> 4;

    // Tiles of the waves.  Wave t < Tn holds diagonal tile t in slot 0.  When
    // the other waves can hold every off-diagonal tile outside tile row 0,
    // wave t also holds only tile (0, t), which is idle after tile column 0;
    // the wave that factors the next diagonal tile then updates no other tile
    // in that step.  Otherwise the off-diagonal tiles go round robin.
    const bool owners_free = Tn <= 7 && (Tn - 1) * (Tn - 1) <= CH_SLOTS * (W - Tn);
    int tp[CH_SLOTS], tq[CH_SLOTS];
    f64x4 x[CH_SLOTS];
#pragma unroll
    for (int s = 0; s < CH_SLOTS; s++) {
        int P = -1, Q = -1;
        if (owners_free) {
            if (wave < Tn) {
                if (s == 0) P = Q = wave;
                else if (s == 1 && wave > 0) { P = 0; Q = wave; }
            } else {
                const int t = (wave - Tn) + s * (W - Tn);  // rows 1 .. Tn-1, Q != P
                if (t < (Tn - 1) * (Tn - 1)) {
                    P = 1 + t / (Tn - 1);
                    const int c = t - (P - 1) * (Tn - 1);
                    Q = c < P ? c : c + 1;
                }
            }
        } else {
            const int u = wave + s * W;
            if (u < Tn) {
                P = Q = u;
            } else if (u - Tn < Tn * (Tn - 1)) {
                const int t = u - Tn;
                P = t / (Tn - 1);
                const int c = t - P * (Tn - 1);
                Q = c < P ? c : c + 1;
            }
        }
        tp[s] = P;
        tq[s] = Q;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int a = 16 * P + g + 4 * r, b = 16 * Q + i;
            x[s][r] = (P >= 0 && a <= b && b < n) ? Gs[a * ld + b] : 0.0;
        }
    }
    if (tid == 0) sh.clamped = 0;
    __syncthreads();
    const double tol = *tolp;
    // padding rows: a pivot above the clamp threshold, nothing to eliminate
    const double padv = fmax(1.0, 2.0 * tol);
#pragma unroll
    for (int s = 0; s < CH_SLOTS; s++)
        if (tp[s] >= 0 && tp[s] == tq[s])
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int a = 16 * tp[s] + g + 4 * r;
                if (a >= n && a == 16 * tq[s] + i) x[s][r] = padv;
            }
    for (int K = 0; K < Tn; K++) {
        // C of tile column K - 1 (after its B), with A of tile column K: the
        // owner of diagonal tile K updates it first and factors it, then the
        // other tiles are updated
        const bool own = wave == K;
        if (own) {
            if (K > 0) chol_update_tile(x[0], K, K, K - 1, sh);
            chol_factor16(x[0], K, n, tol, g, i, sh);
        }
        if (K > 0) {
            const int Kp = K - 1;
#pragma unroll
            for (int s = 0; s < CH_SLOTS; s++) {
                if (tp[s] <= Kp || (s == 0 && own)) continue;
                // E tiles right of tile column Kp are still zero
                if (tq[s] >= tp[s] || tq[s] <= Kp) chol_update_tile(x[s], tp[s], tq[s], Kp, sh);
            }
        }
        __syncthreads();
        // B. the rest of tile row K
#pragma unroll
        for (int s = 0; s < CH_SLOTS; s++)
            if (tp[s] == K && tq[s] != K) chol_row_tile(x[s], tq[s], K, sh);
        __syncthreads();
    }
    // C of the last tile column has no rows below it
    if (tid == 0 && sh.clamped) *clamped = 1;
    for (int a = tid; a < n; a += blockDim.x) {
        const double sq = sqrt(sh.d[a]);
        sh.sq[a] = sq;
        sh.rs[a] = 1.0 / sq;
        mark[a] = sh.dm[a];
    }
    __syncthreads();
    // R[a][b] = v_a[b] / sqrt(d_a) (b > a), sqrt(d_a) (b = a), 0 below;
    // R^{-1}[b][a] = E[a][b] / sqrt(d_a) (b < a), 1/sqrt(d_a) (b = a), 0 above.
#pragma unroll
    for (int s = 0; s < CH_SLOTS; s++) {
        if (tp[s] < 0) continue;
#pragma unroll
        for (int r = 0; r < 4; r++) {
            const int a = 16 * tp[s] + g + 4 * r, b = 16 * tq[s] + i;
            if (a >= n || b >= n) continue;
            const double rsq = sh.rs[a];
            const double xv = x[s][r];
            const double rv = b > a ? xv * rsq : (b == a ? sh.sq[a] : 0.0);
            Rout[a * ld + b] = rv;
            if (Rcopy) Rcopy[a * ld + b] = rv;
            Rinv[b * ld + a] = b < a ? xv * rsq : (b == a ? rsq : 0.0);
        }
    }
}

// Large l (> 128): the Cholesky runs as a sequence of launches.  Diagonal
// block k (at most 128 wide) is factored by one work-group per problem
// (k_chol_rt, stage k); the block products between the factors run on many
// work-groups, one 16 x 16 output tile each (k_chol_gemm):
//   ROW k : R_kj = (R^{-1}_kk)^T G_kj                  (block row of R)
//   TR  k : G_jj -= R_kj^T R_kj, upper tiles only      (trailing update)
//   TM j,i: Tm = sum_{i<m<=j} R_im R^{-1}_mj
//   RI j,i: R^{-1}_ij = -R^{-1}_ii Tm                  (i = j-1 .. 0)
// Problems of the launch that have no such step return at once.
enum CholGemm : int32_t { CG_ROW = 0, CG_TR = 1, CG_TM = 2, CG_RI = 3 };
constexpr int CG_TILES = 128;  // work-groups per problem (>= the tiles of any product, l <= 264)

__device__ __forceinline__ void chol_blocks(int l, int& nb, int& bs) {
    nb = (l + CRT_LMAX - 1) / CRT_LMAX;
    bs = ((l + nb - 1) / nb + 3) / 4 * 4;
}

__device__ double g_zero_chol[2] = {0.0, 0.0};

// One 16 x 16 tile of C = alpha op(A) op(B) + beta C (op(A)[i][k] is
// A[k lda + i] when ta, else A[i lda + k]; likewise op(B)); the four waves
// take every fourth K step of 4 and their partial tiles are added in LDS in
// wave order.  Loads are unconditional (an address select: operands outside
// the matrices come from a zero word).
__device__ __forceinline__ void gemm_tile(int ti, int tj, int M, int N, int K, double alpha,
                                          const double* __restrict__ A, int lda, bool ta,
                                          const double* __restrict__ B, int ldb, bool tb,
                                          double beta, double* __restrict__ C, int ldc) {
    __shared__ double part[3][4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int ar = 16 * ti + li, bc = 16 * tj + li;
    const bool okr = ar < M, okc = bc < N;
    gdouble* ap = as_global(A) + (ta ? ar : ar * lda);
    gdouble* bp = as_global(B) + (tb ? bc * ldb : bc);
    const int as = ta ? lda : 1, bs = tb ? 1 : ldb;
    gdouble* zw = as_global(g_zero_chol);
    f64x4 acc = f64x4{0.0, 0.0, 0.0, 0.0};
    const int ns = (K + 3) / 4;  // K steps of 4
    for (int s0 = wave; s0 < ns; s0 += 16) {  // four steps per wave per round
        double av[4], bv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int k = 4 * (s0 + 4 * u) + lg;
            const bool ok = k < K;
            av[u] = *((ok && okr) ? ap + k * as : zw);
            bv[u] = *((ok && okc) ? bp + k * bs : zw);
        }
#pragma unroll
        for (int u = 0; u < 4; u++) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
    }
    if (wave > 0)
#pragma unroll
        for (int e = 0; e < 4; e++) part[wave - 1][e][lane] = acc[e];
    __syncthreads();
    if (wave != 0) return;
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int r = 16 * ti + lg + 4 * e;
        if (r < M && okc) {
            const double v = ((acc[e] + part[0][e][lane]) + part[1][e][lane]) + part[2][e][lane];
            double* c = C + r * ldc + bc;
            *c = beta == 0.0 ? alpha * v : fma(alpha, v, beta * *c);
        }
    }
}

__global__ __launch_bounds__(256) void k_chol_gemm(const Prob* __restrict__ probs,
                                                   const int32_t* __restrict__ pidx, int cnt,
                                                   int mode, int iter, int type, int a, int b) {
    const int pi = blockIdx.x / CG_TILES, tile = blockIdx.x - pi * CG_TILES;
    if (pi >= cnt) return;
    const Prob& P = probs[pidx[pi]];
    if (iter >= 0 && iter > P.q) return;
    if (mode == CHOL_SECOND && !second_pass(P, iter)) return;
    const int l = P.l;
    int nb, bs;
    chol_blocks(l, nb, bs);
    double* __restrict__ G = P.G;
    double* __restrict__ R = P.R;
    double* __restrict__ Ri = P.Rinv;
    double* __restrict__ Tm = P.Qt;
    int M, N, K;
    double alpha = 1.0, beta = 0.0;
    const double* Am;
    const double* Bm;
    double* Cm;
    bool ta = false;
    if (type == CG_ROW || type == CG_TR) {
        const int k = a;
        if (k >= nb - 1) return;
        const int o = k * bs, o2 = o + bs, rest = l - o2;
        K = bs;
        if (type == CG_ROW) {
            M = bs; N = rest;
            Am = Ri + o * l + o; ta = true;
            Bm = G + o * l + o2;
            Cm = R + o * l + o2;
        } else {
            M = rest; N = rest; alpha = -1.0; beta = 1.0;
            Am = R + o * l + o2; ta = true;
            Bm = R + o * l + o2;
            Cm = G + o2 * l + o2;
        }
    } else {
        const int j = a, i = b;
        if (j >= nb) return;
        const int oj = j * bs, nj = min(bs, l - oj), oi = i * bs, ni = bs;
        M = ni; N = nj;
        if (type == CG_TM) {
            K = oj + nj - (oi + ni);
            Am = R + oi * l + oi + ni;
            Bm = Ri + (oi + ni) * l + oj;
            Cm = Tm;
            // R is final from here on: the first such step copies it for the
            // accumulated factor of the pass
            if (j == 1 && mode == CHOL_FIRST)
                for (int e = tile * 256 + threadIdx.x; e < l * l; e += CG_TILES * 256) P.Racc[e] = R[e];
        } else {
            K = ni; alpha = -1.0;
            Am = Ri + oi * l + oi;
            Bm = Tm;
            Cm = Ri + oi * l + oj;
        }
    }
    const int nt = (N + 15) / 16;
    const int ti = tile / nt, tj = tile - ti * nt;
    if (ti >= (M + 15) / 16) return;
    if (type == CG_TR && tj < ti) return;  // the lower triangle of G is never read
    gemm_tile(ti, tj, M, N, K, alpha, Am, l, ta, Bm, l, false, beta, Cm, l);
}

// The Cholesky stage: G = R^T R and R^{-1}.  stage < 0 (l <= 128 for the
// whole launch): one block factor in registers.  stage = k (l > 128 in the
// launch): diagonal block k of nb = ceil(l / 128) blocks, right looking; the
// products between the factors are the k_chol_gemm launches above.  The pivot
// threshold tol is taken from G before the first block and kept in rep[96].
__global__ __launch_bounds__(CRT_THREADS) void k_chol_rt(const Prob* __restrict__ probs,
                                                        const int32_t* __restrict__ pidx,
                                                        const int32_t* __restrict__ toff, int cnt,
                                                        int mode, int iter, int stage) {
    __shared__ double s_tol;
    __shared__ int s_clamped_any;
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    if (iter >= 0 && iter > P.q) return;
    if (mode == CHOL_SECOND && !second_pass(P, iter)) return;
    const int l = P.l;
    const int tid = threadIdx.x, nth = blockDim.x;
    int nb, bs;
    chol_blocks(l, nb, bs);
    const int k = stage < 0 ? 0 : stage;
    if (k >= nb) return;
    double* __restrict__ G = P.G;
    double* __restrict__ R = P.R;
    double* __restrict__ Ri = P.Rinv;
    if (tid == 0) s_clamped_any = 0;
    if (k == 0) {
        if (tid < 64) {
            // the diagonal's loads all issued before the first is used
            constexpr int NU = (LMAX + 63) / 64;
            double dv[NU];
#pragma unroll
            for (int u = 0; u < NU; u++) {
                const int i = tid + 64 * u;
                dv[u] = i < l ? fabs(G[i * l + i]) : 0.0;
            }
            double mx = 0.0;
#pragma unroll
            for (int u = 0; u < NU; u++) mx = fmax(mx, dv[u]);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
            if (tid == 0) {
                const double t = (double)l * 0x1.0p-52 * mx;
                s_tol = t > 0.0 ? t : 0x1.0p-1000;
                P.rep[96] = s_tol;
            }
        }
        // blocks of R and R^{-1} below the diagonal blocks are zero
        if (nb > 1)
            for (int a = tid >> 6; a < l; a += nth >> 6)
                for (int b = tid & 63; b < (a / bs) * bs; b += 64) {
                    R[a * l + b] = 0.0;
                    Ri[a * l + b] = 0.0;
                }
    } else if (tid == 0) {
        s_tol = P.rep[96];
    }
    // no barrier here: chol_block reads s_tol after its first one
    const int o = k * bs, n = min(bs, l - o);
    // one diagonal block: R of the first CholeskyQR pass is also kept in Racc
    double* Rc = (nb == 1 && mode == CHOL_FIRST) ? P.Racc : nullptr;
    chol_block(G + o * l + o, n, R + o * l + o, Ri + o * l + o, Rc, l, &s_tol, &s_clamped_any,
               P.tau + o);
    __syncthreads();
    if (tid == 0 && s_clamped_any) atomicOr(P.flags, FLAG_RANK_DEF);
}

hipError_t launch_chol(const LaunchGroup& g, int mode, int lmax, int iter, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    if (lmax <= CRT_LMAX) {
        // one wave per 16 x 16 tile of the block, at most CH_SLOTS tiles per
        // wave (16 waves for blocks of 113 .. 128)
        const int tn = (lmax + 15) / 16;
        const int threads = 64 * std::min(16, tn * tn);
        hipLaunchKernelGGL(k_chol_rt, dim3(g.blocks), dim3(threads), 0, s, g.probs, g.pidx,
                           g.toff, g.count, mode, iter, -1);
        return hipGetLastError();
    }
    const int nbmax = (lmax + CRT_LMAX - 1) / CRT_LMAX;
    auto gemm = [&](int type, int a, int b) {
        hipLaunchKernelGGL(k_chol_gemm, dim3(g.count * CG_TILES), dim3(256), 0, s, g.probs,
                           g.pidx, g.count, mode, iter, type, a, b);
        return hipGetLastError();
    };
    for (int k = 0; k < nbmax; k++) {
        hipLaunchKernelGGL(k_chol_rt, dim3(g.blocks), dim3(CRT_THREADS), 0, s, g.probs, g.pidx,
                           g.toff, g.count, mode, iter, k);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if (k + 1 < nbmax) {
            if ((e = gemm(CG_ROW, k, 0)) != hipSuccess) return e;
            if ((e = gemm(CG_TR, k, 0)) != hipSuccess) return e;
        }
    }
    for (int j = 1; j < nbmax; j++)
        for (int i = j - 1; i >= 0; i--) {
            hipError_t e = gemm(CG_TM, j, i);
            if (e != hipSuccess) return e;
            if ((e = gemm(CG_RI, j, i)) != hipSuccess) return e;
        }
    return hipSuccess;
}

// R2 = R' R (both upper triangular): the R factor of Y2 after both
// CholeskyQR passes (dst 0), or R1 of the last Y1 for eq. (18) (dst 1).  One
// block per 16 x 16 output tile.
__global__ __launch_bounds__(256) void k_r2(const Prob* __restrict__ probs,
                                            const int32_t* __restrict__ pidx,
                                            const int32_t* __restrict__ toff, int cnt, int iter,
                                            int dst) {
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    if (iter != P.q) return;  // only the R factors of the last Y1, Y2 are used
    if (dst == 1 && P.mmode != M_APPROX) return;
    double* const out = dst == 1 ? P.R1 : P.R2;
    // Rows 16 ta .. 16 ta + 15 of R and columns 16 tb .. 16 tb + 15 of Racc
    // through LDS: every load of the block is in flight at once.
    __shared__ double sa[16][LPMAX + 1];
    __shared__ double sb[LPMAX][17];
    const int l = P.l, nt = P.lp / 16;
    const int ta = local / nt, tb = local % nt;
    for (int e = threadIdx.x; e < 16 * l; e += 256) {
        const int r = e / l, c = e - r * l;
        sa[r][c] = 16 * ta + r < l ? P.R[(16 * ta + r) * l + c] : 0.0;
    }
    for (int e = threadIdx.x; e < 16 * l; e += 256) {
        const int t = e >> 4, j = e & 15;
        sb[t][j] = 16 * tb + j < l ? P.Racc[t * l + 16 * tb + j] : 0.0;
    }
    __syncthreads();
    const int a = ta * 16 + (threadIdx.x >> 4), b = tb * 16 + (threadIdx.x & 15);
    if (a >= l || b >= l) return;
    const double* Ra = sa[threadIdx.x >> 4];
    const int jb = threadIdx.x & 15;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int t = a;
    for (; t + 3 <= b; t += 4) {
        s0 += Ra[t] * sb[t][jb];
        s1 += Ra[t + 1] * sb[t + 1][jb];
        s2 += Ra[t + 2] * sb[t + 2][jb];
        s3 += Ra[t + 3] * sb[t + 3][jb];
    }
    for (; t <= b; t++) s0 += Ra[t] * sb[t][jb];
    out[a * l + b] = (s0 + s1) + (s2 + s3);
}

hipError_t launch_r2(const LaunchGroup& g, int iter, int dst, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_r2, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count, iter,
                       dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Eq. (18): D = Q1^T Y1 (Q2^T X)^+ = R1 G^-1 with G = Q2^T X (l x l, full
// rank for a full-rank sketch).  The QRCP reads M^T, so the kernel solves
// G^T D^T = R1^T: Gauss-Jordan elimination with partial pivoting (largest
// |entry| of the column, lowest row on ties) on [G^T | R1^T], one block per
// problem, the l x 2l work matrix in the problem's Gram partials (L2).  The
// result D^T goes to Mx.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_dapprox(const Prob* __restrict__ probs,
                                                  const int32_t* __restrict__ pidx,
                                                  const int32_t* __restrict__ toff, int cnt) {
    __shared__ unsigned long long s_key;
    __shared__ double s_prow[2 * LMAX];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    if (P.mmode != M_APPROX) return;
    const int l = P.l, w2 = 2 * l, tid = threadIdx.x;
    double* __restrict__ W = P.gpart;  // [l][2l]
    for (int e = tid; e < l * w2; e += blockDim.x) {
        const int r = e / w2, c = e - r * w2;
        W[e] = c < l ? P.G[c * l + r] : P.R1[(c - l) * l + r];  // G^T | R1^T
    }
    __syncthreads();
    for (int j = 0; j < l; j++) {
        if (tid == 0) s_key = 0ull;
        __syncthreads();
        // pivot: largest |W[i][j]| over rows i >= j, lowest row on ties
        for (int i = j + tid; i < l; i += blockDim.x) {
            const double v = fabs(W[i * w2 + j]);
            const unsigned long long key =
                ((unsigned long long)__double_as_longlong(v) & ~0x3FFull) | (unsigned long long)(1023 - i);
            atomicMax(&s_key, key);
        }
        __syncthreads();
        const int pr = 1023 - (int)(s_key & 0x3FFull);
        // swap rows j and pr, scale the pivot row
        const double piv = W[pr * w2 + j];
        const double inv = piv != 0.0 ? 1.0 / piv : 0.0;
        for (int c = tid; c < w2; c += blockDim.x) {
            const double a = W[pr * w2 + c], b = W[j * w2 + c];
            const double sa = a * inv;
            s_prow[c] = sa;
            W[pr * w2 + c] = b;
            W[j * w2 + c] = sa;
        }
        __syncthreads();
        // eliminate column j from every other row
        for (int e = tid; e < l * w2; e += blockDim.x) {
            const int r = e / w2, c = e - r * w2;
            if (r == j || c < j) continue;
            const double f = W[r * w2 + j];
            if (c == j) continue;
            W[e] = fma(-f, s_prow[c], W[e]);
        }
        __syncthreads();
        for (int r = tid; r < l; r += blockDim.x)
            if (r != j) W[r * w2 + j] = 0.0;
        __syncthreads();
    }
    for (int e = tid; e < l * l; e += blockDim.x) {
        const int r = e / l, c = e - r * l;
        P.Mx[e] = W[r * w2 + l + c];  // D^T
    }
}

hipError_t launch_dapprox(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dapprox, dim3(g.blocks), dim3(1024), 0, s, g.probs, g.pidx, g.toff,
                       g.count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pivot keys of the QRCP: during the trailing update each column posts
//   key = (bits of its squared norm with the 9 low mantissa bits cleared) |
//   (511 - position) with a 64-bit LDS atomicMax; for non-negative doubles
// the bit pattern orders like the value, so the winner is the largest norm
// and, among norms equal to 43 bits, the lowest position.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long qr_key(double nn, int c) {
    return (__double_as_longlong(nn) & ~0x1FFull) | (unsigned long long)(511 - c);
}

__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_mov<0xB1>(v);  // quad_perm 1,0,3,2
    v += dpp_mov<0x4E>(v);  // quad_perm 2,3,0,1
    return v;
}

// ---------------------------------------------------------------------------
// QRCP of M = R2^T for l > 224, first part: the first l - 224 steps (one
// block of up to 1024 threads per problem); k_qrcp_hy takes the remaining 224
// steps on the trailing 224 x 224 block (rows >= l - 224, the columns not yet
// pivoted, in their original order so that ties still go to the lowest
// column index).
//   M does not fit the registers of one work-group, so it stays in a global
//   work array W (l x l, row-major, in P.R, which is free once R2 is formed;
//   it stays in L2).  Four lanes own a column, lane t the rows i = 4 u + t
//   (a lane group takes a second column when l > 256).
//   Columns stay in place and a retired column is never written again, so W
//   itself keeps every pivot column as it was at its step.  Step j:
//     1. the pivot column goes into an LDS buffer (one element per thread),
//        and every lane forms beta, tau and scale = 1/(alpha - beta) as in
//        the register-resident kernel;
//     2. every remaining column: w = tau (col_j + scale sum_{i>j} raw_i col_i)
//        over its rows at and below j (loads in batches of 64 rows, four
//        partial sums per lane, a quad sum), then col -= w v, stored back, and
//        the squared norm below j posted as the next key.
//   Rows above j are skipped in batches (uniform branches).  At the end it
//   writes what its steps fix: tau, signs, perm and the reflectors of steps
//   < l - 224, the block of T on those rows and columns, and the map from the
//   trailing block's columns to the columns of M (int32, in P.Racc, free
//   after R2 = R' R).  W keeps the rows above the trailing block, which
//   k_qrcp_hy reads for the rest of T.
// ---------------------------------------------------------------------------
constexpr int QST_THREADS = 1024;
constexpr int QST_COLS = QST_THREADS / 4;  // columns per pass over the lane groups

__global__ __launch_bounds__(QST_THREADS) void k_qrcp_st(const Prob* __restrict__ probs,
                                                        const int32_t* __restrict__ pidx,
                                                        const int32_t* __restrict__ toff, int cnt) {
    constexpr int UB = 8;  // u per batch (32 rows)
    __shared__ double s_piv[LMAX];
    __shared__ double s_nrm[LMAX];
    __shared__ double s_tau[LMAX], s_scale[LMAX], s_beta[LMAX];
    __shared__ int s_perm[LMAX];
    __shared__ unsigned char s_ret[LMAX];  // column pivoted
    __shared__ int s_wcnt[QST_THREADS / 64];
    __shared__ unsigned long long s_key[2];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    const int l = P.l;
    if (l <= QHY_LMAX) return;  // k_qrcp_rt, k_qrcp_hy
    const int jend = l - QHY_LMAX;  // steps taken here
    const int tid = threadIdx.x, t = tid & 3;
    const int ngroups = blockDim.x >> 2;
    // a lane group owns column tid/4 and, when l exceeds the group count,
    // column tid/4 + ngroups as well
    const int ncs = (l + ngroups - 1) / ngroups;  // 1 or 2
    const int rpt = (l + 3) >> 2;       // rows per lane
    const int nb = (rpt + UB - 1) / UB; // batches per lane
    double* __restrict__ W = P.R;
    const double* __restrict__ R2 = P.msrc;  // M^T: R2 (M = R2^T), or Mx

    // W = M = R2^T, and the squared column norms
    if (tid < 2) s_key[tid] = 0ull;
    for (int c = tid; c < l; c += blockDim.x) s_ret[c] = 0;
    __syncthreads();
    for (int cs = 0; cs < ncs; cs++) {
        const int c = (tid >> 2) + cs * ngroups;
        double nn = 0.0;
        for (int u = 0; u < rpt; u++) {
            const int i = 4 * u + t;
            if (c < l && i < l) {
                const double v = R2[c * l + i];
                W[i * l + c] = v;
                nn = fma(v, v, nn);
            }
        }
        nn = quad_sum(nn);
        if (c < l && t == 0) {
            s_nrm[c] = nn;
            atomicMax(&s_key[0], qr_key(nn, c));
        }
    }
    bool active[2] = {(tid >> 2) < l, (tid >> 2) + ngroups < l};
    __syncthreads();

    for (int j = 0; j < jend; j++) {
        const unsigned long long key = s_key[j & 1];
        const int p = 511 - (int)(key & 0x1FFull);
        // the pivot column into LDS, one element per thread (one round trip);
        // the key slot of the next step (last read in step j - 1) is cleared
        // before the barrier, so no posting can precede the clearing
        if (tid < l) s_piv[tid] = W[tid * l + p];
        if (tid == 0) s_key[(j + 1) & 1] = 0ull;
        __syncthreads();
        // every lane forms the reflector's scalars (no further barrier)
        const double alpha = s_piv[j];
        const double ss = s_nrm[p];  // sum over rows >= j of column p squared
        double tau = 0.0, beta = alpha, scale = 1.0;
        if (ss > 0.0) {
            const double h = 0.5 * ss;
            double y = __builtin_amdgcn_rsq(ss);
#pragma unroll
            for (int it = 0; it < 2; it++) y = fma(y, fma(-h * y, y, 0.5), y);
            const double xnorm = ss * y;
            const double sg = alpha >= 0.0 ? -1.0 : 1.0;
            beta = sg * xnorm;
            scale = recip_nr(alpha - beta);
            tau = (beta - alpha) * (sg * y);
        }
        if (tid == 0) {
            s_tau[j] = tau;
            s_scale[j] = scale;
            s_beta[j] = beta;
            s_perm[j] = p;
            s_ret[p] = 1;
        }
        for (int cs = 0; cs < ncs; cs++) {
            const int c = (tid >> 2) + cs * ngroups;
            if (c == p) active[cs] = false;
            if (!active[cs]) continue;
            // dot pass: two batches of rows per round trip
            double d4[4] = {0.0, 0.0, 0.0, 0.0};
            for (int q = 0; q < nb; q += 2) {
                if (4 * UB * q + 8 * UB - 1 < j) continue;  // both batches above j
                double cv[2 * UB], pv[2 * UB];
#pragma unroll
                for (int e = 0; e < 2 * UB; e++) {
                    const int i = min(4 * (UB * q + e) + t, l - 1);
                    cv[e] = W[i * l + c];
                    pv[e] = s_piv[i];
                }
#pragma unroll
                for (int e = 0; e < 2 * UB; e++) {
                    const int i = 4 * (UB * q + e) + t;
                    const double v = (i < l && i > j) ? pv[e] * scale : (i == j ? 1.0 : 0.0);
                    d4[e & 3] = fma(v, cv[e], d4[e & 3]);
                }
            }
            const double w = tau * quad_sum((d4[0] + d4[1]) + (d4[2] + d4[3]));
            double n4[4] = {0.0, 0.0, 0.0, 0.0};
            for (int q = 0; q < nb; q += 2) {
                if (4 * UB * q + 8 * UB - 1 < j) continue;
                double cv[2 * UB], pv[2 * UB];
#pragma unroll
                for (int e = 0; e < 2 * UB; e++) {
                    const int i = min(4 * (UB * q + e) + t, l - 1);
                    cv[e] = W[i * l + c];
                    pv[e] = s_piv[i];
                }
#pragma unroll
                for (int e = 0; e < 2 * UB; e++) {
                    const int i = 4 * (UB * q + e) + t;
                    if (i < l && i >= j) {
                        const double v = i > j ? pv[e] * scale : 1.0;
                        const double x = fma(-w, v, cv[e]);
                        W[i * l + c] = x;
                        if (i > j) n4[e & 3] = fma(x, x, n4[e & 3]);
                    }
                }
            }
            const double n = quad_sum((n4[0] + n4[1]) + (n4[2] + n4[3]));
            if (t == 0) {
                s_nrm[c] = n;
                atomicMax(&s_key[(j + 1) & 1], qr_key(n, c));
            }
        }
        __syncthreads();
    }

    // Outputs of the steps taken here: column perm[b] of W holds raw_b
    // (frozen since step b); T on rows and columns < jend, reflector rows < jend.
    for (int e = tid; e < jend * l; e += blockDim.x) {
        const int a = e / l, b = e % l;
        if (b < jend) {
            double tv = 0.0;
            if (a < b) tv = W[a * l + s_perm[b]] * (s_beta[a] < 0.0 ? -1.0 : 1.0);
            else if (a == b) tv = fabs(s_beta[a]);
            P.T[a * l + b] = tv;
        }
        // reflector a, component b
        double vv = 0.0;
        if (b == a) vv = 1.0;
        else if (b > a) vv = W[b * l + s_perm[a]] * s_scale[a];
        P.Qt[e] = vv;
    }
    for (int j = tid; j < jend; j += blockDim.x) {
        P.tau[j] = s_tau[j];
        P.tau[LMAX + j] = s_beta[j] < 0.0 ? -1.0 : 1.0;
        P.perm[j] = s_perm[j];
    }
    // the columns left for the trailing block, in increasing order
    const int lane = tid & 63, wave = tid >> 6;
    const bool act = tid < l && !s_ret[tid];
    const unsigned long long bal = __ballot(act);
    if (lane == 0) s_wcnt[wave] = __popcll(bal);
    __syncthreads();
    int off = __popcll(bal & ((1ull << lane) - 1ull));
    for (int w = 0; w < wave; w++) off += s_wcnt[w];
    if (act) ((int32_t*)P.Racc)[off] = tid;
}

// ---------------------------------------------------------------------------
// The same first l - 224 steps on QMB_G work-groups per problem, the trailing
// matrix held in registers (the alternative to k_qrcp_st for launches small
// enough that every group of every problem is resident at once).  Group y
// owns the columns c = y (mod QMB_G): four lanes a column, lane t the rows
// i = 4 u + t.  Step j: each group posts its candidate -- the key of its
// largest trailing norm, that norm and the whole column -- into a
// double-buffered slot (in the Gram array, free until the QRCP ends), the
// groups meet at a counter in the problem's flag words, and every group then
// reads all candidates in one round trip, takes the largest key as the pivot
// (the same choice in every group), forms the reflector from the pivot column
// and applies it to its own active columns, leaving the pivot column frozen
// with its raw values in its owner's registers (the column k_qrcp_st leaves
// in its work array).  At the end every group writes its columns to the work
// array, the T entries and the reflector row of each pivot it owns; group 0
// writes tau, the signs, perm and the column map for k_qrcp_hy.
// A wait past its spin bound sets FLAG_SYNC_TIMEOUT and the group leaves the
// loop; the last group out resets the counter words to zero.
// ---------------------------------------------------------------------------
constexpr int QMB_THREADS = 256;
constexpr int QMB_COLS = QMB_THREADS / 4;                 // columns per group
constexpr int QMB_G = (LMAX + QMB_COLS - 1) / QMB_COLS;   // groups per problem
constexpr int QMB_RPT = (LMAX + 3) / 4;                   // register rows per lane
constexpr int QMB_ST = (QMB_RPT + 1) / 2 * 2;             // LDS doubles per lane row of v
constexpr int QMB_SLOT = LMAX + 8;  // doubles per candidate: column, key, norm
constexpr int QMB_MAX_PROBS = 48;   // problems per launch
constexpr int QMB_SPIN = 1 << 21;   // polls before a wait gives up (seconds)
static_assert(2 * QMB_G * QMB_SLOT <= (QHY_LMAX + 1) * (QHY_LMAX + 1), "slots fit the Gram array");
static_assert(LMAX <= 2 * QMB_THREADS && QMB_RPT % 2 == 0, "two column entries per thread");
static_assert(QMB_THREADS > LMAX - QHY_LMAX, "rows past the first thread row are below every j");

// Arrival at the step barrier of a problem's groups: every thread's stores
// are released at agent scope, thread 0 counts the group in and polls until
// `target` groups have arrived, then every thread acquires.  False when the
// wait gave up.
__device__ __forceinline__ bool qmb_sync(int32_t* ctr, int target, int* s_ok) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(ctr, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        int ok = 1, spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > QMB_SPIN) {
                ok = 0;
                break;
            }
        }
        *s_ok = ok;
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return *s_ok != 0;
}

__global__ __launch_bounds__(QMB_THREADS) void k_qrcp_mb(const Prob* __restrict__ probs,
                                                        const int32_t* __restrict__ pidx,
                                                        const int32_t* __restrict__ toff, int cnt) {
    __shared__ __align__(16) double s_v[4 * QMB_ST];  // reflector vector, [t][u]
    __shared__ double s_tau[LMAX], s_scale[LMAX], s_beta[LMAX];
    __shared__ int s_perm[LMAX];
    __shared__ unsigned char s_ret[LMAX];  // column pivoted
    __shared__ int s_wcnt[QMB_THREADS / 64];
    __shared__ unsigned long long s_key[2];
    __shared__ int s_ok;
    const int y = blockIdx.x % QMB_G;
    const Prob& P = probs[pidx[find_group(toff, cnt, blockIdx.x / QMB_G)]];
    const int l = P.l;
    if (l <= QHY_LMAX) return;  // k_qrcp_rt, k_qrcp_hy
    const int jend = l - QHY_LMAX;
    const int tid = threadIdx.x, t = tid & 3;
    const int c = y + QMB_G * (tid >> 2);  // this lane group's column
    const bool mine = c < l;
    double* __restrict__ slots = P.G;
    int32_t* ctr = P.flags + 4;  // [0] arrivals, [1] exits
    const double* __restrict__ R2 = P.msrc;  // M^T: R2 (M = R2^T), or Mx

    double col[QMB_RPT];
    double nn = 0.0;
#pragma unroll
    for (int u = 0; u < QMB_RPT; u++) {
        const int i = 4 * u + t;
        col[u] = (mine && i < l) ? R2[c * l + i] : 0.0;
        nn = fma(col[u], col[u], nn);
    }
    nn = quad_sum(nn);
    for (int i = tid; i < LMAX; i += QMB_THREADS) s_ret[i] = 0;
    if (tid < 2) s_key[tid] = 0ull;
    __syncthreads();
    if (mine && t == 0) atomicMax(&s_key[0], qr_key(nn, c));
    bool active = mine;
    int mystep = -1;  // the step that pivoted this column
    bool ok = true;

    for (int j = 0; j < jend; j++) {
        const int par = j & 1;
        __syncthreads();  // s_key[par] complete, s_piv free
        // post this group's candidate for step j
        {
            const unsigned long long bk = s_key[par];
            double* sl = slots + (par * QMB_G + y) * QMB_SLOT;
            if (active && qr_key(nn, c) == bk) {
#pragma unroll
                for (int u = 0; u < QMB_RPT; u++) sl[4 * u + t] = col[u];  // zeros past l
                if (t == 0) sl[LMAX + 1] = nn;
            }
            if (tid == 0) {
                reinterpret_cast<unsigned long long*>(sl)[LMAX] = bk;
                s_key[par ^ 1] = 0ull;  // last read above; filled after the barrier
            }
        }
        if (!qmb_sync(ctr, QMB_G * (j + 1), &s_ok)) {
            ok = false;
            break;
        }
        // every candidate in one round trip; the largest key wins
        const double* sl = slots + par * QMB_G * QMB_SLOT;
        unsigned long long kk[QMB_G];
        double cn[QMB_G], ca[QMB_G], c0[QMB_G], c1[QMB_G];
#pragma unroll
        for (int g = 0; g < QMB_G; g++) {
            kk[g] = reinterpret_cast<const unsigned long long*>(sl + g * QMB_SLOT)[LMAX];
            cn[g] = sl[g * QMB_SLOT + LMAX + 1];
            ca[g] = sl[g * QMB_SLOT + j];
            c0[g] = tid < l ? sl[g * QMB_SLOT + tid] : 0.0;
            c1[g] = tid + QMB_THREADS < l ? sl[g * QMB_SLOT + tid + QMB_THREADS] : 0.0;
        }
        unsigned long long key = kk[0];
        double ss = cn[0], alpha = ca[0], p0 = c0[0], p1 = c1[0];
#pragma unroll
        for (int g = 1; g < QMB_G; g++) {
            if (kk[g] > key) {
                key = kk[g];
                ss = cn[g];  // sum over rows >= j of the pivot column squared
                alpha = ca[g];
                p0 = c0[g];
                p1 = c1[g];
            }
        }
        const int p = 511 - (int)(key & 0x1FFull);
        // the reflector's scalars (every lane, as in k_qrcp_st)
        double tau = 0.0, beta = alpha, scale = 1.0;
        if (ss > 0.0) {
            const double h = 0.5 * ss;
            double yr = __builtin_amdgcn_rsq(ss);
#pragma unroll
            for (int it = 0; it < 2; it++) yr = fma(yr, fma(-h * yr, yr, 0.5), yr);
            const double xnorm = ss * yr;
            const double sg = alpha >= 0.0 ? -1.0 : 1.0;
            beta = sg * xnorm;
            scale = recip_nr(alpha - beta);
            tau = (beta - alpha) * (sg * yr);
        }
        // v (v_j = 1, scale piv_i below j, zero above j and past l) into LDS,
        // lane-row major: lane t reads its rows u, u + 1 as one 16-byte word
        s_v[(tid & 3) * QMB_ST + (tid >> 2)] = tid > j ? p0 * scale : (tid == j ? 1.0 : 0.0);
        if (tid + QMB_THREADS < 4 * QMB_RPT) {
            const int i = tid + QMB_THREADS;
            s_v[(i & 3) * QMB_ST + (i >> 2)] = p1 * scale;  // i > 255 >= jend > j
        }
        if (tid == 0) {
            s_tau[j] = tau;
            s_scale[j] = scale;
            s_beta[j] = beta;
            s_perm[j] = p;
            s_ret[p] = 1;
        }
        __syncthreads();
        if (active && c == p) {
            active = false;
            mystep = j;
        }
        if (active) {
            // w = tau v^T col (the zeros of v above j included), col -= w v,
            // and the trailing norm below j; register rows wholly above j are
            // skipped in blocks of 8
            const double* pv = s_v + t * QMB_ST;
            double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ub = 0; ub < QMB_RPT; ub += 8) {
                if (4 * (ub + 8) <= j) continue;
#pragma unroll
                for (int u = ub; u < ub + 8 && u < QMB_RPT; u += 2) {
                    const double2 r = *reinterpret_cast<const double2*>(pv + u);
                    d4[u & 3] = fma(r.x, col[u], d4[u & 3]);
                    d4[(u + 1) & 3] = fma(r.y, col[u + 1], d4[(u + 1) & 3]);
                }
            }
            const double w = tau * quad_sum((d4[0] + d4[1]) + (d4[2] + d4[3]));
            double n4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ub = 0; ub < QMB_RPT; ub += 8) {
                if (4 * (ub + 8) <= j) continue;
#pragma unroll
                for (int u = ub; u < ub + 8 && u < QMB_RPT; u += 2) {
                    const double2 r = *reinterpret_cast<const double2*>(pv + u);
                    col[u] = fma(-w, r.x, col[u]);
                    col[u + 1] = fma(-w, r.y, col[u + 1]);
                    const double x0 = 4 * u + t > j ? col[u] : 0.0;
                    const double x1 = 4 * u + 4 + t > j ? col[u + 1] : 0.0;
                    n4[u & 3] = fma(x0, x0, n4[u & 3]);
                    n4[(u + 1) & 3] = fma(x1, x1, n4[(u + 1) & 3]);
                }
            }
            nn = quad_sum((n4[0] + n4[1]) + (n4[2] + n4[3]));
            if (t == 0) atomicMax(&s_key[par ^ 1], qr_key(nn, c));
        }
    }

    if (ok) {
        __syncthreads();  // s_tau, s_scale, s_beta, s_perm, s_ret complete
        double* __restrict__ W = P.R;
        if (mine) {
#pragma unroll
            for (int u = 0; u < QMB_RPT; u++) {
                const int i = 4 * u + t;
                if (i < l) W[i * l + c] = col[u];
            }
        }
        if (mystep >= 0) {
            // column b of T (rows < jend) and reflector b, from the frozen pivot column
            const int b = mystep;
            const double sc = s_scale[b];
#pragma unroll
            for (int u = 0; u < QMB_RPT; u++) {
                const int a = 4 * u + t;
                if (a < jend)
                    P.T[a * l + b] = a < b ? col[u] * (s_beta[a] < 0.0 ? -1.0 : 1.0)
                                           : (a == b ? fabs(s_beta[b]) : 0.0);
                if (a < l) P.Qt[b * l + a] = a == b ? 1.0 : (a > b ? col[u] * sc : 0.0);
            }
        }
        if (y == 0) {
            for (int jj = tid; jj < jend; jj += QMB_THREADS) {
                P.tau[jj] = s_tau[jj];
                P.tau[LMAX + jj] = s_beta[jj] < 0.0 ? -1.0 : 1.0;
                P.perm[jj] = s_perm[jj];
            }
            // the columns left for the trailing block, in increasing order
            const int lane = tid & 63, wave = tid >> 6;
            int base = 0;
            for (int c0 = 0; c0 < l; c0 += QMB_THREADS) {
                const int cc = c0 + tid;
                const bool act = cc < l && !s_ret[cc];
                const unsigned long long bal = __ballot(act);
                if (lane == 0) s_wcnt[wave] = __popcll(bal);
                __syncthreads();
                int off = base + __popcll(bal & ((1ull << lane) - 1ull));
                for (int w = 0; w < wave; w++) off += s_wcnt[w];
                if (act) ((int32_t*)P.Racc)[off] = cc;
                for (int w = 0; w < QMB_THREADS / 64; w++) base += s_wcnt[w];
                __syncthreads();
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        if (!ok) atomicOr(P.flags, FLAG_SYNC_TIMEOUT);
        const int e = __hip_atomic_fetch_add(ctr + 1, 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (e == QMB_G - 1) {  // every group is past its last wait
            __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(ctr + 1, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// ---------------------------------------------------------------------------
// QRCP of M = R2^T for 128 < l <= 224: registers and LDS (one block of 4 l
// threads per problem).  Four lanes own a column, lane t the rows
// i = 4 u + t; the first LRC rows per lane (u < LRC) live in LDS and the next
// QHY_RR in registers, so that once the steps pass row 4 LRC the LDS rows are
// above j and no step touches them again (thread-major with an odd stride,
// so that the row offsets are immediates and 8-byte reads are free of bank
// conflicts; LRC is the launch's LDS row count rounded up to 4, rows past l
// are zeros and stay zeros).  Step j as in the
// register-resident kernel: the pivot group puts its raw column into an LDS
// buffer laid out [t][u] (16-byte reads) and into a global archive (P.R,
// column j = raw_j, read only at the end) and forms beta, tau and scale;
// every other column takes w = tau (col_j + scale sum_{i>j} raw_i col_i),
// col_i -= (w scale) raw_i below j, col_j -= w, and posts its squared norm
// below j: one FMA per element and pass, masks only in the block of row j.
// Register rows above j are skipped in blocks of 16 (uniform branches).
// For l > 224 it takes the steps after k_qrcp_st's first l - 224: the
// trailing 224 x 224 block (rows >= l - 224 of the columns k_qrcp_st left, read
// from its work array through its column map), with its archive in P.Rinv, and
// writes the rest of T, the reflectors, tau, signs and perm (mapped back to
// the columns of M).
// ---------------------------------------------------------------------------

template <int LRC>
__global__ __launch_bounds__(4 * QHY_LMAX) void k_qrcp_hy(const Prob* __restrict__ probs,
                                                        const int32_t* __restrict__ pidx,
                                                        const int32_t* __restrict__ toff,
                                                        int cnt) {
    constexpr int RR = QHY_RR, CH = 4;  // register rows, skipped in blocks of 4 CH rows
    static_assert(RR % CH == 0 && CH % 2 == 0, "register rows in whole blocks of pairs");
    static_assert(LRC % 4 == 0 && LRC <= QHY_LR, "LDS rows");
    constexpr int LR = LRC;
    constexpr int LRP = LRC + 1;  // LDS doubles per thread (odd: conflict-free 8-byte reads)
    constexpr int ST = RR + LR + 2;  // doubles per lane row of the pivot buffer
    extern __shared__ __align__(16) double s_m[];  // [thread][u], u < LR
    __shared__ __align__(16) double s_pv[4 * ST];  // raw pivot column, [t][u]
    __shared__ double s_nrm[QHY_LMAX];
    __shared__ double s_tau[QHY_LMAX], s_scale[QHY_LMAX], s_beta[QHY_LMAX];
    __shared__ int s_perm[QHY_LMAX];
    __shared__ unsigned long long s_key[2];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    const int L = P.l;
    if (L <= QRT_LMAX) return;
    const bool tail = L > QHY_LMAX;  // the trailing block after k_qrcp_st
    const int l = tail ? QHY_LMAX : L;
    const int j0 = L - l;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int c = tid >> 2, t = tid & 3;
    const bool incol = c < l;
    // archive: column j = raw pivot column of step j (global address space, so
    // that its stores do not hold up the LDS waits)
    gdouble_rw* __restrict__ arc = (gdouble_rw*)(tail ? P.Rinv : P.R);
    gdouble* __restrict__ R2 = as_global(P.msrc);  // M^T: R2 (M = R2^T), or Mx
    gdouble* __restrict__ W = as_global(P.R);      // k_qrcp_st's work array (tail)
    const int32_t* __restrict__ cmap = (const int32_t*)P.Racc;
    const int mc = tail && incol ? cmap[c] : 0;     // column of M held by this group

    // rows past l are zero and stay zero (the pivot column is zero there);
    // the norm takes the rows in increasing order, as every step does
    double col[RR];
    double nn = 0.0;
#pragma unroll
    for (int k = 0; k < LR; k++) {
        const int i = 4 * k + t;
        const double v =
            (incol && i < l) ? (tail ? W[(j0 + i) * L + mc] : R2[c * l + i]) : 0.0;
        s_m[tid * LRP + k] = v;
        nn = fma(v, v, nn);
    }
#pragma unroll
    for (int u = 0; u < RR; u++) {
        const int i = 4 * (LR + u) + t;
        // M[i][c] = R2[c][i]; tail: row j0 + i of column mc of the work array
        col[u] = (incol && i < l) ? (tail ? W[(j0 + i) * L + mc] : R2[c * l + i]) : 0.0;
        nn = fma(col[u], col[u], nn);
    }
    nn = quad_sum(nn);
    if (tid < 2) s_key[tid] = 0ull;
    __syncthreads();
    if (incol && t == 0) {
        s_nrm[c] = nn;
        atomicMax(&s_key[0], qr_key(nn, c));
    }
    bool active = incol;
    __syncthreads();

    for (int j = 0; j < l; j++) {
        const unsigned long long key = s_key[j & 1];
        const int p = 511 - (int)(key & 0x1FFull);
        if (c == p) {
            double* pv = s_pv + t * ST;
#pragma unroll
            for (int u = 0; u < RR; u += 2)
                *reinterpret_cast<double2*>(pv + LR + u) = make_double2(col[u], col[u + 1]);
            // LDS rows in blocks of 16 rows that lie above j are not read from
            // the pivot buffer again (the archive takes them from s_m)
#pragma unroll
            for (int q = 0; q < LR / 4; q++) {
                if (16 * q + 15 < j) continue;
#pragma unroll
                for (int kk = 0; kk < 4; kk++) pv[4 * q + kk] = s_m[tid * LRP + 4 * q + kk];
                __builtin_amdgcn_sched_barrier(0);  // 4 rows in flight
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double alpha = s_pv[(j & 3) * ST + (j >> 2)];
            const double ss = s_nrm[p];  // sum over rows >= j of column p squared
            double tau = 0.0, beta = alpha, scale = 1.0;
            if (ss > 0.0) {
                const double h = 0.5 * ss;
                double y = __builtin_amdgcn_rsq(ss);
#pragma unroll
                for (int it = 0; it < 2; it++) y = fma(y, fma(-h * y, y, 0.5), y);
                const double xnorm = ss * y;
                const double sg = alpha >= 0.0 ? -1.0 : 1.0;
                beta = sg * xnorm;
                scale = recip_nr(alpha - beta);
                tau = (beta - alpha) * (sg * y);
            }
            if (t == 0) {
                s_tau[j] = tau;
                s_scale[j] = scale;
                s_beta[j] = beta;
                s_perm[j] = p;
                s_key[(j + 1) & 1] = 0ull;
            }
            active = false;
        }
        __syncthreads();
        // archive the raw pivot column (global stores, off the pivot group's
        // path); rows of LDS blocks above j come from the pivot group's s_m
        if (tid < l) {
            const int k = tid >> 2;
            arc[j * l + tid] = (k < LR && 16 * (k >> 2) + 15 < j) ? s_m[(4 * p + (tid & 3)) * LRP + k]
                                                                    : s_pv[(tid & 3) * ST + k];
        }
        if (active) {
            const double tau = s_tau[j], scale = s_scale[j];
            const double* pv = s_pv + t * ST;
            // row i = 4 u' + t of this lane (u' = u + LR in registers, u' = k
            // in LDS) is below / at row j iff 4 u' > / == jt (compares
            // against constants: no per-row index registers)
            const int jt = j - t;
            // w = tau (col_j + scale sum_{i > j} raw_i col_i); only the block
            // that holds row j needs per-element masks.  Each partial sum
            // takes its rows in increasing order (LDS rows, then register
            // rows), so the result does not depend on the LDS row count.
            double d4[4] = {0.0, 0.0, 0.0, 0.0};
            double cj = 0.0;  // col_j in the lane that holds row j
#pragma unroll
            for (int q = 0; q < LR / 4; q++) {  // LDS rows in blocks of 16
                const int lo = 16 * q, hi = lo + 15;
                if (hi < j) continue;
#pragma unroll
                for (int kk = 0; kk < 4; kk++) {
                    const int k = 4 * q + kk, i4 = 4 * k;
                    const double x = s_m[tid * LRP + k];
                    if (lo > j) {
                        d4[kk] = fma(pv[k], x, d4[kk]);
                    } else {
                        d4[kk] = fma(i4 > jt ? pv[k] : 0.0, x, d4[kk]);
                        cj = i4 == jt ? x : cj;
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < RR / CH; q++) {
                const int lo = 4 * (LR + CH * q), hi = lo + 4 * CH - 1;
                if (hi < j) continue;
#pragma unroll
                for (int u = q * CH; u < q * CH + CH; u += 2) {
                    const double2 r = *reinterpret_cast<const double2*>(pv + LR + u);
                    if (lo > j) {
                        d4[u & 3] = fma(r.x, col[u], d4[u & 3]);
                        d4[(u + 1) & 3] = fma(r.y, col[u + 1], d4[(u + 1) & 3]);
                    } else {
                        const int i0 = 4 * (LR + u), i1 = i0 + 4;
                        d4[u & 3] = fma(i0 > jt ? r.x : 0.0, col[u], d4[u & 3]);
                        d4[(u + 1) & 3] = fma(i1 > jt ? r.y : 0.0, col[u + 1], d4[(u + 1) & 3]);
                        cj = i0 == jt ? col[u] : (i1 == jt ? col[u + 1] : cj);
                    }
                }
            }
            const double w = tau * quad_sum(fma(scale, (d4[0] + d4[1]) + (d4[2] + d4[3]), cj));
            const double ws = w * scale;
            // col_i -= ws raw_i below j, col_j -= w; squared norm below j
            double n4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < LR / 4; q++) {
                const int lo = 16 * q, hi = lo + 15;
                if (hi < j) continue;
#pragma unroll
                for (int kk = 0; kk < 4; kk++) {
                    const int k = 4 * q + kk, i4 = 4 * k;
                    double x = s_m[tid * LRP + k];
                    if (lo > j) {
                        x = fma(-ws, pv[k], x);
                        n4[kk] = fma(x, x, n4[kk]);
                    } else {
                        x = i4 > jt ? fma(-ws, pv[k], x) : (i4 == jt ? x - w : x);
                        if (i4 > jt) n4[kk] = fma(x, x, n4[kk]);
                    }
                    s_m[tid * LRP + k] = x;
                }
            }
#pragma unroll
            for (int q = 0; q < RR / CH; q++) {
                const int lo = 4 * (LR + CH * q), hi = lo + 4 * CH - 1;
                if (hi < j) continue;
#pragma unroll
                for (int u = q * CH; u < q * CH + CH; u += 2) {
                    const double2 r = *reinterpret_cast<const double2*>(pv + LR + u);
                    if (lo > j) {
                        col[u] = fma(-ws, r.x, col[u]);
                        col[u + 1] = fma(-ws, r.y, col[u + 1]);
                        n4[u & 3] = fma(col[u], col[u], n4[u & 3]);
                        n4[(u + 1) & 3] = fma(col[u + 1], col[u + 1], n4[(u + 1) & 3]);
                    } else {
                        const int i0 = 4 * (LR + u), i1 = i0 + 4;
                        col[u] = i0 > jt ? fma(-ws, r.x, col[u]) : (i0 == jt ? col[u] - w : col[u]);
                        col[u + 1] = i1 > jt ? fma(-ws, r.y, col[u + 1]) : (i1 == jt ? col[u + 1] - w : col[u + 1]);
                        if (i0 > jt) n4[u & 3] = fma(col[u], col[u], n4[u & 3]);
                        if (i1 > jt) n4[(u + 1) & 3] = fma(col[u + 1], col[u + 1], n4[(u + 1) & 3]);
                    }
                }
            }
            const double n = quad_sum((n4[0] + n4[1]) + (n4[2] + n4[3]));
            if (t == 0) {
                s_nrm[c] = n;
                atomicMax(&s_key[(j + 1) & 1], qr_key(n, c));
            }
        }
        __syncthreads();
    }

    // Outputs from the archive: arc[b * l + i] = raw_b[i] (the archive writes
    // of the pivot groups are visible after the barriers of the loop)
    if (!tail) {
        for (int e = tid; e < l * l; e += nth) {
            const int a = e / l, b = e % l;
            double tv = 0.0;
            if (a < b) tv = arc[b * l + a] * (s_beta[a] < 0.0 ? -1.0 : 1.0);
            else if (a == b) tv = fabs(s_beta[a]);
            P.T[e] = tv;
            // reflector a, component b
            double vv = 0.0;
            if (b == a) vv = 1.0;
            else if (b > a) vv = arc[a * l + b] * s_scale[a];
            P.Qt[e] = vv;
        }
        for (int jj = tid; jj < l; jj += nth) {
            P.tau[jj] = s_tau[jj];
            P.tau[LMAX + jj] = s_beta[jj] < 0.0 ? -1.0 : 1.0;
            P.perm[jj] = s_perm[jj];
        }
        return;
    }
    // Tail: rows < j0 of T beyond column j0 are the final values of the
    // columns pivoted here at those rows (W, untouched after step a < j0),
    // with k_qrcp_st's row signs; rows >= j0 come from this block's archive.
    for (int e = tid; e < L * L; e += nth) {
        const int a = e / L, b = e % L;
        if (a < j0) {
            if (b >= j0) P.T[e] = W[a * L + cmap[s_perm[b - j0]]] * P.tau[LMAX + a];
            continue;
        }
        const int a2 = a - j0, b2 = b - j0;
        double tv = 0.0, vv = 0.0;
        if (b2 >= 0) {
            if (a2 < b2) tv = arc[b2 * l + a2] * (s_beta[a2] < 0.0 ? -1.0 : 1.0);
            else if (a2 == b2) tv = fabs(s_beta[a2]);
            if (b2 == a2) vv = 1.0;
            else if (b2 > a2) vv = arc[a2 * l + b2] * s_scale[a2];
        }
        P.T[e] = tv;
        P.Qt[e] = vv;
    }
    for (int jj = tid; jj < l; jj += nth) {
        P.tau[j0 + jj] = s_tau[jj];
        P.tau[LMAX + j0 + jj] = s_beta[jj] < 0.0 ? -1.0 : 1.0;
        P.perm[j0 + jj] = cmap[s_perm[jj]];
    }
}

// ---------------------------------------------------------------------------
// Register-resident QRCP of M = R2^T for l <= 128 (one block per problem).
//   LPC = 8 adjacent lanes own one column of M; lane t of the group
//   keeps rows i = LPC u + t (u < RPT) in registers, so the trailing matrix
//   never leaves the register file and per-column dot products and norms are
//   group sums (DPP steps).  Columns stay in place; the pivot column of step
//   j is found with the 64-bit key above and retired after the step.  Step j:
//     1. the pivot group copies its raw column into slot j of an LDS archive
//        (laid out [t][u] so that a lane moves 16 bytes at a time), reads
//        alpha = M[j][p] back and forms beta, tau and scale = 1/(alpha-beta)
//        (reflector v_i = scale*M[i][p] below j, v_j = 1, zero above);
//     2. every remaining column reads the archived pivot column:
//        w = tau (col_j + scale sum_{i>j} raw_i col_i), col_j -= w,
//        col_i -= (w scale) raw_i below j, and posts the squared norm of its
//        rows below j as the next step's key.
//   Rows above j are skipped in blocks of LPC*CH rows (uniform branches);
//   only the block holding row j needs per-element selects.  Two barriers per
//   step and no global memory access inside the loop: T, the reflectors,
//   tau, the signs of T_jj and perm are written from the archive at the end.
//   Eight lanes per column (rather than four) halve the serial work of a
//   lane and double the waves that hide the FP64 latency.
// ---------------------------------------------------------------------------
template <int LPC>
__device__ __forceinline__ double group_sum(double v) {
    v += dpp_mov<0xB1>(v);  // quad_perm 1,0,3,2
    v += dpp_mov<0x4E>(v);  // quad_perm 2,3,0,1
    if constexpr (LPC == 8) v += dpp_mov<0x141>(v);  // row_half_mirror: the two quads
    return v;
}

template <int RPT>
__host__ __device__ constexpr int qrt_stride() { return RPT + 2; }  // doubles per archived lane row

// dynamic LDS of the archive for l steps
template <int RPT, int LPC>
__host__ __device__ constexpr size_t qrt_lds_bytes(int l) {
    return sizeof(double) * (size_t)l * LPC * qrt_stride<RPT>();
}

template <int RPT, int LPC>
__global__ __launch_bounds__(LPC * LPC * RPT) void k_qrcp_rt(const Prob* __restrict__ probs,
                                                         const int32_t* __restrict__ pidx,
                                                         const int32_t* __restrict__ toff,
                                                         int cnt) {
    constexpr int LR = LPC * RPT;  // rows covered
    constexpr int ST = qrt_stride<RPT>();
    constexpr int CH = RPT < 8 ? RPT : 8;  // u per row block
    constexpr int NCH = RPT / CH;
    constexpr int LSH = LPC == 8 ? 3 : 2;
    // Partial sums per lane (short FP64 chains).  LPC and NP are the same for
    // every l, so a problem's arithmetic does not depend on the largest l of
    // its launch (RPT only adds rows of zeros).
    constexpr int NP = 4;
    extern __shared__ __align__(16) double s_arc[];  // [l steps][LPC lanes][ST]
    __shared__ double s_nrm[LR];
    __shared__ double s_tau[LR], s_scale[LR], s_beta[LR];
    __shared__ int s_perm[LR];
    __shared__ unsigned long long s_key[2];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    const int l = P.l;
    if (l > LR) return;
    const int tid = threadIdx.x;
    const int c = tid >> LSH, t = tid & (LPC - 1);
    const bool incol = c < l;
    const double* __restrict__ R2 = P.msrc;  // M^T: R2 (M = R2^T), or Mx

    double col[RPT];
#pragma unroll
    for (int u = 0; u < RPT; u++) {
        const int i = LPC * u + t;
        col[u] = (incol && i < l) ? R2[c * l + i] : 0.0;  // M[i][c] = R2[c][i]
    }
    double nn = 0.0;
#pragma unroll
    for (int u = 0; u < RPT; u++) nn = fma(col[u], col[u], nn);
    nn = group_sum<LPC>(nn);
    if (tid < 2) s_key[tid] = 0ull;
    __syncthreads();
    if (incol && t == 0) {
        s_nrm[c] = nn;
        atomicMax(&s_key[0], qr_key(nn, c));
    }
    bool active = incol;
    __syncthreads();

    for (int j = 0; j < l; j++) {
        const unsigned long long key = s_key[j & 1];
        const int p = 511 - (int)(key & 0x1FFull);
        double* arc = s_arc + j * LPC * ST;
        if (c == p) {
#pragma unroll
            for (int u = 0; u < RPT; u += 2)
                *reinterpret_cast<double2*>(arc + t * ST + u) = make_double2(col[u], col[u + 1]);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            const double alpha = arc[(j & (LPC - 1)) * ST + (j >> LSH)];
            const double ss = s_nrm[p];  // sum over rows >= j of column p squared
            double tau = 0.0, beta = alpha, scale = 1.0;
            if (ss > 0.0) {
                // ||x|| = ss y with y = 1/sqrt(ss) (estimate + two Newton
                // steps); 1/beta = -+y, so tau needs no division.
                const double h = 0.5 * ss;
                double y = __builtin_amdgcn_rsq(ss);
#pragma unroll
                for (int it = 0; it < 2; it++) y = fma(y, fma(-h * y, y, 0.5), y);
                const double xnorm = ss * y;
                const double sg = alpha >= 0.0 ? -1.0 : 1.0;
                beta = sg * xnorm;
                scale = recip_nr(alpha - beta);
                tau = (beta - alpha) * (sg * y);
            }
            if (t == 0) {
                s_tau[j] = tau;
                s_scale[j] = scale;
                s_beta[j] = beta;
                s_perm[j] = p;
                s_key[(j + 1) & 1] = 0ull;
            }
            active = false;
        }
        __syncthreads();
        if (active) {
            const double tau = s_tau[j], scale = s_scale[j];
            const double* arct = arc + t * ST;
            // v_i = scale raw_i below row j, 1 at row j, 0 above.  NP
            // partial sums per lane keep the dependent FP64 chains short.
            double vv[RPT], d8[NP];
#pragma unroll
            for (int e = 0; e < NP; e++) d8[e] = 0.0;
#pragma unroll
            for (int q = 0; q < NCH; q++) {
                const int lo = LPC * CH * q, hi = lo + LPC * CH - 1;
                if (hi < j) continue;
#pragma unroll
                for (int u = q * CH; u < q * CH + CH; u += 2) {
                    const double2 r2 = *reinterpret_cast<const double2*>(arct + u);
                    vv[u] = r2.x * scale;
                    vv[u + 1] = r2.y * scale;
                }
                if (lo <= j) {
#pragma unroll
                    for (int u = q * CH; u < q * CH + CH; u++) {
                        const int i = LPC * u + t;
                        vv[u] = i > j ? vv[u] : (i == j ? 1.0 : 0.0);
                    }
                }
#pragma unroll
                for (int u = q * CH; u < q * CH + CH; u++) d8[u % NP] = fma(vv[u], col[u], d8[u % NP]);
            }
            double dsum = (d8[0] + d8[1]) + (d8[2] + d8[3]);
            if constexpr (NP == 8) dsum += (d8[4] + d8[5]) + (d8[6] + d8[7]);
            const double w = tau * group_sum<LPC>(dsum);
            double n8[NP];
#pragma unroll
            for (int e = 0; e < NP; e++) n8[e] = 0.0;
#pragma unroll
            for (int q = 0; q < NCH; q++) {
                const int lo = LPC * CH * q, hi = lo + LPC * CH - 1;
                if (hi < j) continue;
                if (lo > j) {
#pragma unroll
                    for (int u = q * CH; u < q * CH + CH; u++) {
                        col[u] = fma(-w, vv[u], col[u]);
                        n8[u % NP] = fma(col[u], col[u], n8[u % NP]);
                    }
                } else {
#pragma unroll
                    for (int u = q * CH; u < q * CH + CH; u++) {
                        const int i = LPC * u + t;
                        col[u] = fma(-w, vv[u], col[u]);
                        if (i > j) n8[u % NP] = fma(col[u], col[u], n8[u % NP]);
                    }
                }
            }
            double nsum = (n8[0] + n8[1]) + (n8[2] + n8[3]);
            if constexpr (NP == 8) nsum += (n8[4] + n8[5]) + (n8[6] + n8[7]);
            const double n = group_sum<LPC>(nsum);
            if (t == 0) {
                s_nrm[c] = n;
                atomicMax(&s_key[(j + 1) & 1], qr_key(n, c));
            }
        }
        __syncthreads();
    }

    // Outputs from the archive: raw_j[i] = M[i][perm j] after step j - 1.
    for (int e = tid; e < l * l; e += blockDim.x) {
        const int a = e / l, b = e % l;
        // T[a][b] (row a, column b): rows above b hold the archived column b.
        double tv = 0.0;
        if (a < b) tv = s_arc[(b * LPC + (a & (LPC - 1))) * ST + (a >> LSH)] * (s_beta[a] < 0.0 ? -1.0 : 1.0);
        else if (a == b) tv = fabs(s_beta[a]);
        P.T[e] = tv;
        // reflector a, component b
        double vv = 0.0;
        if (b == a) vv = 1.0;
        else if (b > a) vv = s_arc[(a * LPC + (b & (LPC - 1))) * ST + (b >> LSH)] * s_scale[a];
        P.Qt[e] = vv;
    }
    for (int j = tid; j < l; j += blockDim.x) {
        P.tau[j] = s_tau[j];
        P.tau[LMAX + j] = s_beta[j] < 0.0 ? -1.0 : 1.0;
        P.perm[j] = s_perm[j];
    }
}

template <int RPT, int LPC>
static hipError_t launch_qrcp_rt(const LaunchGroup& g, int lmax, hipStream_t s) {
    constexpr int LR = RPT * LPC;
    const size_t lds = qrt_lds_bytes<RPT, LPC>(std::min(lmax, LR));
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_qrcp_rt<RPT, LPC>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)qrt_lds_bytes<RPT, LPC>(LR));
        if (e != hipSuccess) return e;
        attr = true;
    }
    // LPC lanes per column, columns rounded up to whole waves
    const int threads = (LPC * std::min(lmax, LR) + 63) / 64 * 64;
    hipLaunchKernelGGL((k_qrcp_rt<RPT, LPC>), dim3(g.blocks), dim3(threads), lds, s, g.probs, g.pidx,
                       g.toff, g.count);
    return hipGetLastError();
}

template <int LRC>
static hipError_t launch_qrcp_hy(const LaunchGroup& g, int lh, hipStream_t s) {
    const int threads = (4 * lh + 63) / 64 * 64;
    constexpr int LRP = LRC ? LRC + 1 : 0;
    const size_t lds = sizeof(double) * (size_t)LRP * threads;
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)k_qrcp_hy<LRC>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)(sizeof(double) * LRP * 4 * QHY_LMAX));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(k_qrcp_hy<LRC>, dim3(g.blocks), dim3(threads), lds, s, g.probs, g.pidx,
                       g.toff, g.count);
    return hipGetLastError();
}

hipError_t launch_qrcp(const LaunchGroup& g, int lmax, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    {
        const int lr = std::min(lmax, QRT_LMAX);
        hipError_t e = lr <= 16   ? launch_qrcp_rt<2, 8>(g, lr, s)
                       : lr <= 32 ? launch_qrcp_rt<4, 8>(g, lr, s)
                       : lr <= 64 ? launch_qrcp_rt<8, 8>(g, lr, s)
                                  : launch_qrcp_rt<16, 8>(g, lr, s);
        if (e != hipSuccess || lmax <= QRT_LMAX) return e;
    }
    // l > 224: the first l - 224 steps with M streamed from the L2-resident
    // work array, 4 lanes per column; k_qrcp_hy takes the rest
    // (QMB_G groups per problem with the matrix in registers when every group
    // of the launch fits on the chip at once, else one block streaming it)
    if (lmax > QHY_LMAX) {
        if (g.blocks <= QMB_MAX_PROBS) {
            hipLaunchKernelGGL(k_qrcp_mb, dim3(g.blocks * QMB_G), dim3(QMB_THREADS), 0, s, g.probs,
                               g.pidx, g.toff, g.count);
        } else {
            const int threads = std::min(QST_THREADS, (4 * lmax + 63) / 64 * 64);
            hipLaunchKernelGGL(k_qrcp_st, dim3(g.blocks), dim3(threads), 0, s, g.probs, g.pidx,
                               g.toff, g.count);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    // 128 < l <= 224, and the trailing 224 steps of larger l: registers and LDS
    const int lh = std::min(lmax, QHY_LMAX);
    // LDS rows per lane for the largest l of the launch, rounded up to 4
    const int lrc = std::max(0, ((lh + 3) / 4 - QHY_RR + 3) / 4 * 4);
    return lrc == 0    ? launch_qrcp_hy<0>(g, lh, s)
           : lrc == 4  ? launch_qrcp_hy<4>(g, lh, s)
           : lrc == 8  ? launch_qrcp_hy<8>(g, lh, s)
           : lrc == 12 ? launch_qrcp_hy<12>(g, lh, s)
           : lrc == 16 ? launch_qrcp_hy<16>(g, lh, s)
                       : launch_qrcp_hy<20>(g, lh, s);
}

// ---------------------------------------------------------------------------
// The reflectors of the QRCP applied to rows: where u_via_qs, to the rows of
// the l x l identity, giving Qs = H_0 H_1 ... H_{l-1} diag(sign) in G (free
// after the last Cholesky), and U = Q1 Qs is then one FP64 MFMA product
// (k_apply); otherwise straight to the rows of Q1, giving U.  Sixteen lanes
// share a row; lane k holds the entries a = k (mod 16) in registers, so a
// reflector costs a dot product (four partial sums), a four-step DPP
// reduction and an axpy.  Each row is a chain of l dependent reflectors, so
// the time is that chain's, and for l > 128 work-groups of 16 rows put one
// wave on each SIMD: 65 us at l = 220 (99 us with 8 lanes per row in 32-row
// groups, 81 us with 16 lanes per row in 32-row groups, two waves per SIMD).
// Smaller l keeps 32-row groups (half the reflector panel loads for the many
// rows of Q1 or of a batch of small problems).  The reflectors stream
// through LDS in panels of 32; the next reflector's entries are read while
// the current one is applied.
// ---------------------------------------------------------------------------
constexpr int FU_PANEL = 32;
constexpr int FU_LANES = 16;                      // lanes per row
constexpr int FU_TNMAX = (LMAX + FU_LANES - 1) / FU_LANES;

template <int TN>
__global__ __launch_bounds__(formqs_rows(FU_LANES * TN) * FU_LANES) void k_form_qs(const Prob* __restrict__ probs,
                                                const int32_t* __restrict__ pidx,
                                                const int32_t* __restrict__ toff, int cnt) {
    constexpr int LPAD = FU_LANES * TN;            // reflector rows padded with zeros
    constexpr int FU_ROWS = formqs_rows(LPAD);     // rows per work-group
    constexpr int FU_THREADS = FU_ROWS * FU_LANES;
    extern __shared__ __align__(16) double vt[];   // FU_PANEL x LPAD
    __shared__ double s_tau[FU_PANEL];
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    const int l = P.l;
    const bool ident = u_via_qs(P.m, l);
    const int tid = threadIdx.x;
    const int rr = tid / FU_LANES, k = tid % FU_LANES;
    const int64_t row = (int64_t)local * FU_ROWS + rr;
    const bool rv = row < (ident ? (int64_t)l : P.m);
    double u[TN];
#pragma unroll
    for (int t = 0; t < TN; t++) {
        const int a = k + FU_LANES * t;
        u[t] = ident ? ((rv && a == row) ? 1.0 : 0.0) : ((rv && a < l) ? P.Q1[row * l + a] : 0.0);
    }
    for (int j0 = 0; j0 < l; j0 += FU_PANEL) {
        const int pj = min(FU_PANEL, l - j0);
        __syncthreads();
        {
            // the panel (FU_PANEL x LPAD entries, NLD per thread), all
            // loads in flight (entries outside Qt read a zero word)
            constexpr int NLD = FU_PANEL * LPAD / FU_THREADS;
            static_assert(NLD * FU_THREADS == FU_PANEL * LPAD, "whole panel entries per thread");
            gdouble* qt = as_global(P.Qt);
            gdouble* zw = as_global(g_zero_chol);
            double pv[NLD];
#pragma unroll
            for (int u = 0; u < NLD; u++) {
                const int e = tid + FU_THREADS * u;
                const int jj = e / LPAD, a = e - (e / LPAD) * LPAD;
                pv[u] = *((jj < pj && a < l) ? qt + (int64_t)(j0 + jj) * l + a : zw);
            }
#pragma unroll
            for (int u = 0; u < NLD; u++) vt[tid + FU_THREADS * u] = pv[u];
        }
        if (tid < pj) s_tau[tid] = P.tau[j0 + tid];
        __syncthreads();
        // the next reflector's entries are read while this one is applied
        double vv[TN];
#pragma unroll
        for (int t = 0; t < TN; t++) vv[t] = vt[k + FU_LANES * t];
        for (int jj = 0; jj < pj; jj++) {
            const double* vnx = vt + min(jj + 1, pj - 1) * LPAD + k;
            double vn[TN];
#pragma unroll
            for (int t = 0; t < TN; t++) vn[t] = vnx[FU_LANES * t];
            double d4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int t = 0; t < TN; t++) d4[t & 3] = fma(u[t], vv[t], d4[t & 3]);
            const double d = sum16_dpp((d4[0] + d4[1]) + (d4[2] + d4[3]));
            const double w = s_tau[jj] * d;
#pragma unroll
            for (int t = 0; t < TN; t++) u[t] -= w * vv[t];
#pragma unroll
            for (int t = 0; t < TN; t++) vv[t] = vn[t];
        }
    }
    if (!rv) return;
#pragma unroll
    for (int t = 0; t < TN; t++) {
        const int a = k + FU_LANES * t;
        if (a < l) (ident ? P.G : P.U)[row * l + a] = u[t] * P.tau[LMAX + a];
    }
}

hipError_t launch_form_qs(const LaunchGroup& g, int l, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    const size_t lds = sizeof(double) * FU_PANEL * FU_LANES * FU_TNMAX;
    const int tn = (l + FU_LANES - 1) / FU_LANES;
#define FU_CASE(N)                                                                              \
    if (tn <= N) {                                                                              \
        static bool attr = false;                                                               \
        if (!attr) {                                                                            \
            hipError_t e = hipFuncSetAttribute((const void*)k_form_qs<N>,                        \
                                               hipFuncAttributeMaxDynamicSharedMemorySize,      \
                                               (int)lds);                                       \
            if (e != hipSuccess) return e;                                                      \
            attr = true;                                                                        \
        }                                                                                       \
        hipLaunchKernelGGL(k_form_qs<N>, dim3(g.blocks), dim3(formqs_rows(FU_LANES * N) * FU_LANES), \
                           lds, s, g.probs,                                                     \
                           g.pidx,                                                              \
                           g.toff, g.count);                                                    \
        return hipGetLastError();                                                               \
    }
    FU_CASE(2) FU_CASE(4) FU_CASE(8) FU_CASE(12) FU_CASE(FU_TNMAX)
#undef FU_CASE
    return hipErrorInvalidValue;
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
    // explicit or eq. (18) compression: ||M - R2^T||_F / ||M||_F (Mx and R2
    // both hold transposes)
    double dm = 0.0, mm = 0.0;
    if (P.mmode != M_R2T)
        for (int e = threadIdx.x; e < l * l; e += 256) {
            const double v = P.Mx[e], d = v - P.R2[e];
            dm += d * d;
            mm += v * v;
        }
    dm = block_sum256(dm, red);
    mm = block_sum256(mm, red);
    if (threadIdx.x == 0) {
        double na = 0.0;
        for (int b = 0; b < NORM_BLOCKS; b++) na += P.rep[32 + b];
        P.rep[4] = na;
        P.rep[0] = na > 0.0 ? sqrt(fmax(0.0, 1.0 - t2 / na)) : 0.0;
        P.rep[1] = na > 0.0 ? sqrt(fmax(0.0, 1.0 - tk2 / na)) : 0.0;
        P.rep[5] = mm > 0.0 ? sqrt(dm / mm) : 0.0;
    }
}

hipError_t launch_report(const LaunchGroup& g, int phase, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_report, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count,
                       phase);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// ULV requests run as the URV of A^T: the transposed copy At (n x m, leading
// dimension P.lda) of the caller's A (m x n, leading dimension P.ulv_lda),
// 32 x 32 tiles through LDS so that both sides are read and written in
// contiguous runs; and at the end T = T'^T (lower triangular).  P.m, P.n are
// the dimensions of A^T.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void transpose_tile(const T* __restrict__ a, int64_t m, int64_t n, int64_t lda,
                               T* __restrict__ at, int64_t ldt, int64_t tr, int64_t tc) {
    __shared__ T tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 8 rows per pass
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = tr + r, j = tc + tx;
        if (i < m && j < n) tile[r][tx] = a[i * lda + j];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t j = tc + r, i = tr + tx;  // At[j][i] = A[i][j]
        if (i < m && j < n) at[j * ldt + i] = tile[tx][r];
    }
}

__global__ __launch_bounds__(256) void k_transpose_a(const Prob* __restrict__ probs,
                                                     const int32_t* __restrict__ pidx,
                                                     const int32_t* __restrict__ toff, int cnt) {
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    if (!P.ulv) return;
    const int64_t m = P.n, n = P.m;  // the caller's matrix
    const int64_t tcs = (n + 31) / 32;
    const int64_t tr = (int64_t)(local / tcs) * 32, tc = (int64_t)(local % tcs) * 32;
    switch (P.prec) {
        case P_F64:
            transpose_tile<double>(reinterpret_cast<const double*>(P.ulv_src), m, n, P.ulv_lda,
                                   reinterpret_cast<double*>(const_cast<void*>(P.A)), P.lda, tr, tc);
            break;
        case P_F32:
            transpose_tile<float>(reinterpret_cast<const float*>(P.ulv_src), m, n, P.ulv_lda,
                                  reinterpret_cast<float*>(const_cast<void*>(P.A)), P.lda, tr, tc);
            break;
        default:
            transpose_tile<uint16_t>(reinterpret_cast<const uint16_t*>(P.ulv_src), m, n, P.ulv_lda,
                                     reinterpret_cast<uint16_t*>(const_cast<void*>(P.A)), P.lda, tr,
                                     tc);
            break;
    }
}

hipError_t launch_transpose_a(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_transpose_a, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff,
                       g.count);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_ulv_t(const Prob* __restrict__ probs,
                                               const int32_t* __restrict__ pidx,
                                               const int32_t* __restrict__ toff, int cnt) {
    int local;
    const Prob& P = group_prob2(probs, pidx, toff, cnt, local);
    if (!P.ulv) return;
    const int l = P.l;
    const int e = local * 256 + threadIdx.x;
    if (e >= l * l) return;
    const int a = e / l, b = e - (e / l) * l;
    P.Tout[e] = P.T[b * l + a];
}

hipError_t launch_ulv_t(const LaunchGroup& g, hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_ulv_t, dim3(g.blocks), dim3(256), 0, s, g.probs, g.pidx, g.toff, g.count);
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

// Column scales of cor_quantize: a block takes 64 columns, its four waves
// stride over the rows (each wave reads 64 consecutive floats of a row), and
// the four partial maxima meet in LDS.
__global__ __launch_bounds__(256) void k_colscale(const float* __restrict__ a, int64_t m, int64_t n,
                                                  int64_t lda, float* __restrict__ s) {
    __shared__ float part[4][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t c = (int64_t)blockIdx.x * 64 + lane;
    float mx = 0.0f;
    if (c < n)
        for (int64_t r = wave; r < m; r += 4) mx = fmaxf(mx, fabsf(a[r * lda + c]));
    part[wave][lane] = mx;
    __syncthreads();
    if (wave == 0 && c < n) {
        mx = fmaxf(fmaxf(part[0][lane], part[1][lane]), fmaxf(part[2][lane], part[3][lane]));
        s[c] = mx > 0.0f ? mx / 448.0f : 1.0f;
    }
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
    hipLaunchKernelGGL(k_colscale, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, a32, m, n,
                       lda, colscale);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_to_fp8, dim3(blocks), dim3(256), 0, s, a32, m, n, lda, colscale,
                       reinterpret_cast<uint8_t*>(out));
    return hipGetLastError();
}

}  // namespace cor
