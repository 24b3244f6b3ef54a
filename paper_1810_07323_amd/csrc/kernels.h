// Host-side launch interface of the device kernels (internal to libcorutv).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace cor {

struct Prob;

// A launch over a group of problems: block b serves problem probs[pidx[j]]
// with toff[j] <= b < toff[j + 1]; toff has count + 1 entries (device).
struct LaunchGroup {
    const Prob* probs;
    const int32_t* pidx;
    const int32_t* toff;
    int32_t count;
    int32_t blocks;
};

// SIDE_F: the n-side rows summed over the row splits of the fused power step.
enum Side : int32_t { SIDE_M = 0, SIDE_N = 1, SIDE_F = 2 };

// Passes over A (split-K partial sums).
hipError_t launch_sketch(int prec, bool trans, int nt, const LaunchGroup& g, int iter,
                         hipStream_t s);
int sketch_rows_per_block(int prec, int nt, bool trans);  // output rows per block of A X / A^T X
int sketch_k_tile(int prec);
// Fused power step: per row split, the partial sums of A^T (A X) (n x lp, in
// the accumulation format) into ypart; blocks per problem s_f.  nt = lp / 16 of
// the launch (at most ATA_NTMAX), prec F32 or F64, tpw = tiles of the n x lp
// sum per wave (ata_tiles_per_wave, at most ata_max_tiles_per_wave), lds =
// the largest ata_lds_bytes of the launch (at most ATA_LDS).
constexpr int ATA_ROWS = 128;      // granularity of a row split
constexpr int ATA_NTMAX = 4;       // l <= 64
constexpr int ATA_NMAX32 = 2400;   // largest n (FP32): a 16-row chunk of A in LDS
constexpr int ATA_NMAX64 = 1024;   // largest n (FP64)
constexpr int ATA_LDS = 160 * 1024;
int ata_tiles_per_wave(int64_t n, int lp);
int ata_max_tiles_per_wave(int prec, int lp);
size_t ata_lds_bytes(int64_t n, int lp, int prec);
hipError_t launch_ata(int prec, int nt, int tpw, size_t lds, const LaunchGroup& g, int iter,
                      hipStream_t s);

// Row-block kernels.
hipError_t launch_omega(const LaunchGroup& g, hipStream_t s);          // blocks: ceil(n*l/2/256)
hipError_t launch_make_op(const LaunchGroup& g, int side, hipStream_t s);  // blocks: ceil(lp*ld/256)
hipError_t launch_sum(const LaunchGroup& g, int side, int iter, hipStream_t s);  // ceil(rows*lp/4/256)
// Gram partial sums of a row-major rows x l FP64 matrix picked by `src`.
enum GramSrc : int32_t { GSRC_Y = 0, GSRC_QA = 1, GSRC_U = 2, GSRC_V = 3,
                         GSRC_XM = 4,   // Q1^T (A Q2): every tile (compression of eq. (14))
                         GSRC_XA = 5,   // Q2^T X: every tile (eq. (18))
                         GSRC_XY = 6 }; // X^T (A^T A X) of the fused power step: symmetric
constexpr int GRAM_THREADS = 256;
// One upper 16 x 16 tile of the l x l Gram matrix per block (four waves
// split the chunk's rows); a launch covers (row chunks) x (upper tiles) blocks.
hipError_t launch_gram(const LaunchGroup& g, int side, int src, int iter, hipStream_t s);
hipError_t launch_gram_reduce(const LaunchGroup& g, int side, int second, int iter,
                              hipStream_t s);
// Cross products of GSRC_XM (into Mx, transposed) or GSRC_XA (into G); blocks ceil(l*l/64).
hipError_t launch_xreduce(const LaunchGroup& g, int src, hipStream_t s);
// Xk = Q2 at the last power step (eq. (18) problems); blocks ceil(n*l/256).
hipError_t launch_keep_x(const LaunchGroup& g, int iter, hipStream_t s);
// Operand copies: tiles of MO_ROWS rows x MO_COLS columns per block, blocks
// per problem ceil(ld / MO_ROWS) * (lp / MO_COLS).
constexpr int MO_ROWS = 64;
constexpr int MO_COLS = 16;
// dst = src R^{-1}, row blocks of APPLY_ROWS; lmax = largest l of the group.
constexpr int APPLY_ROWS = 16;
// Rows per work-group of the reflector product (k_form_qs): 16 for l > 128
// (one wave per SIMD on the few rows of Qs), 32 below (many rows of Q1 or of
// a batch's small problems: half the reflector panel loads).
__host__ __device__ constexpr int formqs_rows(int l) { return l > 128 ? 16 : 32; }
enum ApplyMode : int32_t { AP_Y_RINV_QA = 0, AP_QA_RINV_Q = 1, AP_Y_RINV_Q = 2,
                           AP_Q1_QS_U = 3,   // U = Q1 Qs (Qs in G, after the QRCP)
                           AP_Y_RINV_Y = 4 };  // Y <- Y R1^{-1} in place (fused power step)
hipError_t launch_apply(const LaunchGroup& g, int side, int mode, int lmax, int iter,
                        hipStream_t s);
hipError_t launch_gather_v(const LaunchGroup& g, hipStream_t s);  // blocks: ceil(n*l/256)
// Column maxima of the FP64 factor and FP8 operand scales: per row chunk
// (`chunks`: blocks per problem = its chunk count), then per problem (`one`:
// one block per problem).
hipError_t launch_op_scales(const LaunchGroup& chunks, const LaunchGroup& one, int side, int iter,
                            hipStream_t s);

// One block per problem.
enum CholMode : int32_t { CHOL_FIRST = 0, CHOL_SECOND = 1 };
hipError_t launch_chol(const LaunchGroup& g, int mode, int lmax, int iter, hipStream_t s);
hipError_t launch_qrcp(const LaunchGroup& g, int lmax, hipStream_t s);
// R2 = R' R of the last Y2 (dst 0) or R1 of the last Y1 (dst 1, eq. (18)); blocks: nt*nt
hipError_t launch_r2(const LaunchGroup& g, int iter, int dst, hipStream_t s);
// Eq. (18): Mx = (R1 G^-1)^T with G = Q2^T X; one block per problem.
hipError_t launch_dapprox(const LaunchGroup& g, hipStream_t s);
// ULV requests: the transposed copy of A (tiles of 32 x 32; blocks
// ceil(m/32) * ceil(n/32) of the caller's matrix) and T = T'^T at the end
// (blocks ceil(l*l/256)).
hipError_t launch_transpose_a(const LaunchGroup& g, hipStream_t s);
hipError_t launch_ulv_t(const LaunchGroup& g, hipStream_t s);
// Reflectors applied to rows of the identity (u_via_qs: Qs into G, blocks
// ceil(l/32)) or of Q1 (U, blocks ceil(m/32)).
hipError_t launch_form_qs(const LaunchGroup& g, int l, hipStream_t s);
hipError_t launch_report(const LaunchGroup& g, int phase, hipStream_t s);
hipError_t launch_normA(const LaunchGroup& g, hipStream_t s);

// Stand-alone helpers of the C ABI.
hipError_t launch_quantize(const float* a32, int64_t m, int64_t n, int64_t lda, int to, void* out,
                           float* colscale, hipStream_t s);
hipError_t launch_omega_raw(uint64_t seed, int64_t n, int32_t l, double* out, hipStream_t s);
// Zero `bytes` (a multiple of 16) at the 16-byte aligned device address p.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);

}  // namespace cor
