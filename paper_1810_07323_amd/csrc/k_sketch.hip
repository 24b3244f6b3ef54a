// Passes over A: the sketch products of CoR-UTV (Alg. 3, power loop).
//
//   TRANS = false:  Y1 = A X    (m x l), contraction over the n columns of A
//   TRANS = true :  Y2 = A^T X  (n x l), contraction over the m rows of A
//
// A is streamed exactly once per pass.  A block owns BM = 128 output rows and
// one K range (split-K); every wave owns RT = 2 row tiles of 16 and all NT
// column tiles of 16, so each element of A loaded into LDS feeds NT MFMAs
// from registers and the skinny operand X is the only operand re-read
// (from LDS) per row tile.  Tiles are 128 bytes of K per row (BK elements),
// double-buffered in LDS; the 16-byte granules of a row are XOR-swizzled by
// the row index, so that the 16-byte operand reads (16 rows x 4 granules per
// wave instruction) and the row-major tile stores are free of bank conflicts
// (rows padded to 144 bytes, the obvious alternative, still conflict on the
// reads).
//
// MFMA forms (gfx950):  f64 16x16x4,  f32 16x16x4,  bf16 16x16x32,
// fp8 (E4M3FN) 16x16x128 with unit block scales.  Lane l = 16 g + i supplies
// row i and K slots [g*KL, (g+1)*KL) of both operands, KL = K per MFMA / 4.
// The order in which K is visited does not change a dot product, so each lane
// reads one 16-byte vector of K from LDS and feeds it to consecutive MFMAs.
//
// BF16 and FP8 A^T X tiles are transposed in registers: a thread loads four
// consecutive rows of A (one 16-byte chunk of each), byte permutes turn them
// into one 4-element K run per column, and 8-byte (BF16) or 4-byte (FP8) LDS
// writes put these into [output row][K] rows of 128 bytes whose 16-byte
// granules are XOR-swizzled by the row, so that both these writes (at most
// two lanes per bank) and the 16-byte MFMA operand reads (none) spread over
// the banks.
//
// Output: FP32 partial sums (FP64 in F64 mode) ypart[split][row][lp]; the
// splits are added in a fixed order by the reduction kernel, so the result
// does not depend on scheduling.
#include "common.h"
#include "kernels.h"

namespace cor {

template <int PREC> struct SkCfg;
template <> struct SkCfg<P_F64> { static constexpr int BK = 16, VEC = 2; };
template <> struct SkCfg<P_F32> { static constexpr int BK = 32, VEC = 4; };
template <> struct SkCfg<P_BF16> { static constexpr int BK = 64, VEC = 8; };
template <> struct SkCfg<P_FP8> { static constexpr int BK = 128, VEC = 16; };

// Block shapes.  A X blocks in FP32/FP64: 4 waves, 128 output rows (each A
// row contributes a long contiguous K run).  A^T X blocks: 8 waves, 256
// output rows, so that every row of A a block reads is a 1 KB (FP32)
// contiguous run rather than 512 B.  BF16 A X blocks: 8 waves too, which
// halves the X tile traffic per byte of A (the X tile is as large as the A
// tile at l = 220).  Eight waves mean two per SIMD and half the register file
// each: shapes whose accumulators do not fit that (FP64 beyond 8 column
// tiles, FP32 beyond 12, FP8 beyond 9, FP8 A X) keep 4 waves -- except FP64
// beyond 8 column tiles, FP32 where it would have one wave per SIMD (A X
// beyond 9 column tiles, A^T X beyond 12) and FP8 beyond 9 (A^T X: 10, 12
// and 14, the counts that do not spill), which take 8 waves in 4 row groups
// x 2 column groups: a wave's accumulators (2 row tiles -- 4 for FP8 A^T X,
// whose register transpose wants 256-row tiles -- x half the column tiles)
// then leave room for two waves per SIMD (with one wave of 2 x NT tiles per
// SIMD the MFMA pipe waits on every tile's loads).
template <int PREC, bool TRANS> __host__ __device__ constexpr bool sk_split_cols(int nt) {
    return (PREC == P_F64 && nt >= 9) || (PREC == P_F32 && nt >= (TRANS ? 13 : 10)) ||
           (PREC == P_FP8 && nt >= 10 && (!TRANS || (nt <= 14 && nt % 2 == 0)));
}
template <int PREC, int NT, bool TRANS> __host__ __device__ constexpr int sk_waves() {
    constexpr int ntmax = PREC == P_F64 ? 8 : PREC == P_F32 ? 12 : PREC == P_FP8 ? 9 : NTMAX;
    // BF16 with at most 7 column tiles (l <= 112): 4 waves, whose smaller LDS
    // tiles let two or three blocks share a CU, so more A tiles are in flight where
    // the MFMA work per tile is too short to hide one tile's load.
    if (PREC == P_BF16 && NT <= 7) return 4;
    if (sk_split_cols<PREC, TRANS>(NT)) return 8;
    return (NT <= ntmax && (TRANS || PREC == P_BF16)) ? 8 : 4;
}
template <int PREC, int NT, bool TRANS> __host__ __device__ constexpr int sk_threads() { return 64 * sk_waves<PREC, NT, TRANS>(); }
// Waves of a block as a grid of row groups x WC column groups: each wave owns
// RT = 2 WC row tiles of 16 and ceil(NT / WC) column tiles.  BF16 with eight
// to fourteen column tiles splits the columns in two (4 x 2 waves, 64 rows x
// NT/2 columns each): the same accumulators as 32 rows x NT, but each wave
// reads 4 A and NT/2 X fragments from LDS per K step instead of 2 and NT,
// about a third less LDS traffic per MFMA.
template <int PREC, int NT, bool TRANS> __host__ __device__ constexpr int sk_wc() {
    return ((PREC == P_BF16 && NT >= 8 && NT <= 14 && sk_waves<PREC, NT, TRANS>() == 8) ||
            sk_split_cols<PREC, TRANS>(NT))
               ? 2
               : 1;
}
// Row tiles per wave: 2 WC for BF16 and FP8 A^T X (64 rows per wave with two
// column groups), 2 for the FP32 / FP64 / FP8 A X column split.
template <int PREC, int NT, bool TRANS> __host__ __device__ constexpr int sk_rt() {
    return (PREC == P_BF16 || (PREC == P_FP8 && TRANS)) ? 2 * sk_wc<PREC, NT, TRANS>() : 2;
}
template <int PREC, int NT, bool TRANS> __host__ __device__ constexpr int sk_bm() {
    return 16 * sk_rt<PREC, NT, TRANS>() * (sk_waves<PREC, NT, TRANS>() / sk_wc<PREC, NT, TRANS>());
}
// Non-transposed A tiles and all X tiles: rows of 128 bytes of K (eight
// 16-byte granules, no padding); granule g of row r sits in slot g ^ s(r).
// s(r) = r & 7 makes the FP32 / FP64 / BF16 fragment reads (16 rows x 4
// consecutive granules per wave instruction) free of bank conflicts; the FP8
// reads (granules 2 g and 2 g + 1 of 16 rows) need row bit 3 as well,
// s(r) = (r ^ (r >> 3)) & 7.  (Both were picked by measuring the bank-conflict
// counter over all linear maps from row bits to slots; the row-major tile
// stores are conflict-free with any of them.)
constexpr int ROWB = 128;
template <int PREC> __device__ __forceinline__ int sk_off(int r, int g) {
    const int sw = PREC == P_FP8 ? (r ^ (r >> 3)) : r;
    return r * ROWB + 16 * (g ^ (sw & 7));
}

template <int PREC, int NT, bool TRANS>
__host__ __device__ constexpr int sk_a_bytes() {
    // Non-transposed (and 1/2-byte transposed) tiles: BM rows of 128 bytes.
    // F32/F64 transposed tiles: BK rows of BM elements (+16 bytes).
    return (TRANS && (PREC == P_F32 || PREC == P_F64))
               ? SkCfg<PREC>::BK * (sk_bm<PREC, NT, TRANS>() * PrecT<PREC>::SZ + 16)
               : sk_bm<PREC, NT, TRANS>() * ROWB;
}

template <int PREC, int NT, bool TRANS>
__host__ __device__ constexpr int sk_lds_bytes() {
    return 2 * (sk_a_bytes<PREC, NT, TRANS>() + NT * 16 * ROWB);
}

// Swizzled [output row][K] layout of a transposed BF16 / FP8 tile: row r holds
// 128 bytes of K (eight 16-byte granules); granule g sits in slot
// g ^ at_swz(r).  BF16: a thread's columns are 8 rows apart, and the term
// r >> 3 spreads the rows one 8-byte store instruction writes.  FP8: a
// thread's columns are 16 rows apart (r >> 4 spreads those); row bits 1-3 map
// to slot bits 1, 2, 0, which keeps the FP8 fragment reads conflict-free, and
// row bit 0 is left out so that rows 2 i and 2 i + 1 share a slot: their
// 4-byte stores then sit a constant 128 bytes apart and pair into one
// two-address store instruction.
__device__ __forceinline__ int at_swz_bf16(int r) { return ((r >> 1) ^ (r >> 3)) & 7; }
__device__ __forceinline__ int at_swz_fp8(int r) { return ((r & 6) ^ ((r >> 3) & 1) ^ (r >> 4)) & 7; }
constexpr int AT_ROWB = 128;

// Sixteen zero bytes in global memory: out-of-range rows of a full tile are
// loaded from here (an address select, not a branch).  Never written.
__device__ __align__(16) uint32_t g_zero16[4] = {0u, 0u, 0u, 0u};

typedef const __attribute__((address_space(1))) i32x4 gi32x4;

// 16-byte global load with element-wise bounds (zero fill) when needed.
template <typename T, int VEC>
__device__ __forceinline__ i32x4 load16(const T* p, int64_t valid, bool vec_ok) {
    i32x4 v;
    if (vec_ok && valid >= VEC) {
        v = *reinterpret_cast<const i32x4*>(p);
    } else {
        union { i32x4 v; T e[VEC]; } u;
#pragma unroll
        for (int e = 0; e < VEC; e++) u.e[e] = (e < valid) ? p[e] : T(0);
        v = u.v;
    }
    return v;
}

template <int PREC, int NT, bool TRANS>
__global__ __launch_bounds__((sk_threads<PREC, NT, TRANS>())) void k_sketch(const Prob* __restrict__ probs,
                                                       const int32_t* __restrict__ pidx,
                                                       const int32_t* __restrict__ toff, int cnt,
                                                       int iter) {
    typedef typename PrecT<PREC>::T T;
    typedef typename PrecT<PREC>::Acc Acc;
    constexpr int SK_THREADS = sk_threads<PREC, NT, TRANS>();
    constexpr int SK_WC = sk_wc<PREC, NT, TRANS>();
    constexpr int SK_RT = sk_rt<PREC, NT, TRANS>();
    constexpr int NTW = (NT + SK_WC - 1) / SK_WC;  // column tiles per wave
    static_assert(SK_RT * 16 * (SK_THREADS / 64 / SK_WC) == sk_bm<PREC, NT, TRANS>(), "rows per block");
    constexpr int SK_BM = sk_bm<PREC, NT, TRANS>();
    constexpr int SZ = PrecT<PREC>::SZ;
    constexpr int BK = SkCfg<PREC>::BK;
    constexpr int VEC = SkCfg<PREC>::VEC;
    constexpr int ABYTES = sk_a_bytes<PREC, NT, TRANS>();
    constexpr int XBYTES = NT * 16 * ROWB;

    extern __shared__ __align__(16) unsigned char smem[];

    const int j = find_group(toff, cnt, blockIdx.x);
    const Prob& P = probs[pidx[j]];
    if (iter > P.q) return;
    if (iter < 0 && P.mmode != M_EXPLICIT) return;  // the pass A Q2 of eq. (14)
    const int local = blockIdx.x - toff[j];

    const int64_t rows = TRANS ? P.n : P.m;    // output rows
    const int64_t K = TRANS ? P.m : P.n;       // contraction length
    const int nrb = (int)((rows + SK_BM - 1) / SK_BM);
    // Blocks go to the eight XCDs in turn (block b to XCD b mod 8), each with
    // its own L2.  With 8 K splits, split = b mod 8: the blocks of an XCD all
    // read the same slice of the skinny operand, which is then fetched into
    // one L2 instead of all eight.
    const int nsplit = TRANS ? P.s_atx : P.s_ax;
    const int rb = nsplit == 8 ? local >> 3 : local % nrb;
    const int split = nsplit == 8 ? local & 7 : local / nrb;
    const int64_t kc = TRANS ? P.kc_atx : P.kc_ax;
    const int64_t kbeg = (int64_t)split * kc;
    const int64_t kend = min(K, kbeg + kc);
    const int64_t row0 = (int64_t)rb * SK_BM;
    const int lp = P.lp;

    const T* __restrict__ A = reinterpret_cast<const T*>(P.A);
    const T* __restrict__ X = reinterpret_cast<const T*>(TRANS ? P.qop : P.xop);
    const int64_t ldx = TRANS ? P.ldq : P.ldx;
    const int64_t lda = P.lda;
    const bool avec = P.avec != 0;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int li = lane & 15;
    const int lg = lane >> 4;
    constexpr bool ATRANS_SCALAR = TRANS && (PREC == P_F32 || PREC == P_F64);
    constexpr bool ATRANS_BF16 = TRANS && PREC == P_BF16;
    constexpr bool ATRANS_FP8 = TRANS && PREC == P_FP8;
    constexpr int AROWB = SK_BM * SZ + 16;  // row stride of a transposed F32/F64 tile

    // ---------------- global -> register staging ----------------
    // A tile: non-transposed: SK_BM rows x 8 chunks;  transposed: BK rows x
    // (SK_BM*SZ/16) chunks.  X tile: NT*16 rows x 8 chunks.
    constexpr int A_CHUNKS = SK_BM * BK * SZ / 16;
    constexpr int A_LD = A_CHUNKS / SK_THREADS;
    constexpr int X_CHUNKS = NT * 16 * 8;
    constexpr int X_LD = (X_CHUNKS + SK_THREADS - 1) / SK_THREADS;
    i32x4 ra[A_LD];
    i32x4 rx[X_LD];
    // Chunk t of this thread in a transposed tile: K row a_kr(t), column chunk
    // a_ch.  BF16 / FP8: K rows 4 q .. 4 q + 3 per thread (transposed in
    // registers).  BF16 256-row tiles: the 32 lanes of a half wave take 16 column chunks of
    // two K-row groups, so that their 8-byte LDS writes pair up in the
    // 16-byte granules.
    constexpr int CPR = SK_BM * SZ / 16;  // chunks per A row segment (transposed)
    if constexpr (ATRANS_BF16 || ATRANS_FP8)
        static_assert(A_LD == 4 && SK_THREADS / CPR * 4 == BK, "4 K rows per thread");
    // BF16 256 x 64 tiles (CPR = 32, 512 threads): the paired-lane map
    constexpr bool BPAIR = ATRANS_BF16 && CPR == 32 && SK_THREADS == 512;
    const int bq = BPAIR ? ((tid >> 6) << 1) | ((tid >> 4) & 1) : tid / CPR;  // K-row group
    const int bch = BPAIR ? (tid & 15) | (((tid >> 5) & 1) << 4) : tid % CPR;  // column chunk
    auto a_kr = [&](int t) {
        if constexpr (ATRANS_BF16 || ATRANS_FP8) return 4 * bq + t;
        else return (tid + t * SK_THREADS) / CPR;
    };
    auto a_ch = [&](int t) {
        if constexpr (ATRANS_BF16 || ATRANS_FP8) return bch;
        else return (tid + t * SK_THREADS) % CPR;
    };

    // Full tiles (every K of the tile inside the split, 16-byte aligned rows,
    // and for the transposed pass every output row inside the matrix) load
    // with unconditional 16-byte global loads; rows past the matrix read the
    // zero block.  Straight-line loads let the compiler keep them all in
    // flight while the previous tile's MFMAs run.  Other tiles take the
    // element-wise path below.
    // A transposed tile whose 16-byte chunks are each wholly inside or wholly
    // past the last output row also takes the full path (chunks past it read
    // the zero block), so the last row block is not slower than the others.
    const bool rows_full = !TRANS || row0 + SK_BM <= rows || rows % VEC == 0;
    auto load_tile_full = [&](int64_t k0) {
        gi32x4* z16 = (gi32x4*)g_zero16;
        if constexpr (!TRANS) {
#pragma unroll
            for (int t = 0; t < A_LD; t++) {
                const int c = tid + t * SK_THREADS;
                const int r = c >> 3, ch = c & 7;
                const int64_t gr = row0 + r;
                const T* a = A + min(gr, rows - 1) * lda + k0 + ch * VEC;
                ra[t] = *(gr < rows ? (gi32x4*)a : z16);
            }
        } else {
#pragma unroll
            for (int t = 0; t < A_LD; t++) {
                const int kr = a_kr(t), ch = a_ch(t);
                const int64_t gc = row0 + ch * VEC;
                const T* a = A + (k0 + kr) * lda + min(gc, rows - VEC);
                ra[t] = *(gc < rows ? (gi32x4*)a : z16);
            }
        }
#pragma unroll
        for (int t = 0; t < X_LD; t++) {
            // chunks past X_CHUNKS repeat the last one (their LDS store is skipped)
            const int c = min(tid + t * SK_THREADS, X_CHUNKS - 1);
            const int r = c >> 3, ch = c & 7;
            // X is [lp][ldx] with zeros past the factor: every K < ldx is readable.
            const T* x = X + (int64_t)min(r, lp - 1) * ldx + k0 + ch * VEC;
            rx[t] = *(gi32x4*)x;
        }
    };
    auto load_tile = [&](int64_t k0) {
        if (avec && rows_full && k0 + BK <= kend) {
            load_tile_full(k0);
            return;
        }
        if constexpr (!TRANS) {
#pragma unroll
            for (int t = 0; t < A_LD; t++) {
                int c = tid + t * SK_THREADS;
                int r = c >> 3, ch = c & 7;
                int64_t gr = row0 + r;
                int64_t gk = k0 + ch * VEC;
                if (gr < rows && gk < kend)
                    ra[t] = load16<T, VEC>(A + gr * lda + gk, kend - gk, avec);
                else
                    ra[t] = i32x4{0, 0, 0, 0};
            }
        } else {
#pragma unroll
            for (int t = 0; t < A_LD; t++) {
                const int kr = a_kr(t), ch = a_ch(t);
                int64_t gk = k0 + kr;
                int64_t gc = row0 + ch * VEC;
                if (gk < kend && gc < rows)
                    ra[t] = load16<T, VEC>(A + gk * lda + gc, rows - gc, avec);
                else
                    ra[t] = i32x4{0, 0, 0, 0};
            }
        }
#pragma unroll
        for (int t = 0; t < X_LD; t++) {
            int c = tid + t * SK_THREADS;
            int r = c >> 3, ch = c & 7;
            int64_t gk = k0 + ch * VEC;
            if (c < X_CHUNKS && r < lp && gk < kend)
                rx[t] = load16<T, VEC>(X + (int64_t)r * ldx + gk, kend - gk, true);
            else
                rx[t] = i32x4{0, 0, 0, 0};
        }
    };

    auto store_tile = [&](int buf) {
        unsigned char* As = smem + buf * (ABYTES + XBYTES);
        unsigned char* Xs = As + ABYTES;
        if constexpr (!TRANS) {
#pragma unroll
            for (int t = 0; t < A_LD; t++) {
                int c = tid + t * SK_THREADS;
                int r = c >> 3, ch = c & 7;
                *reinterpret_cast<i32x4*>(As + sk_off<PREC>(r, ch)) = ra[t];
            }
        } else if constexpr (ATRANS_SCALAR) {
#pragma unroll
            for (int t = 0; t < A_LD; t++)
                *reinterpret_cast<i32x4*>(As + a_kr(t) * AROWB + a_ch(t) * 16) = ra[t];
        } else if constexpr (ATRANS_BF16) {
            // ra[t] = columns 8 ch .. 8 ch + 7 of K row k0 + t (two per dword);
            // column e becomes the K run k0 .. k0 + 3 of output row 8 ch + e.
            const int q = bq, ch = bch;
            const int g = q >> 1;  // 16-byte granule of K row 4 q
#pragma unroll
            for (int e = 0; e < 8; e++) {
                const int d = e >> 1;
                const uint32_t sel = (e & 1) ? 0x07060302u : 0x05040100u;
                const uint32_t lo = __builtin_amdgcn_perm((uint32_t)ra[1][d], (uint32_t)ra[0][d], sel);
                const uint32_t hi = __builtin_amdgcn_perm((uint32_t)ra[3][d], (uint32_t)ra[2][d], sel);
                const int r = ch * 8 + e;
                *reinterpret_cast<uint2*>(As + r * AT_ROWB + 16 * (g ^ at_swz_bf16(r)) + 8 * (q & 1)) =
                    make_uint2(lo, hi);
            }
        } else {
            // FP8: ra[t] = columns 16 ch .. 16 ch + 15 of K row k0 + t; a 4 x 4
            // byte transpose per dword gives column e the K run k0 .. k0 + 3.
            const int q = bq, ch = bch;
            const int g = q >> 2;  // 16-byte granule of K row 4 q
#pragma unroll
            for (int d = 0; d < 4; d++) {
                const uint32_t x01 = __builtin_amdgcn_perm((uint32_t)ra[1][d], (uint32_t)ra[0][d], 0x05010400u);
                const uint32_t y01 = __builtin_amdgcn_perm((uint32_t)ra[1][d], (uint32_t)ra[0][d], 0x07030602u);
                const uint32_t x23 = __builtin_amdgcn_perm((uint32_t)ra[3][d], (uint32_t)ra[2][d], 0x05010400u);
                const uint32_t y23 = __builtin_amdgcn_perm((uint32_t)ra[3][d], (uint32_t)ra[2][d], 0x07030602u);
                const uint32_t o[4] = {__builtin_amdgcn_perm(x23, x01, 0x05040100u),
                                       __builtin_amdgcn_perm(x23, x01, 0x07060302u),
                                       __builtin_amdgcn_perm(y23, y01, 0x05040100u),
                                       __builtin_amdgcn_perm(y23, y01, 0x07060302u)};
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const int r = ch * 16 + 4 * d + b;
                    *reinterpret_cast<uint32_t*>(As + r * AT_ROWB + 16 * (g ^ at_swz_fp8(r)) + 4 * (q & 3)) = o[b];
                }
            }
        }
#pragma unroll
        for (int t = 0; t < X_LD; t++) {
            int c = tid + t * SK_THREADS;
            if (c < X_CHUNKS) {
                int r = c >> 3, ch = c & 7;
                *reinterpret_cast<i32x4*>(Xs + sk_off<PREC>(r, ch)) = rx[t];
            }
        }
    };

    // ---------------- accumulators ----------------
    typedef typename std::conditional<PREC == P_F64, f64x4, f32x4>::type AccV;
    AccV acc[SK_RT][NTW];
#pragma unroll
    for (int r = 0; r < SK_RT; r++)
#pragma unroll
        for (int c = 0; c < NTW; c++)
#pragma unroll
            for (int e = 0; e < 4; e++) acc[r][c][e] = Acc(0);

    constexpr int WRN = SK_THREADS / 64 / SK_WC;  // row groups
    const int wrow = (wave % WRN) * (SK_RT * 16);
    const int c0 = SK_WC == 1 ? 0 : (wave / WRN) * NTW;  // first column tile of this wave

    auto compute_tile = [&](int buf) {
        const unsigned char* As = smem + buf * (ABYTES + XBYTES);
        const unsigned char* Xs = As + ABYTES;
        if constexpr (PREC == P_F32 || PREC == P_F64) {
            // One 16-byte vector holds VEC consecutive K of one lane: VEC MFMAs.
#pragma unroll
            for (int ss = 0; ss < BK / (4 * VEC); ss++) {
                const int kk = ss * 4 * VEC + lg * VEC;  // this lane's first K slot
                T av[SK_RT][VEC];
#pragma unroll
                for (int r = 0; r < SK_RT; r++) {
                    const int orow = wrow + r * 16 + li;
                    if constexpr (!TRANS) {
                        union { i32x4 v; T e[VEC]; } u;
                        u.v = *reinterpret_cast<const i32x4*>(As + sk_off<PREC>(orow, kk * SZ / 16));
#pragma unroll
                        for (int e = 0; e < VEC; e++) av[r][e] = u.e[e];
                    } else {
                        // F32/F64 tiles stay [K][row] in LDS (a transposing
                        // store of 4-byte elements costs more than these reads)
#pragma unroll
                        for (int e = 0; e < VEC; e++)
                            av[r][e] = *reinterpret_cast<const T*>(As + (kk + e) * AROWB + orow * SZ);
                    }
                }
                // All of the wave's column tiles' operand vectors first, then
                // MFMAs ordered so that the RT*NTW accumulators are visited
                // round-robin: consecutive MFMAs never update the same
                // accumulator.  (A second column group past NT repeats the
                // last tile; its accumulators are never stored.)
                T bv[NTW][VEC];
#pragma unroll
                for (int c = 0; c < NTW; c++) {
                    const int cc = SK_WC == 1 ? c : min(c0 + c, NT - 1);
                    union { i32x4 v; T e[VEC]; } b;
                    b.v = *reinterpret_cast<const i32x4*>(Xs + sk_off<PREC>(cc * 16 + li, kk * SZ / 16));
#pragma unroll
                    for (int e = 0; e < VEC; e++) bv[c][e] = b.e[e];
                }
#pragma unroll
                for (int e = 0; e < VEC; e++)
#pragma unroll
                    for (int c = 0; c < NTW; c++)
#pragma unroll
                        for (int r = 0; r < SK_RT; r++) {
                            if constexpr (PREC == P_F32)
                                acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[r][e], bv[c][e], acc[r][c], 0, 0, 0);
                            else
                                acc[r][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[r][e], bv[c][e], acc[r][c], 0, 0, 0);
                        }
            }
        } else if constexpr (PREC == P_BF16) {
#pragma unroll
            for (int ss = 0; ss < BK / 32; ss++) {
                const int kk = ss * 32 + lg * 8;
                bf16x8 av[SK_RT];
#pragma unroll
                for (int r = 0; r < SK_RT; r++) {
                    const int orow = wrow + r * 16 + li;
                    if constexpr (TRANS)
                        av[r] = *reinterpret_cast<const bf16x8*>(As + orow * AT_ROWB + 16 * ((kk >> 3) ^ at_swz_bf16(orow)));
                    else
                        av[r] = *reinterpret_cast<const bf16x8*>(As + sk_off<PREC>(orow, kk >> 3));
                }
#pragma unroll
                for (int c = 0; c < NTW; c++) {
                    const int cc = c0 + c;  // column tile (wave-uniform test)
                    if (SK_WC > 1 && cc >= NT) break;
                    bf16x8 bv = *reinterpret_cast<const bf16x8*>(Xs + sk_off<PREC>(cc * 16 + li, kk >> 3));
#pragma unroll
                    for (int r = 0; r < SK_RT; r++)
                        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[r], bv, acc[r][c], 0, 0, 0);
                }
            }
        } else {  // FP8: one MFMA consumes 32 consecutive K bytes (granules 2 lg, 2 lg + 1) per lane
            i32x8 av[SK_RT];
#pragma unroll
            for (int r = 0; r < SK_RT; r++) {
                const int orow = wrow + r * 16 + li;
                i32x4 lo, hi;
                if constexpr (TRANS) {
                    const unsigned char* p = As + orow * AT_ROWB;
                    const int sw = at_swz_fp8(orow);
                    lo = *reinterpret_cast<const i32x4*>(p + 16 * ((2 * lg) ^ sw));
                    hi = *reinterpret_cast<const i32x4*>(p + 16 * ((2 * lg + 1) ^ sw));
                } else {
                    lo = *reinterpret_cast<const i32x4*>(As + sk_off<PREC>(orow, 2 * lg));
                    hi = *reinterpret_cast<const i32x4*>(As + sk_off<PREC>(orow, 2 * lg + 1));
                }
                av[r] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
            }
#pragma unroll
            for (int c = 0; c < NTW; c++) {
                const int cc = c0 + c;  // column tile (wave-uniform test)
                if (SK_WC > 1 && cc >= NT) break;
                i32x4 lo = *reinterpret_cast<const i32x4*>(Xs + sk_off<PREC>(cc * 16 + li, 2 * lg));
                i32x4 hi = *reinterpret_cast<const i32x4*>(Xs + sk_off<PREC>(cc * 16 + li, 2 * lg + 1));
                i32x8 bv = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
#pragma unroll
                for (int r = 0; r < SK_RT; r++)
                    acc[r][c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(
                        av[r], bv, acc[r][c], 0, 0, 0, 127, 0, 127);
            }
        }
    };

    // ---------------- main loop: double-buffered LDS ----------------
    const int ntile = (int)((kend - kbeg + BK - 1) / BK);
    if (ntile > 0) {
        load_tile(kbeg);
        store_tile(0);
        __syncthreads();
        for (int t = 0; t < ntile; t++) {
            const bool more = (t + 1) < ntile;
            if (more) load_tile(kbeg + (int64_t)(t + 1) * BK);
            compute_tile(t & 1);
            if (more) store_tile((t + 1) & 1);
            __syncthreads();
        }
    }

    // ---------------- epilogue: partial sums ----------------
    Acc* __restrict__ out = reinterpret_cast<Acc*>(P.ypart) + (int64_t)split * rows * lp;
#pragma unroll
    for (int r = 0; r < SK_RT; r++)
#pragma unroll
        for (int c = 0; c < NTW; c++) {
            const int cc = c0 + c;
            if (SK_WC > 1 && cc >= NT) break;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                // f32 forms: (row 4g + e, col i); f64 form: (row g + 4e, col i)
                int tr = (PREC == P_F64) ? (lg + 4 * e) : (4 * lg + e);
                int64_t gr = row0 + wrow + r * 16 + tr;
                if (gr < rows) out[gr * lp + cc * 16 + li] = acc[r][c][e];
            }
        }
}

// ---------------------------------------------------------------------------
// Host launchers: one template instance per (format, column tiles, side).
// ---------------------------------------------------------------------------
template <int PREC, int NT, bool TRANS>
static hipError_t launch_nt(const LaunchGroup& g, int iter, hipStream_t s) {
    constexpr int lds = sk_lds_bytes<PREC, NT, TRANS>();
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)k_sketch<PREC, NT, TRANS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    hipLaunchKernelGGL((k_sketch<PREC, NT, TRANS>), dim3(g.blocks), dim3(sk_threads<PREC, NT, TRANS>()), lds, s,
                       g.probs, g.pidx, g.toff, g.count, iter);
    return hipGetLastError();
}

template <int PREC, bool TRANS>
static hipError_t launch_prec(const LaunchGroup& g, int nt, int iter, hipStream_t s) {
    switch (nt) {
#define NT_CASE(N) case N: return launch_nt<PREC, N, TRANS>(g, iter, s);
        NT_CASE(1) NT_CASE(2) NT_CASE(3) NT_CASE(4) NT_CASE(5) NT_CASE(6) NT_CASE(7) NT_CASE(8)
        NT_CASE(9) NT_CASE(10) NT_CASE(11) NT_CASE(12) NT_CASE(13) NT_CASE(14) NT_CASE(15)
        NT_CASE(16) NT_CASE(17)
#undef NT_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sketch(int prec, bool trans, int nt, const LaunchGroup& g, int iter,
                         hipStream_t s) {
    if (g.blocks <= 0) return hipSuccess;
    switch (prec) {
        case P_F64: return trans ? launch_prec<P_F64, true>(g, nt, iter, s) : launch_prec<P_F64, false>(g, nt, iter, s);
        case P_F32: return trans ? launch_prec<P_F32, true>(g, nt, iter, s) : launch_prec<P_F32, false>(g, nt, iter, s);
        case P_BF16: return trans ? launch_prec<P_BF16, true>(g, nt, iter, s) : launch_prec<P_BF16, false>(g, nt, iter, s);
        case P_FP8: return trans ? launch_prec<P_FP8, true>(g, nt, iter, s) : launch_prec<P_FP8, false>(g, nt, iter, s);
    }
    return hipErrorInvalidValue;
}

template <int PREC, bool TRANS>
static int rows_nt(int nt) {
    switch (nt) {
#define NT_CASE(N) case N: return sk_bm<PREC, N, TRANS>();
        NT_CASE(1) NT_CASE(2) NT_CASE(3) NT_CASE(4) NT_CASE(5) NT_CASE(6) NT_CASE(7) NT_CASE(8)
        NT_CASE(9) NT_CASE(10) NT_CASE(11) NT_CASE(12) NT_CASE(13) NT_CASE(14) NT_CASE(15)
        NT_CASE(16) NT_CASE(17)
#undef NT_CASE
        default: return 128;
    }
}

int sketch_rows_per_block(int prec, int nt, bool trans) {
    switch (prec) {
        case P_F64: return trans ? rows_nt<P_F64, true>(nt) : rows_nt<P_F64, false>(nt);
        case P_F32: return trans ? rows_nt<P_F32, true>(nt) : rows_nt<P_F32, false>(nt);
        case P_BF16: return trans ? rows_nt<P_BF16, true>(nt) : rows_nt<P_BF16, false>(nt);
        default: return trans ? rows_nt<P_FP8, true>(nt) : rows_nt<P_FP8, false>(nt);
    }
}

int sketch_k_tile(int prec) {
    switch (prec) {
        case P_F64: return SkCfg<P_F64>::BK;
        case P_F32: return SkCfg<P_F32>::BK;
        case P_BF16: return SkCfg<P_BF16>::BK;
        default: return SkCfg<P_FP8>::BK;
    }
}

}  // namespace cor
