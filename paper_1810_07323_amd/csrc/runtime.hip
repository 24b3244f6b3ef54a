// Host runtime of libcorutv: plans (workspace layout, grouped launch tables,
// the stage sequence of Alg. 3), the C ABI of include/cor_utv.h, and kernel
// timing for roofline reports.  The served path lives in server.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/cor_utv.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

namespace cor {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

cor_status fail(cor_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

cor_status hip_fail(hipError_t e, const char* what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return COR_E_DEVICE;
}

#define HIPCHK(expr)                                                      \
    do {                                                                  \
        hipError_t e_ = (expr);                                           \
        if (e_ != hipSuccess) return hip_fail(e_, #expr);                 \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel timing (roofline reports)
// ---------------------------------------------------------------------------
struct ProfState {
    std::mutex mu;
    int on = 0;  // bit 0: the two-pass kernels (A X, A^T X); bit 1: the fused power step
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> free_ev;
    double bytes = 0.0, flops = 0.0;
    int64_t launches = 0;
};
static ProfState g_prof;

static void prof_begin(hipStream_t s, hipEvent_t* a, hipEvent_t* b, int kind) {
    *a = *b = nullptr;
    if (!(g_prof.on & kind)) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (g_prof.free_ev.empty()) {
        hipEvent_t x, y;
        if (hipEventCreate(&x) != hipSuccess) return;
        if (hipEventCreate(&y) != hipSuccess) return;
        g_prof.free_ev.push_back({x, y});
    }
    auto pr = g_prof.free_ev.back();
    g_prof.free_ev.pop_back();
    *a = pr.first;
    *b = pr.second;
    (void)hipEventRecord(*a, s);
}

static void prof_end(hipStream_t s, hipEvent_t a, hipEvent_t b, double bytes, double flops) {
    if (!a) return;
    (void)hipEventRecord(b, s);
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.pending.push_back({a, b});
    g_prof.bytes += bytes;
    g_prof.flops += flops;
    g_prof.launches += 1;
}

// ---------------------------------------------------------------------------
// Plans
// ---------------------------------------------------------------------------
static int64_t roundup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }
static int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
static int prec_size(int p) { return p == P_F64 ? 8 : p == P_F32 ? 4 : p == P_BF16 ? 2 : 1; }

enum {
    O_XOP, O_QOP, O_XSC, O_QSC, O_YPART, O_Y, O_QA, O_Q1, O_Q2, O_GPART, O_G, O_R, O_RINV,
    O_RACC, O_R2, O_QT, O_TAU, O_REP, O_FLAGS, O_PERM, O_SCPART, O_MX, O_R1, O_XK, O_AT, O_TT,
    O_COUNT
};

struct Layout {
    // per-problem sizes
    int32_t l, lp, nt;
    int64_t ldx, ldq;
    int32_t s_ax, s_atx, s_f;
    int64_t kc_ax, kc_atx, kc_f;
    int32_t rb_m, rb_n, gb_m, gb_n;
    size_t off[O_COUNT];
    size_t total;
};


// K splits of a pass: about `target` blocks in all (row blocks x splits, never
// more), at most 8 splits (64 with fewer than 32 row blocks), each split at least 16 K tiles long in BF16 and FP8
// and 4 in FP32 and FP64.  The layout of
// a problem depends on its own shape only, never on what it is batched with,
// so a decomposition gives bitwise the same result alone, batched or served.
static void split_k(int64_t rows, int64_t K, int bk, int target, int prec, int nt, bool trans,
                    int32_t* s, int64_t* kc) {
    const int64_t nrb = cdiv(rows, sketch_rows_per_block(prec, nt, trans));
    // Few output row blocks (the transposed pass of a tall matrix: n small,
    // K = m long) need more splits to fill the GPU: up to 64 there.
    const int64_t cap = nrb >= 32 ? 8 : 64;
    int64_t sp = std::min<int64_t>(cap, std::max<int64_t>(1, target / nrb));
    // Short BF16 and FP8 splits cost more in prologue, epilogue and partial
    // sums than they win (small problems of a batch); an FP32 or FP64 tile
    // holds 2-4x fewer elements of K, so more MFMA work, and small problems
    // alone on the GPU gain from the shorter chain of tiles.
    const int64_t min_tiles = (prec == P_BF16 || prec == P_FP8) ? 16 : 4;
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, K / (min_tiles * bk)));
    int64_t c = roundup(cdiv(K, sp), bk);
    *kc = c;
    *s = (int32_t)cdiv(K, c);
}

// Row chunks of the FP8 operand-scale column maxima (at least 128 rows each).
static int32_t scale_chunks(int64_t rows) {
    return (int32_t)std::min<int64_t>(SCALE_CHUNKS, std::max<int64_t>(1, cdiv(rows, 128)));
}

static int gram_side(int lp) { return (lp / 16 + 1) / 2; }  // 2 x 2 tile groups per side
static int gram_groups(int lp) {  // blocks per row chunk: the upper 2 x 2 tile groups
    const int ns = gram_side(lp);
    return ns * (ns + 1) / 2;
}

static void gram_chunks(int64_t rows, int lp, int target, int32_t* rb, int32_t* gb) {
    // Row chunks of the Gram partial sums: about `target` blocks per problem
    // (chunks x tiles), at least 256 rows per chunk (64 per wave).  Fewer
    // chunks mean fewer l x l partials to write and reduce, and small
    // problems of a batch fewer blocks.
    // A multiple of 8 chunks where there are 8 or more lets the Gram kernel
    // keep each chunk's blocks on one XCD (one L2).
    const int ngroups = gram_groups(lp);
    int64_t g = std::max<int64_t>(1, cdiv(target, ngroups));
    g = std::min<int64_t>(g, std::max<int64_t>(1, cdiv(rows, 256)));
    if (g >= 8) g = g / 8 * 8;
    int64_t r = roundup(cdiv(rows, g), 4);
    *rb = (int32_t)r;
    *gb = (int32_t)cdiv(rows, r);
}

// Blocks per pass of a single decomposition: one resident set of the sketch
// kernel (256 CUs x 2 blocks) by default; COR_SPLIT_TARGET overrides it for
// tuning.
static int sketch_block_target() {
    static int t = [] {
        const char* e = getenv("COR_SPLIT_TARGET");
        const int v = e ? atoi(e) : 0;
        return v >= 16 ? v : 512;
    }();
    return t;
}

// Leading dimension (elements) of the transposed copy of A behind a ULV
// request: rows of 16-byte multiples.
static int64_t at_ld(int64_t n, int prec) { return roundup(n, 16); }

// ---------------------------------------------------------------------------
// Split tuning table: (m, n, l, prec) of the matrix the passes read -> the K
// splits of A X and A^T X.  Filled by cor_tune (measured on the caller's
// matrix) or from a JSON file (cor_tune_load, or the file named by
// COR_TUNE_FILE, read at the first plan); a plan for a tuned shape uses its
// splits, every other shape the fixed rule of split_k.  A shape's layout
// still depends on nothing but the shape and the table, so a problem gives
// the same result alone, batched or served.
// ---------------------------------------------------------------------------
struct TuneKey {
    int64_t m, n;
    int32_t l, prec;
    bool operator<(const TuneKey& o) const {
        return std::tie(m, n, l, prec) < std::tie(o.m, o.n, o.l, o.prec);
    }
};
struct TuneVal {
    int32_t s_ax, s_atx;
    double us_ax, us_atx;
};
static std::mutex g_tune_mu;
static std::map<TuneKey, TuneVal> g_tune;
static bool g_tune_env = false;
static thread_local int32_t g_force_ax = 0, g_force_atx = 0;  // the tuner's candidates
cor_status tune_load_file(const char* path);

static bool tuned_splits(int64_t m, int64_t n, int32_t l, int prec, int32_t* s_ax,
                         int32_t* s_atx) {
    if (g_force_ax > 0 || g_force_atx > 0) {
        *s_ax = g_force_ax;
        *s_atx = g_force_atx;
        return true;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_tune_env) {
        g_tune_env = true;
        const char* f = getenv("COR_TUNE_FILE");
        if (f && *f) {
            g_tune_mu.unlock();
            (void)tune_load_file(f);
            g_tune_mu.lock();
        }
    }
    auto it = g_tune.find(TuneKey{m, n, l, prec});
    if (it == g_tune.end()) return false;
    *s_ax = it->second.s_ax;
    *s_atx = it->second.s_atx;
    return true;
}

// s splits of K (> 0) in whole K tiles; 0 keeps the rule's choice.
static void apply_splits(int64_t K, int bk, int32_t s, int32_t* sp, int64_t* kc) {
    if (s <= 0) return;
    s = std::min<int32_t>(s, 64);
    const int64_t c = roundup(cdiv(K, s), bk);
    *kc = c;
    *sp = (int32_t)cdiv(K, c);
}

// Row splits of the fused power step: one block per CU (the kernel holds
// its n x lp partial sum in LDS), whole chunks of ATA_ROWS rows each.
static void fused_splits(int64_t m, int32_t* s, int64_t* kc) {
    const int64_t sp = std::max<int64_t>(1, std::min<int64_t>(256, cdiv(m, ATA_ROWS)));
    *kc = roundup(cdiv(m, sp), ATA_ROWS);
    *s = (int32_t)cdiv(m, *kc);
}

// m, n are the dimensions of the matrix the passes read (A^T for ULV).
static Layout make_layout(int64_t m, int64_t n, int32_t l, int prec, int sketch_target,
                          int gram_target, int mmode = M_R2T, int ulv = 0, int fused = 0) {
    Layout L;
    L.l = l;
    L.lp = (int32_t)roundup(l, 16);
    L.nt = L.lp / 16;
    L.ldx = roundup(n, 64);
    L.ldq = roundup(m, 64);
    const int bk = sketch_k_tile(prec);
    // 8-wave blocks are twice as large (one per CU at a time): half the target
    split_k(m, n, bk,
            sketch_rows_per_block(prec, L.nt, false) > 128 ? sketch_target / 2 : sketch_target,
            prec, L.nt, false, &L.s_ax, &L.kc_ax);
    split_k(n, m, bk,
            sketch_rows_per_block(prec, L.nt, true) > 128 ? sketch_target / 2 : sketch_target,
            prec, L.nt, true, &L.s_atx, &L.kc_atx);
    {
        int32_t ta = 0, tt = 0;
        if (tuned_splits(m, n, l, prec, &ta, &tt)) {
            apply_splits(n, bk, ta, &L.s_ax, &L.kc_ax);
            apply_splits(m, bk, tt, &L.s_atx, &L.kc_atx);
        }
    }
    gram_chunks(m, L.lp, gram_target, &L.rb_m, &L.gb_m);
    gram_chunks(n, L.lp, gram_target, &L.rb_n, &L.gb_n);
    L.s_f = 0;
    L.kc_f = 0;
    if (fused) fused_splits(m, &L.s_f, &L.kc_f);
    const int sz = prec_size(prec);
    const int acc = prec == P_F64 ? 8 : 4;
    size_t sizes[O_COUNT];
    sizes[O_XOP] = (size_t)L.lp * L.ldx * sz;
    sizes[O_QOP] = (size_t)L.lp * L.ldq * sz;
    sizes[O_XSC] = (size_t)L.lp * 4;
    sizes[O_QSC] = (size_t)L.lp * 4;
    sizes[O_YPART] = (size_t)std::max({(int64_t)L.s_ax * m, (int64_t)L.s_atx * n,
                                       (int64_t)L.s_f * n}) * L.lp * acc;
    const int64_t mx = std::max(m, n);
    sizes[O_Y] = (size_t)mx * l * 8;
    sizes[O_QA] = (size_t)mx * l * 8;
    sizes[O_Q1] = (size_t)m * l * 8;
    sizes[O_Q2] = (size_t)n * l * 8;
    // Gram partials; eq. (18) also solves in them (an l x 2l work matrix)
    sizes[O_GPART] = (size_t)std::max(std::max(L.gb_m, L.gb_n), mmode == M_APPROX ? 2 : 1) * l * l * 8;
    sizes[O_G] = sizes[O_R] = sizes[O_RINV] = sizes[O_RACC] = sizes[O_R2] = sizes[O_QT] =
        (size_t)l * l * 8;
    sizes[O_TAU] = 2 * LMAX * 8;
    sizes[O_REP] = 128 * 8;
    sizes[O_FLAGS] = 64;
    sizes[O_PERM] = (size_t)l * 4;
    sizes[O_SCPART] = prec == P_FP8 ? (size_t)SCALE_CHUNKS * L.lp * 4 : 0;
    sizes[O_MX] = mmode != M_R2T ? (size_t)l * l * 8 : 0;
    sizes[O_R1] = mmode == M_APPROX ? (size_t)l * l * 8 : 0;
    sizes[O_XK] = mmode == M_APPROX ? (size_t)n * l * 8 : 0;
    sizes[O_AT] = ulv ? (size_t)m * at_ld(n, prec) * sz : 0;
    sizes[O_TT] = ulv ? (size_t)l * l * 8 : 0;
    size_t off = 0;
    for (int i = 0; i < O_COUNT; i++) {
        L.off[i] = off;
        off += (size_t)roundup((int64_t)sizes[i], 256);
    }
    L.total = off;
    return L;
}

static bool valid_prec(int p) { return p >= COR_F64 && p <= COR_FP8; }

static cor_status validate_opts(const cor_opts* o, const cor_problem& p) {
    if (!o) return COR_OK;
    if (o->compress < COR_M_R2T || o->compress > COR_M_APPROX)
        return fail(COR_E_INVAL, "unknown compression mode");
    if (o->orient != COR_URV && o->orient != COR_ULV) return fail(COR_E_INVAL, "unknown orientation");
    if (o->orient == COR_ULV && p.prec == COR_FP8)
        return fail(COR_E_INVAL, "ULV needs A^T in the storage format: not available for COR_FP8");
    return COR_OK;
}

// The fused power step (A^T (A X) in one read of A): FP32 or FP64 passes,
// l <= 64, and the n x lp partial sum plus a chunk of A X in one CU's LDS.
// n is the column count of the matrix the passes read (m for ULV).
cor_status fused_check(const cor_problem& p, int ulv) {
    const int64_t n = ulv ? p.m : p.n;
    const int lp = (int)roundup((int64_t)p.k + p.p, 16);
    if (p.prec != COR_F64 && p.prec != COR_F32)
        return fail(COR_E_INVAL, "the fused power step needs COR_F64 or COR_F32 passes");
    if (lp / 16 > ATA_NTMAX) return fail(COR_E_INVAL, "the fused power step needs l <= 64");
    const bool f64 = p.prec == COR_F64;
    if (n > (f64 ? ATA_NMAX64 : ATA_NMAX32) ||
        ata_tiles_per_wave(n, lp) > ata_max_tiles_per_wave(p.prec, lp) ||
        ata_lds_bytes(n, lp, p.prec) > ATA_LDS)
        return fail(COR_E_INVAL, "the fused power step needs n <= 2400 (FP32) or n <= 1024 "
                                 "(FP64) and ceil(n / 16) * roundup(l, 16) / 16 <= 8 T with "
                                 "T = 24 (FP32, l <= 32), 16 (FP32), 12 (FP64, l <= 32), 8 (FP64)");
    return COR_OK;
}

static cor_status validate(const cor_problem& p) {
    const int64_t l = (int64_t)p.k + p.p;
    if (!p.A || !p.U || !p.T || !p.V) return fail(COR_E_INVAL, "null A, U, T or V");
    if (!valid_prec(p.prec)) return fail(COR_E_INVAL, "unknown precision");
    if (p.m < 1 || p.n < 1) return fail(COR_E_INVAL, "m and n must be positive");
    if (p.k < 1) return fail(COR_E_INVAL, "k must be >= 1");
    if (p.p < 0) return fail(COR_E_INVAL, "p must be >= 0");
    if (p.q < 0 || p.q > 16) return fail(COR_E_INVAL, "q must be in [0, 16]");
    if (l < 2) return fail(COR_E_INVAL, "l = k + p must be >= 2");
    if (l >= std::min(p.m, p.n)) return fail(COR_E_INVAL, "l = k + p must be < min(m, n)");
    if (l > LMAX) return fail(COR_E_INVAL, "l = k + p must be <= 264");
    if (p.lda < p.n) return fail(COR_E_INVAL, "lda must be >= n");
    if (p.prec == COR_FP8 && !p.colscale) return fail(COR_E_INVAL, "FP8 needs colscale");
    return COR_OK;
}

struct Plan {
    int device = 0;
    int count = 0;
    int max_q = 0;
    int report = 0;
    int prec_mix = 0;  // bitmask of precisions present
    bool has_explicit = false, has_approx = false, has_ulv = false, has_fused = false;
    int nj = 1;        // ceil(max l / 64): column tiles of the row-block products
    int lmax = 0;      // largest l of the plan
    std::vector<cor_problem> reqs;
    std::vector<Layout> lay;
    std::vector<Prob> hp;     // host copies of the descriptors
    void* mem = nullptr;      // device: descriptors + tables + workspace
    size_t mem_bytes = 0;
    Prob* d_probs = nullptr;

    struct Grp {
        LaunchGroup g{};
        int nt = 0;
        int prec = 0;
        int aux = 0;      // fused step: tiles per wave
        size_t lds = 0;   // fused step: dynamic LDS bytes
        double bytes = 0, flops = 0;  // algorithmic cost of one launch
    };
    Grp omega, opM, opN, sumM, sumN, gramM, gramN, redM, redN, small, applyM, applyN, vg, r2, norm;
    Grp scM, scN;  // FP8 operand scales: row chunks of the column maxima
    Grp xgM, xgN, xred, keepx, tra, ulvt;  // compression modes and ULV
    std::vector<Grp> skAX, skATX;  // per (precision, column tiles)
    std::vector<Grp> ata;          // fused power step, per (precision, column tiles)
    std::vector<Grp> formU;        // per register-tile class of l (nt holds l)
    Grp applyU;                    // U = Q1 Qs for the problems with u_via_qs
    // per iteration of the power loop: whether any problem of the plan takes
    // the second CholeskyQR pass, and whether it is any problem's last one
    // (kernels return at once for the others; their launches are skipped)
    std::vector<char> second, last;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    struct HostStream* hs = nullptr;  // A in host memory, streamed in row panels
    bool async = false;
    bool owned = true;  // mem was allocated by the plan (else caller-provided)
    std::vector<int32_t> tab_host;
    // Passes of several column-tile classes: the classes' launches run side
    // by side on these streams (fork and join through events), so that one
    // class's last blocks overlap the others' instead of each launch ending
    // in its own tail.  ev[0] forks, ev[1 + i] joins aux[i].
    std::vector<hipStream_t> aux;
    std::vector<hipEvent_t> ev;
};

constexpr int PASS_AUX_STREAMS = 4;

// Build a launch table: per-problem block counts -> (pidx, toff) in device memory.
struct TableBuilder {
    std::vector<int32_t> host;  // concatenated [pidx..., toff...] of all tables
    struct Ref { size_t pidx_off, toff_off; int count, blocks; };
    Ref add(const std::vector<int>& probs, const std::vector<int64_t>& blocks) {
        Ref r;
        r.count = (int)probs.size();
        r.pidx_off = host.size();
        for (int p : probs) host.push_back(p);
        r.toff_off = host.size();
        int64_t acc = 0;
        for (size_t i = 0; i < probs.size(); i++) {
            host.push_back((int32_t)acc);
            acc += blocks[i];
        }
        host.push_back((int32_t)acc);
        r.blocks = (int)acc;
        return r;
    }
};

cor_status plan_create(const cor_problem* probs, int32_t count, const cor_opts* opts,
                       Plan** out, hipStream_t astream, bool async, void* ext_mem,
                       size_t ext_bytes) {
    if (!probs || count < 1 || !out) return fail(COR_E_INVAL, "no problems");
    for (int i = 0; i < count; i++) {
        cor_status st = validate(probs[i]);
        if (st == COR_OK) st = validate_opts(opts, probs[i]);
        if (st != COR_OK) return st;
    }
    const int mmode = opts ? opts->compress : M_R2T;
    const int ulv = (opts && opts->orient == COR_ULV) ? 1 : 0;
    const int fused = (opts && opts->fused_power) ? 1 : 0;
    if (fused)
        for (int i = 0; i < count; i++) {
            cor_status st = fused_check(probs[i], ulv);
            if (st != COR_OK) return st;
            if (probs[i].q != probs[0].q)
                return fail(COR_E_INVAL, "a plan with the fused power step needs one q for all "
                                         "its problems");
        }
    // A ULV request is run as the URV of A^T (an n x m matrix in the
    // workspace): the problem the stages see has m and n, U and V swapped.
    const cor_problem* const caller = probs;
    std::vector<cor_problem> iprobs(probs, probs + count);
    if (ulv)
        for (auto& q : iprobs) {
            std::swap(q.m, q.n);
            std::swap(q.U, q.V);
            q.lda = at_ld(q.n, q.prec);
        }
    probs = iprobs.data();
    Plan* P = new Plan();
    HIPCHK(hipGetDevice(&P->device));
    P->count = count;
    P->report = opts ? opts->report : 0;
    P->reqs.assign(caller, caller + count);  // the caller's requests (before the ULV swap)
    const int sk_target = sketch_block_target();
    const int gr_target = 1024;
    size_t ws = 0;
    std::vector<size_t> base(count);
    for (int i = 0; i < count; i++) {
        const cor_problem& q = probs[i];
        P->lay.push_back(
            make_layout(q.m, q.n, q.k + q.p, q.prec, sk_target, gr_target, mmode, ulv, fused));
        base[i] = ws;
        ws += P->lay.back().total;
        P->max_q = std::max(P->max_q, (int)q.q);
        P->prec_mix |= 1 << q.prec;
        P->nj = std::max(P->nj, (int)((q.k + q.p + 63) / 64));
        P->lmax = std::max(P->lmax, (int)(q.k + q.p));
    }
    P->has_fused = fused != 0;
    P->has_explicit = mmode == M_EXPLICIT;
    P->has_approx = mmode == M_APPROX;
    P->has_ulv = ulv != 0;
    P->second.assign(P->max_q + 1, 0);
    P->last.assign(P->max_q + 1, 0);
    for (int i = 0; i < count; i++)
        for (int it = 0; it <= probs[i].q; it++) {
            if (it == probs[i].q || (opts && opts->cholqr2_all)) P->second[it] = 1;
            if (it == probs[i].q) P->last[it] = 1;
        }

    // Launch tables.
    TableBuilder tb;
    std::vector<int> all(count);
    for (int i = 0; i < count; i++) all[i] = i;
    auto per = [&](auto fn) {
        std::vector<int64_t> b(count);
        for (int i = 0; i < count; i++) b[i] = fn(i);
        return tb.add(all, b);
    };
    auto R_omega = per([&](int i) { return cdiv(cdiv(probs[i].n * P->lay[i].l, 2), 256); });
    auto R_opM = per([&](int i) { return cdiv(P->lay[i].ldq, MO_ROWS) * (P->lay[i].lp / MO_COLS); });
    auto R_opN = per([&](int i) { return cdiv(P->lay[i].ldx, MO_ROWS) * (P->lay[i].lp / MO_COLS); });
    auto R_sumM = per([&](int i) { return cdiv(probs[i].m * P->lay[i].lp / 4, 256); });
    auto R_sumN = per([&](int i) { return cdiv(probs[i].n * P->lay[i].lp / 4, 256); });
    auto R_gramM = per([&](int i) { return (int64_t)P->lay[i].gb_m * gram_groups(P->lay[i].lp); });
    auto R_gramN = per([&](int i) { return (int64_t)P->lay[i].gb_n * gram_groups(P->lay[i].lp); });
    auto R_red = per([&](int i) { return cdiv((int64_t)P->lay[i].l * P->lay[i].l, 64); });
    auto R_small = per([&](int) { return (int64_t)1; });
    auto R_applyM = per([&](int i) { return cdiv(probs[i].m, APPLY_ROWS); });
    auto R_applyN = per([&](int i) { return cdiv(probs[i].n, APPLY_ROWS); });
    auto R_vg = per([&](int i) { return cdiv(probs[i].n * P->lay[i].l, 256); });
    auto R_r2 = per([&](int i) { return (int64_t)P->lay[i].nt * P->lay[i].nt; });
    auto R_norm = per([&](int) { return (int64_t)64; });
    auto R_xgM = per([&](int i) {
        return mmode == M_EXPLICIT ? (int64_t)P->lay[i].gb_m * gram_side(P->lay[i].lp) * gram_side(P->lay[i].lp) : 0; });
    auto R_xgN = per([&](int i) {
        return mmode == M_APPROX ? (int64_t)P->lay[i].gb_n * gram_side(P->lay[i].lp) * gram_side(P->lay[i].lp) : 0; });
    auto R_xred = per([&](int i) {
        return mmode != M_R2T ? cdiv((int64_t)P->lay[i].l * P->lay[i].l, 64) : 0; });
    auto R_keepx = per([&](int i) {
        return mmode == M_APPROX ? cdiv(probs[i].n * P->lay[i].l, 256) : 0; });
    auto R_tra = per([&](int i) { return ulv ? cdiv(probs[i].n, 32) * cdiv(probs[i].m, 32) : 0; });
    auto R_ulvt = per([&](int i) {
        return ulv ? cdiv((int64_t)P->lay[i].l * P->lay[i].l, 256) : 0; });
    auto R_scM = per([&](int i) { return probs[i].prec == COR_FP8 ? (int64_t)scale_chunks(probs[i].m) : 0; });
    auto R_scN = per([&](int i) { return probs[i].prec == COR_FP8 ? (int64_t)scale_chunks(probs[i].n) : 0; });
    // Sketch tables: one per (precision, column-tile count) class.
    std::map<std::pair<int, int>, std::vector<int>> classes;
    for (int i = 0; i < count; i++) classes[{probs[i].prec, P->lay[i].nt}].push_back(i);
    // U assembly tables: one per class of ceil(l/8).
    std::map<int, std::vector<int>> uclasses;
    for (int i = 0; i < count; i++) {
        const int tn = (P->lay[i].l + 7) / 8;
        uclasses[tn <= 4 ? 4 : tn <= 8 ? 8 : tn <= 16 ? 16 : tn <= 24 ? 24 : 33].push_back(i);
    }
    struct URef { int lmax; TableBuilder::Ref r; };
    std::vector<URef> urefs;
    for (auto& kv : uclasses) {
        std::vector<int64_t> b;
        int lmax = 0;
        for (int i : kv.second) {
            b.push_back(cdiv(u_via_qs(probs[i].m, P->lay[i].l) ? (int64_t)P->lay[i].l : probs[i].m,
                             formqs_rows(kv.first > 16 ? 129 : 128)));
            lmax = std::max(lmax, (int)P->lay[i].l);
        }
        urefs.push_back({lmax, tb.add(kv.second, b)});
    }
    std::vector<int> usub;
    std::vector<int64_t> ublk;
    for (int i = 0; i < count; i++)
        if (u_via_qs(probs[i].m, P->lay[i].l)) {
            usub.push_back(i);
            ublk.push_back(cdiv(probs[i].m, APPLY_ROWS));
        }
    const TableBuilder::Ref R_applyU = tb.add(usub, ublk);
    struct SkRef {
        int prec, nt;
        TableBuilder::Ref ax, atx, ata;
        double bax, fax, batx, fatx, bata, fata;
        int tpw;
        size_t lds;
    };
    std::vector<SkRef> skrefs;
    for (auto& kv : classes) {
        std::vector<int64_t> bax, batx, bata;
        double bytes_ax = 0, fl = 0, bytes_atx = 0, bytes_ata = 0;
        int tpw = 0;
        size_t lds = 0;
        for (int i : kv.second) {
            const cor_problem& q = probs[i];
            const Layout& L = P->lay[i];
            bax.push_back(cdiv(q.m, sketch_rows_per_block(q.prec, L.nt, false)) * L.s_ax);
            batx.push_back(cdiv(q.n, sketch_rows_per_block(q.prec, L.nt, true)) * L.s_atx);
            const double sz = prec_size(q.prec);
            const double abytes = (double)q.m * q.n * sz;
            bytes_ax += abytes + (double)q.n * L.l * sz + (double)q.m * L.l * 4.0;
            bytes_atx += abytes + (double)q.m * L.l * sz + (double)q.n * L.l * 4.0;
            fl += 2.0 * q.m * q.n * L.l;
            // fused step: A once, X, and the n x l result
            bata.push_back(L.s_f);
            bytes_ata += abytes + (double)q.n * L.l * sz + (double)q.n * L.l * 8.0;
            if (fused) {
                tpw = std::max(tpw, ata_tiles_per_wave(q.n, L.lp));
                lds = std::max(lds, ata_lds_bytes(q.n, L.lp, q.prec));
            }
        }
        SkRef r{kv.first.first, kv.first.second, tb.add(kv.second, bax), tb.add(kv.second, batx),
                tb.add(kv.second, bata), bytes_ax, fl, bytes_atx, fl, bytes_ata, 2.0 * fl,
                tpw, lds};
        skrefs.push_back(r);
    }

    // One device allocation: descriptors | tables | workspaces.
    const size_t desc_bytes = roundup(sizeof(Prob) * count, 256);
    const size_t tab_bytes = roundup(tb.host.size() * sizeof(int32_t), 256);
    P->mem_bytes = desc_bytes + tab_bytes + ws;
    P->async = async;
    hipError_t e = hipSuccess;
    if (ext_mem) {
        // Caller-provided device memory: nothing is allocated or freed.
        if (P->mem_bytes > ext_bytes) {
            const size_t need = P->mem_bytes;
            delete P;
            return fail(COR_E_INVAL, "problem needs " + std::to_string(need) +
                                         " bytes of workspace, more than the " +
                                         std::to_string(ext_bytes) + " available");
        }
        P->mem = ext_mem;
        P->owned = false;
    } else {
        e = async ? hipMallocAsync(&P->mem, P->mem_bytes, astream)
                  : hipMalloc(&P->mem, P->mem_bytes);
        if (e != hipSuccess) {
            delete P;
            return fail(COR_E_NOMEM, "workspace allocation failed");
        }
    }
    char* mem = (char*)P->mem;
    P->d_probs = (Prob*)mem;
    int32_t* d_tab = (int32_t*)(mem + desc_bytes);
    char* d_ws = mem + desc_bytes + tab_bytes;

    // Descriptors.
    P->hp.resize(count);
    for (int i = 0; i < count; i++) {
        const cor_problem& q = probs[i];
        const Layout& L = P->lay[i];
        char* w = d_ws + base[i];
        Prob& d = P->hp[i];
        memset(&d, 0, sizeof(Prob));
        d.A = ulv ? (const void*)(w + L.off[O_AT]) : q.A;
        d.colscale = q.colscale;
        d.m = q.m; d.n = q.n; d.lda = q.lda;
        d.k = q.k; d.l = L.l; d.lp = L.lp; d.q = q.q;
        d.prec = q.prec;
        d.report = P->report;
        d.cholqr2_all = (opts && opts->cholqr2_all) ? 1 : 0;
        const int sz = prec_size(q.prec);
        d.avec = (((uintptr_t)q.A % 16) == 0 && (q.lda * sz) % 16 == 0) ? 1 : 0;
        d.xop = w + L.off[O_XOP];
        d.qop = w + L.off[O_QOP];
        d.ldx = L.ldx; d.ldq = L.ldq;
        d.xscale = (float*)(w + L.off[O_XSC]);
        d.qscale = (float*)(w + L.off[O_QSC]);
        d.ypart = w + L.off[O_YPART];
        d.s_ax = L.s_ax; d.s_atx = L.s_atx; d.kc_ax = L.kc_ax; d.kc_atx = L.kc_atx;
        d.Y = (double*)(w + L.off[O_Y]);
        d.Qa = (double*)(w + L.off[O_QA]);
        d.Q1 = (double*)(w + L.off[O_Q1]);
        d.Q2 = (double*)(w + L.off[O_Q2]);
        d.gpart = (double*)(w + L.off[O_GPART]);
        d.rb_m = L.rb_m; d.rb_n = L.rb_n; d.gb_m = L.gb_m; d.gb_n = L.gb_n;
        d.G = (double*)(w + L.off[O_G]);
        d.R = (double*)(w + L.off[O_R]);
        d.Rinv = (double*)(w + L.off[O_RINV]);
        d.Racc = (double*)(w + L.off[O_RACC]);
        d.R2 = (double*)(w + L.off[O_R2]);
        d.Qt = (double*)(w + L.off[O_QT]);
        d.tau = (double*)(w + L.off[O_TAU]);
        d.rep = (double*)(w + L.off[O_REP]);
        d.flags = (int32_t*)(w + L.off[O_FLAGS]);
        d.scpart = (float*)(w + L.off[O_SCPART]);
        d.sch_m = scale_chunks(q.m);
        d.sch_n = scale_chunks(q.n);
        d.U = q.U; d.T = ulv ? (double*)(w + L.off[O_TT]) : q.T; d.V = q.V;
        d.mmode = mmode;
        d.ulv = ulv;
        d.Mx = (double*)(w + L.off[O_MX]);
        d.R1 = (double*)(w + L.off[O_R1]);
        d.Xk = (double*)(w + L.off[O_XK]);
        d.msrc = mmode == M_R2T ? d.R2 : d.Mx;
        d.Tout = caller[i].T;
        d.ulv_src = caller[i].A;
        d.ulv_lda = caller[i].lda;
        d.perm = q.perm ? q.perm : (int32_t*)(w + L.off[O_PERM]);
        d.omega = q.omega;
        d.seed = q.seed;
        d.fused = fused;
        d.s_f = L.s_f;
        d.kc_f = L.kc_f;
    }
    P->tab_host.swap(tb.host);
    if (ext_mem) {
        // Stream-ordered uploads (the host copies live in the plan) and a
        // fill kernel for the workspace clear.
        e = hipMemcpyAsync(P->d_probs, P->hp.data(), sizeof(Prob) * count, hipMemcpyHostToDevice,
                           astream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_tab, P->tab_host.data(), P->tab_host.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, astream);
        if (e == hipSuccess) e = launch_zero(d_ws, ws, astream);
    } else if (async) {
        e = hipMemcpyAsync(P->d_probs, P->hp.data(), sizeof(Prob) * count, hipMemcpyHostToDevice,
                           astream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_tab, P->tab_host.data(), P->tab_host.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, astream);
        // Operand buffers are zero outside the written rows x l block.
        if (e == hipSuccess) e = hipMemsetAsync(d_ws, 0, ws, astream);
    } else {
        e = hipMemcpy(P->d_probs, P->hp.data(), sizeof(Prob) * count, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(d_tab, P->tab_host.data(), P->tab_host.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(d_ws, 0, ws);
    }
    if (e != hipSuccess) {
        if (P->owned) {
            if (async) (void)hipFreeAsync(P->mem, astream);
            else (void)hipFree(P->mem);
        }
        delete P;
        return hip_fail(e, "plan upload");
    }
    auto mk = [&](const TableBuilder::Ref& r) {
        Plan::Grp g;
        g.g.probs = P->d_probs;
        g.g.pidx = d_tab + r.pidx_off;
        g.g.toff = d_tab + r.toff_off;
        g.g.count = r.count;
        g.g.blocks = r.blocks;
        return g;
    };
    P->omega = mk(R_omega); P->opM = mk(R_opM); P->opN = mk(R_opN);
    P->sumM = mk(R_sumM); P->sumN = mk(R_sumN);
    P->gramM = mk(R_gramM); P->gramN = mk(R_gramN);
    P->redM = mk(R_red); P->redN = P->redM;
    P->small = mk(R_small);
    P->applyM = mk(R_applyM); P->applyN = mk(R_applyN); P->applyU = mk(R_applyU);
    P->vg = mk(R_vg); P->r2 = mk(R_r2); P->norm = mk(R_norm);
    P->scM = mk(R_scM); P->scN = mk(R_scN);
    P->xgM = mk(R_xgM); P->xgN = mk(R_xgN); P->xred = mk(R_xred); P->keepx = mk(R_keepx);
    P->tra = mk(R_tra); P->ulvt = mk(R_ulvt);
    for (auto& u : urefs) {
        Plan::Grp g = mk(u.r);
        g.nt = u.lmax;
        P->formU.push_back(g);
    }
    for (auto& r : skrefs) {
        Plan::Grp a = mk(r.ax), b = mk(r.atx);
        a.nt = b.nt = r.nt;
        a.prec = b.prec = r.prec;
        a.bytes = r.bax; a.flops = r.fax;
        b.bytes = r.batx; b.flops = r.fatx;
        P->skAX.push_back(a);
        P->skATX.push_back(b);
        if (P->has_fused) {
            Plan::Grp f = mk(r.ata);
            f.nt = r.nt;
            f.prec = r.prec;
            f.bytes = r.bata;
            f.flops = r.fata;
            f.aux = r.tpw;
            f.lds = r.lds;
            P->ata.push_back(f);
        }
    }
    // streams for the classes of a pass (not for caller-provided memory: that
    // entry point creates nothing)
    if (P->owned && P->skAX.size() > 1) {
        const int na = std::min<int>(PASS_AUX_STREAMS, (int)P->skAX.size() - 1);
        hipError_t se = hipSuccess;
        for (int i = 0; i < na && se == hipSuccess; i++) {
            hipStream_t st = nullptr;
            se = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
            if (se == hipSuccess) P->aux.push_back(st);
        }
        for (int i = 0; i <= na && se == hipSuccess; i++) {
            hipEvent_t ev = nullptr;
            se = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (se == hipSuccess) P->ev.push_back(ev);
        }
        if (se != hipSuccess) {
            plan_destroy(P, nullptr);
            return hip_fail(se, "pass streams");
        }
    }
    *out = P;
    return COR_OK;
}

// ---------------------------------------------------------------------------
// A in host memory (the paper's pass model with A stored externally): every
// pass streams A in row panels through NB device staging buffers, the copy
// of panel p + 1 (on a copy stream) overlapping the kernels of panel p.  Each
// panel has descriptors of its own: for A X, rows r0 .. r0 + mp of the
// problem (A = the staging buffer, Y = the panel's rows of Y); for A^T Q1
// and the fused step, a K range of the problem whose split-K partial sums go
// to the panel's own split slots, which the problem's k_sum then adds.
// ---------------------------------------------------------------------------
enum HostPass { HP_AX = 0, HP_ATX = 1, HP_ATA = 2 };
constexpr int HS_NB = 2;  // staging buffers

struct HostStream {
    const char* A = nullptr;  // host, m x n, leading dimension lda (elements)
    int64_t m = 0, n = 0, lda = 0, rows = 0;  // rows per panel
    int npanel = 0, sz = 0, nt = 0, prec = 0;
    void* mem = nullptr;  // device: staging | partial scratch | descriptors | tables
    char* stage[HS_NB] = {nullptr, nullptr};
    hipStream_t cs = nullptr;
    hipEvent_t copied[HS_NB] = {nullptr, nullptr}, freed[HS_NB] = {nullptr, nullptr};
    hipEvent_t start = nullptr;
    bool used[HS_NB] = {false, false};
    // per panel and pass kind: its launch groups
    std::vector<LaunchGroup> sk[3], sum;  // sketch / fused kernel; M-side sum of A X
};

static hipError_t host_pass(Plan* P, int kind, int it, hipStream_t s) {
    HostStream* H = P->hs;
    hipError_t e = hipEventRecord(H->start, s);
    if (e != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(H->cs, H->start, 0)) != hipSuccess) return e;
    for (int p = 0; p < H->npanel; p++) {
        const int slot = p % HS_NB;
        const int64_t r0 = (int64_t)p * H->rows;
        const int64_t mp = std::min(H->rows, H->m - r0);
        if (H->used[slot] && (e = hipStreamWaitEvent(H->cs, H->freed[slot], 0)) != hipSuccess)
            return e;
        const size_t w = (size_t)H->n * H->sz;
        e = H->lda == H->n
                ? hipMemcpyAsync(H->stage[slot], H->A + r0 * w, mp * w, hipMemcpyHostToDevice, H->cs)
                : hipMemcpy2DAsync(H->stage[slot], w, H->A + r0 * H->lda * H->sz,
                                   (size_t)H->lda * H->sz, w, mp, hipMemcpyHostToDevice, H->cs);
        if (e != hipSuccess) return e;
        if ((e = hipEventRecord(H->copied[slot], H->cs)) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(s, H->copied[slot], 0)) != hipSuccess) return e;
        const LaunchGroup& g = H->sk[kind][p];
        hipEvent_t a, b;
        prof_begin(s, &a, &b, kind == HP_ATA ? 2 : 1);
        if (kind == HP_ATA) {
            const Prob& d = P->hp[0];
            e = launch_ata(H->prec, H->nt, ata_tiles_per_wave(H->n, d.lp),
                           ata_lds_bytes(H->n, d.lp, H->prec), g, it, s);
        } else {
            e = launch_sketch(H->prec, kind == HP_ATX, H->nt, g, it, s);
        }
        if (e != hipSuccess) return e;
        const double abytes = (double)mp * H->n * H->sz;
        prof_end(s, a, b, abytes, (kind == HP_ATA ? 4.0 : 2.0) * mp * H->n * P->hp[0].l);
        if (kind == HP_AX && (e = launch_sum(H->sum[p], SIDE_M, it, s)) != hipSuccess) return e;
        if ((e = hipEventRecord(H->freed[slot], s)) != hipSuccess) return e;
        H->used[slot] = true;
    }
    return hipSuccess;
}

static hipError_t run_sketch(const Plan* P, const std::vector<Plan::Grp>& gs, bool trans,
                             int iter, hipStream_t s) {
    const int na = std::min<int>((int)gs.size() - 1, (int)P->aux.size());
    if (na <= 0) {
        for (const auto& g : gs) {
            hipEvent_t a, b;
            prof_begin(s, &a, &b, 1);
            hipError_t e = launch_sketch(g.prec, trans, g.nt, g.g, iter, s);
            if (e != hipSuccess) return e;
            prof_end(s, a, b, g.bytes, g.flops);
        }
        return hipSuccess;
    }
    // classes side by side: class 0 on s, class k on aux[(k - 1) mod na];
    // profiled as one launch from the fork to the join
    double bytes = 0, flops = 0;
    for (const auto& g : gs) {
        bytes += g.bytes;
        flops += g.flops;
    }
    hipEvent_t a, b;
    prof_begin(s, &a, &b, 1);
    hipError_t e = hipEventRecord(P->ev[0], s);
    for (int i = 0; i < na && e == hipSuccess; i++) e = hipStreamWaitEvent(P->aux[i], P->ev[0], 0);
    for (size_t k = 0; k < gs.size() && e == hipSuccess; k++) {
        hipStream_t st = k == 0 ? s : P->aux[(k - 1) % na];
        e = launch_sketch(gs[k].prec, trans, gs[k].nt, gs[k].g, iter, st);
    }
    for (int i = 0; i < na && e == hipSuccess; i++) {
        e = hipEventRecord(P->ev[1 + i], P->aux[i]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, P->ev[1 + i], 0);
    }
    if (e != hipSuccess) return e;
    prof_end(s, a, b, bytes, flops);
    return hipSuccess;
}

// The stage sequence of Alg. 3 for every problem of the plan.
static hipError_t plan_enqueue(Plan* P, hipStream_t s) {
#define E(x)                                   \
    do {                                       \
        hipError_t e_ = (x);                   \
        if (e_ != hipSuccess) return e_;       \
    } while (0)
    const bool fp8 = (P->prec_mix >> P_FP8) & 1;
    if (P->has_ulv) E(launch_transpose_a(P->tra.g, s));  // A^T for the ULV requests
    if (P->report) E(launch_normA(P->norm.g, s));
    E(launch_omega(P->omega.g, s));  // Q2 <- Omega (FP64)
    if (fp8) E(launch_op_scales(P->scN.g, P->small.g, SIDE_N, 0, s));
    E(launch_make_op(P->opN.g, SIDE_N, s));  // X <- Omega in the pass format
    // Q2 R2 = Y (CholeskyQR, two passes for the final pair); X <- Q2
    auto nside = [&](int it) -> hipError_t {
        E(launch_gram(P->gramN.g, SIDE_N, GSRC_Y, it, s));
        E(launch_gram_reduce(P->redN.g, SIDE_N, 0, it, s));
        E(launch_chol(P->small.g, CHOL_FIRST, P->lmax, it, s));
        E(launch_apply(P->applyN.g, SIDE_N, AP_Y_RINV_QA, P->lmax, it, s));
        if (P->second[it]) {
            E(launch_gram(P->gramN.g, SIDE_N, GSRC_QA, it, s));
            E(launch_gram_reduce(P->redN.g, SIDE_N, 1, it, s));
            E(launch_chol(P->small.g, CHOL_SECOND, P->lmax, it, s));
        }
        if (P->last[it]) E(launch_r2(P->r2.g, it, 0, s));
        if (P->second[it]) E(launch_apply(P->applyN.g, SIDE_N, AP_QA_RINV_Q, P->lmax, it, s));
        return hipSuccess;
    };
    for (int it = 0; it <= P->max_q; it++) {
        if (P->has_fused && it < P->max_q) {
            // The loop of Alg. 3 as printed, C2 = A^T (A C2), in one read of
            // A: Y = A^T A X; R1 from X^T Y = (A X)^T (A X) (the Gram of the
            // first sketch); Y <- Y R1^{-1} = A^T Q1; then the n-side
            // orthonormalisation as after the A^T Q1 pass.  (Every problem of
            // a fused plan has the same q.)
            if (P->hs) {
                E(host_pass(P, HP_ATA, it, s));
            } else {
                for (const auto& g : P->ata) {
                    hipEvent_t a, b;
                    prof_begin(s, &a, &b, 2);
                    E(launch_ata(g.prec, g.nt, g.aux, g.lds, g.g, it, s));
                    prof_end(s, a, b, g.bytes, g.flops);
                }
            }
            E(launch_sum(P->sumN.g, SIDE_F, it, s));
            E(launch_gram(P->gramN.g, SIDE_N, GSRC_XY, it, s));
            E(launch_gram_reduce(P->redN.g, SIDE_N, 0, it, s));
            E(launch_chol(P->small.g, CHOL_FIRST, P->lmax, it, s));
            E(launch_apply(P->applyN.g, SIDE_N, AP_Y_RINV_Y, P->lmax, it, s));
            E(nside(it));
            continue;
        }
        // Y1 = A X, Q1 R1 = Y1 (CholeskyQR2)
        if (P->hs) {
            E(host_pass(P, HP_AX, it, s));
        } else {
            E(run_sketch(P, P->skAX, false, it, s));
            E(launch_sum(P->sumM.g, SIDE_M, it, s));
        }
        E(launch_gram(P->gramM.g, SIDE_M, GSRC_Y, it, s));
        E(launch_gram_reduce(P->redM.g, SIDE_M, 0, it, s));
        E(launch_chol(P->small.g, CHOL_FIRST, P->lmax, it, s));
        E(launch_apply(P->applyM.g, SIDE_M, AP_Y_RINV_QA, P->lmax, it, s));
        if (P->second[it]) {
            E(launch_gram(P->gramM.g, SIDE_M, GSRC_QA, it, s));
            E(launch_gram_reduce(P->redM.g, SIDE_M, 1, it, s));
            E(launch_chol(P->small.g, CHOL_SECOND, P->lmax, it, s));
            // eq. (18): R1 = R' R of the last Y1
            if (P->has_approx && P->last[it]) E(launch_r2(P->r2.g, it, 1, s));
            E(launch_apply(P->applyM.g, SIDE_M, AP_QA_RINV_Q, P->lmax, it, s));
        }
        if (fp8) {
            E(launch_op_scales(P->scM.g, P->small.g, SIDE_M, it, s));
            E(launch_make_op(P->opM.g, SIDE_M, s));
        }
        // eq. (18) keeps the last step's input X before Q2 is overwritten
        if (P->has_approx && P->last[it]) E(launch_keep_x(P->keepx.g, it, s));
        // Y2 = A^T Q1, Q2 R2 = Y2 (CholeskyQR2); X <- Q2
        if (P->hs) E(host_pass(P, HP_ATX, it, s));
        else E(run_sketch(P, P->skATX, true, it, s));
        E(launch_sum(P->sumN.g, SIDE_N, it, s));
        E(nside(it));
        if (fp8 && it < P->max_q) {
            E(launch_op_scales(P->scN.g, P->small.g, SIDE_N, it, s));
            E(launch_make_op(P->opN.g, SIDE_N, s));
        }
    }
    // M = Q1^T A Q2 = R2^T (default); or explicitly, one more pass over A
    // (eq. (14) as printed); or eq. (18) from R1 and Q2^T X.
    if (P->has_explicit) {
        if (fp8) {  // the FP8 operand copy of the final Q2
            E(launch_op_scales(P->scN.g, P->small.g, SIDE_N, P->max_q, s));
            E(launch_make_op(P->opN.g, SIDE_N, s));
        }
        E(run_sketch(P, P->skAX, false, -1, s));  // Y = A Q2
        E(launch_sum(P->sumM.g, SIDE_M, -1, s));
        E(launch_gram(P->xgM.g, SIDE_M, GSRC_XM, -1, s));  // Q1^T Y
        E(launch_xreduce(P->xred.g, GSRC_XM, s));
    }
    if (P->has_approx) {
        E(launch_gram(P->xgN.g, SIDE_N, GSRC_XA, -1, s));  // G = Q2^T X
        E(launch_xreduce(P->xred.g, GSRC_XA, s));
        E(launch_dapprox(P->small.g, s));  // M = R1 G^-1
    }
    // M P = Qt T; U = Q1 Qs (Qs = Qt diag(sign)), V = Q2 P.
    E(launch_qrcp(P->small.g, P->lmax, s));
    for (const auto& ug : P->formU) E(launch_form_qs(ug.g, ug.nt, s));
    E(launch_apply(P->applyU.g, SIDE_M, AP_Q1_QS_U, P->lmax, -1, s));
    E(launch_gather_v(P->vg.g, s));
    if (P->report) {
        E(launch_gram(P->gramM.g, SIDE_M, GSRC_U, -1, s));
        E(launch_gram_reduce(P->redM.g, SIDE_M, 0, -1, s));
        E(launch_report(P->small.g, 1, s));
        E(launch_gram(P->gramN.g, SIDE_N, GSRC_V, -1, s));
        E(launch_gram_reduce(P->redN.g, SIDE_N, 0, -1, s));
        E(launch_report(P->small.g, 2, s));
        E(launch_report(P->small.g, 3, s));
    }
    if (P->has_ulv) E(launch_ulv_t(P->ulvt.g, s));  // T = T'^T (lower triangular)
    return hipSuccess;
#undef E
}

cor_status plan_run(Plan* P, hipStream_t s) {
    if (P->gexec) {
        HIPCHK(hipGraphLaunch(P->gexec, s));
        return COR_OK;
    }
    hipError_t e = plan_enqueue(P, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return COR_OK;
}

cor_status plan_capture(Plan* P, hipStream_t s) {
    if (!s) return fail(COR_E_INVAL, "graph capture needs a non-null stream");
    if (P->hs) return fail(COR_E_INVAL, "a plan that streams A from host memory is not captured");
    if (P->gexec) {
        (void)hipGraphExecDestroy(P->gexec);
        (void)hipGraphDestroy(P->graph);
        P->gexec = nullptr;
        P->graph = nullptr;
    }
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    const int prof = g_prof.on;
    g_prof.on = 0;  // no event records inside the graph
    hipError_t e = plan_enqueue(P, s);
    g_prof.on = prof;
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess) return hip_fail(e, "capture enqueue");
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    P->graph = g;
    HIPCHK(hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0));
    return COR_OK;
}

cor_status plan_info(Plan* P, cor_info* infos, hipStream_t s) {
    HIPCHK(hipStreamSynchronize(s));
    for (int i = 0; i < P->count; i++) {
        const Prob& d = P->hp[i];
        int32_t flags = 0;
        double rep[6] = {0, 0, 0, 0, 0, 0};
        HIPCHK(hipMemcpy(&flags, d.flags, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (P->report) HIPCHK(hipMemcpy(rep, d.rep, sizeof(rep), hipMemcpyDeviceToHost));
        if (infos) {
            cor_info& f = infos[i];
            f.err_l = rep[0];
            f.err_k = rep[1];
            f.orth_u = d.ulv ? rep[3] : rep[2];  // a ULV request's U is the V of A^T
            f.orth_v = d.ulv ? rep[2] : rep[3];
            f.m_check = rep[5];
            f.flags = flags;
            f.l = d.l;
        }
        if (flags & FLAG_NONFINITE) return fail(COR_E_NUMERIC, "non-finite value in a Gram matrix");
        if (flags & FLAG_SYNC_TIMEOUT)
            return fail(COR_E_DEVICE, "the QRCP's work-groups timed out waiting for each other");
    }
    return COR_OK;
}

static void host_stream_free(HostStream* H) {
    if (!H) return;
    if (H->cs) (void)hipStreamSynchronize(H->cs);
    for (int i = 0; i < HS_NB; i++) {
        if (H->copied[i]) (void)hipEventDestroy(H->copied[i]);
        if (H->freed[i]) (void)hipEventDestroy(H->freed[i]);
    }
    if (H->start) (void)hipEventDestroy(H->start);
    if (H->cs) (void)hipStreamDestroy(H->cs);
    if (H->mem) (void)hipFree(H->mem);
    delete H;
}

void plan_destroy(Plan* P, hipStream_t s) {
    if (!P) return;
    host_stream_free(P->hs);
    for (hipStream_t st : P->aux) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : P->ev) (void)hipEventDestroy(ev);
    if (P->gexec) (void)hipGraphExecDestroy(P->gexec);
    if (P->graph) (void)hipGraphDestroy(P->graph);
    if (P->mem && P->owned) {
        if (P->async) (void)hipFreeAsync(P->mem, s);
        else (void)hipFree(P->mem);
    }
    delete P;
}

// Flags and report of every problem from a host copy of their device words
// (used by the server, which reads them back asynchronously).
const Prob& plan_desc(const Plan* P, int i) { return P->hp[i]; }
int plan_count(const Plan* P) { return P->count; }
int plan_report(const Plan* P) { return P->report; }

size_t plan_bytes(const Plan* P) { return P->mem_bytes; }

size_t workspace_bytes(int64_t m, int64_t n, int32_t l, int prec, const cor_opts* opts) {
    const int mmode = opts ? opts->compress : M_R2T;
    const int ulv = (opts && opts->orient == COR_ULV) ? 1 : 0;
    const int fused = (opts && opts->fused_power) ? 1 : 0;
    Layout L = ulv ? make_layout(n, m, l, prec, sketch_block_target(), 1024, mmode, 1, fused)
                   : make_layout(m, n, l, prec, sketch_block_target(), 1024, mmode, 0, fused);
    return L.total + 256 + 1024;
}

// Cache of recent single-problem plans (reused when the same call repeats).
// A plan taken from the cache is marked busy until its call returns, so no
// other thread runs or evicts it meanwhile; a thread that finds its plan busy
// builds one of its own.  Eviction drops the oldest idle entry.
struct Cache {
    std::mutex mu;
    struct Item {
        std::vector<char> key;
        Plan* plan;
        bool busy;
    };
    std::vector<Item> items;
};
static Cache g_cache;
constexpr size_t CACHE_PLANS = 4;

static std::vector<char> key_of(const cor_problem& p, const cor_opts* o, int dev) {
    std::vector<char> k(sizeof(cor_problem) + sizeof(cor_opts) + sizeof(int), 0);
    memcpy(k.data(), &p, sizeof(p));
    cor_opts oo{};
    if (o) oo = *o;
    memcpy(k.data() + sizeof(p), &oo, sizeof(oo));
    memcpy(k.data() + sizeof(p) + sizeof(oo), &dev, sizeof(int));
    return k;
}

// Return a plan to the cache after its call (idle again), or destroy it when
// the cache is full of other plans.
static void cache_return(const std::vector<char>& key, Plan* P, bool from_cache) {
    Plan* drop = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache.mu);
        if (from_cache) {
            for (auto& it : g_cache.items)
                if (it.plan == P) it.busy = false;
            return;
        }
        if (g_cache.items.size() >= CACHE_PLANS) {
            auto old = std::find_if(g_cache.items.begin(), g_cache.items.end(),
                                    [](const Cache::Item& it) { return !it.busy; });
            if (old == g_cache.items.end()) {
                drop = P;  // every cached plan is running: do not cache this one
            } else {
                drop = old->plan;
                g_cache.items.erase(old);
            }
        }
        if (drop != P) g_cache.items.push_back({key, P, false});
    }
    if (drop) plan_destroy(drop, nullptr);
}

cor_status run_single(const cor_problem& p, const cor_opts* opts, cor_info* info,
                      hipStream_t s) {
    cor_status st = validate(p);
    if (st != COR_OK) return st;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::vector<char> key = key_of(p, opts, dev);
    Plan* P = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_cache.mu);
        for (auto& it : g_cache.items)
            if (!it.busy && it.key == key) {
                it.busy = true;
                P = it.plan;
                break;
            }
    }
    const bool from_cache = P != nullptr;
    if (!P) {
        st = plan_create(&p, 1, opts, &P, nullptr, false);
        if (st != COR_OK) return st;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e != hipSuccess) st = hip_fail(e, "timing events");
    if (st == COR_OK) st = plan_run(P, s);
    if (st == COR_OK) {
        e = hipEventRecord(e1, s);
        if (e != hipSuccess) st = hip_fail(e, "timing events");
    }
    // plan_info waits for the stream even after a failed launch, so the plan
    // is idle when it goes back to the cache.
    const cor_status st_info = plan_info(P, info, s);
    if (st == COR_OK) st = st_info;
    if (st == COR_OK && info) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        info->device_ms = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    cache_return(key, P, from_cache);
    return st;
}

// A host-streamed plan: panel descriptors and launch tables for a one-problem
// plan whose A (q.A) is in host memory.  panel_rows <= 0: panels of about
// 256 MiB.  The problem descriptor's n-side partial sums are redirected to
// the panels' split slots.
static cor_status host_setup(Plan* P, const cor_problem& q, int64_t panel_rows, int fused) {
    HostStream* H = new HostStream();
    P->hs = H;
    Prob& W = P->hp[0];
    const Layout& L = P->lay[0];
    H->A = (const char*)q.A;
    H->m = q.m;
    H->n = q.n;
    H->lda = q.lda;
    H->sz = prec_size(q.prec);
    H->nt = L.nt;
    H->prec = q.prec;
    const int64_t row_bytes = q.n * H->sz;
    int64_t rows = panel_rows > 0 ? panel_rows : std::max<int64_t>(1, (256ll << 20) / row_bytes);
    rows = roundup(std::max<int64_t>(rows, ATA_ROWS), ATA_ROWS);  // 16-byte aligned operand offsets
    if (rows >= q.m) rows = q.m;
    H->rows = rows;
    H->npanel = (int)cdiv(q.m, rows);
    const int np = H->npanel;
    const int acc = q.prec == P_F64 ? 8 : 4;
    const int bk = sketch_k_tile(q.prec);
    const int tgt = sketch_block_target();
    std::vector<int32_t> sax(np), satx(np), sf(np, 0);
    std::vector<int64_t> kcax(np), kcatx(np), kcf(np, 0), off(np + 1, 0), offf(np + 1, 0);
    int32_t sax_max = 0;
    for (int p = 0; p < np; p++) {
        const int64_t mp = std::min(rows, q.m - (int64_t)p * rows);
        split_k(mp, q.n, bk,
                sketch_rows_per_block(q.prec, L.nt, false) > 128 ? tgt / 2 : tgt, q.prec, L.nt,
                false, &sax[p], &kcax[p]);
        split_k(q.n, mp, bk,
                sketch_rows_per_block(q.prec, L.nt, true) > 128 ? tgt / 2 : tgt, q.prec, L.nt,
                true, &satx[p], &kcatx[p]);
        if (fused) fused_splits(mp, &sf[p], &kcf[p]);
        sax_max = std::max(sax_max, sax[p]);
        off[p + 1] = off[p] + satx[p];
        offf[p + 1] = offf[p] + sf[p];
    }
    // device memory: staging | M-side partials per slot | n-side partials |
    // panel descriptors | launch tables
    const size_t b_stage = roundup(rows * row_bytes, 256);
    const size_t b_scm = roundup((int64_t)sax_max * rows * L.lp * acc, 256);
    const size_t b_scn = roundup(std::max(off[np], offf[np]) * q.n * L.lp * acc, 256);
    const size_t b_desc = roundup(sizeof(Prob) * 3 * np, 256);
    const size_t b_tab = roundup(sizeof(int32_t) * 3 * 4 * np, 256);
    const size_t total = HS_NB * (b_stage + b_scm) + b_scn + b_desc + b_tab;
    if (hipMalloc(&H->mem, total) != hipSuccess) return fail(COR_E_NOMEM, "panel buffers");
    char* base = (char*)H->mem;
    for (int i = 0; i < HS_NB; i++) H->stage[i] = base + i * b_stage;
    char* scm = base + HS_NB * b_stage;
    char* scn = scm + HS_NB * b_scm;
    Prob* d_desc = (Prob*)(scn + b_scn);
    int32_t* d_tab = (int32_t*)((char*)d_desc + b_desc);
    std::vector<Prob> hd(3 * np);
    std::vector<int32_t> tab(3 * 4 * np);
    for (int k = 0; k < 3; k++) H->sk[k].resize(np);
    H->sum.resize(np);
    const int avec = (row_bytes % 16) == 0 ? 1 : 0;  // staging rows start 16-byte aligned
    for (int p = 0; p < np; p++) {
        const int slot = p % HS_NB;
        const int64_t r0 = (int64_t)p * rows, mp = std::min(rows, q.m - r0);
        Prob& ax = hd[3 * p + HP_AX];
        ax = W;
        ax.A = H->stage[slot];
        ax.m = mp;
        ax.lda = q.n;
        ax.avec = avec;
        ax.ypart = scm + slot * b_scm;
        ax.s_ax = sax[p];
        ax.kc_ax = kcax[p];
        ax.Y = W.Y + r0 * L.l;
        Prob& at = hd[3 * p + HP_ATX];
        at = W;
        at.A = H->stage[slot];
        at.m = mp;
        at.lda = q.n;
        at.avec = avec;
        at.qop = (char*)W.qop + r0 * H->sz;
        at.ypart = scn + off[p] * q.n * L.lp * acc;
        at.s_atx = satx[p];
        at.kc_atx = kcatx[p];
        Prob& af = hd[3 * p + HP_ATA];
        af = at;
        af.ypart = scn + offf[p] * q.n * L.lp * acc;
        af.s_f = sf[p];
        af.kc_f = kcf[p];
        // tables: [pidx, toff0, toff1] per (panel, kind) and for the panel's A X sum
        const int64_t blocks[4] = {
            cdiv(mp, sketch_rows_per_block(q.prec, L.nt, false)) * sax[p],
            cdiv(q.n, sketch_rows_per_block(q.prec, L.nt, true)) * satx[p], (int64_t)sf[p],
            cdiv(mp * L.lp / 4, 256)};
        for (int k = 0; k < 4; k++) {
            int32_t* t = tab.data() + 3 * (4 * p + k);
            t[0] = 3 * p + (k == 3 ? HP_AX : k);
            t[1] = 0;
            t[2] = (int32_t)blocks[k];
            LaunchGroup g;
            g.probs = d_desc;
            g.pidx = d_tab + 3 * (4 * p + k);
            g.toff = g.pidx + 1;
            g.count = 1;
            g.blocks = (int32_t)blocks[k];
            if (k < 3) H->sk[k][p] = g;
            else H->sum[p] = g;
        }
    }
    // the problem's n-side sums add the panels' split slots
    W.ypart = scn;
    W.s_atx = (int32_t)off[np];
    W.s_f = (int32_t)offf[np];
    hipError_t e = hipMemcpy(d_desc, hd.data(), sizeof(Prob) * hd.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(d_tab, tab.data(), sizeof(int32_t) * tab.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(P->d_probs, &W, sizeof(Prob), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipStreamCreate(&H->cs);
    for (int i = 0; i < HS_NB && e == hipSuccess; i++) {
        e = hipEventCreateWithFlags(&H->copied[i], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&H->freed[i], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&H->start, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "panel set-up");
    return COR_OK;
}

cor_status run_host(const cor_problem& p, const cor_opts* opts, int64_t panel_rows,
                    cor_info* info, hipStream_t s) {
    cor_status st = validate(p);
    if (st != COR_OK) return st;
    if (opts && (opts->report || opts->compress == COR_M_EXPLICIT || opts->orient == COR_ULV))
        return fail(COR_E_INVAL, "A in host memory: no report, no COR_M_EXPLICIT, no COR_ULV");
    Plan* P = nullptr;
    st = plan_create(&p, 1, opts, &P, nullptr, false);
    if (st != COR_OK) return st;
    st = host_setup(P, p, panel_rows, opts && opts->fused_power ? 1 : 0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (st == COR_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        st = fail(COR_E_DEVICE, "timing events");
    if (st == COR_OK) {
        (void)hipEventRecord(e0, s);
        st = plan_run(P, s);
        (void)hipEventRecord(e1, s);
    }
    const cor_status st_info = plan_info(P, info, s);
    if (st == COR_OK) st = st_info;
    if (st == COR_OK && info) {
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        info->device_ms = ms;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    plan_destroy(P, nullptr);
    return st;
}

void release_all() {
    std::lock_guard<std::mutex> lk(g_cache.mu);
    std::vector<Cache::Item> keep;
    for (auto& it : g_cache.items) {
        if (it.busy) keep.push_back(it);  // running on another thread: stays cached
        else plan_destroy(it.plan, nullptr);
    }
    g_cache.items.swap(keep);
}

// ---------------------------------------------------------------------------
// The split tuner: for the problem's shape (URV, default options), the mean
// time of each pass kernel over `reps` launches for candidate split counts,
// A X first (A^T X at the rule's choice), then A^T X with the best A X; the
// fastest pair goes into the table.  Candidates keep at least one K tile per
// split and at most 4096 blocks per launch.
// ---------------------------------------------------------------------------
static cor_status tune_measure(const cor_problem& p, int32_t s_ax, int32_t s_atx, int reps,
                               hipStream_t s, double* us_ax, double* us_atx, int32_t* got_ax,
                               int32_t* got_atx) {
    g_force_ax = s_ax;
    g_force_atx = s_atx;
    Plan* P = nullptr;
    cor_status st = plan_create(&p, 1, nullptr, &P, nullptr, false);
    g_force_ax = g_force_atx = 0;
    if (st != COR_OK) return st;
    *got_ax = P->lay[0].s_ax;
    *got_atx = P->lay[0].s_atx;
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    hipError_t he = hipSuccess;
    for (int i = 0; i < 3 && he == hipSuccess; i++) he = hipEventCreate(&e[i]);
    if (he == hipSuccess) st = plan_run(P, s);  // every operand initialised
    if (he == hipSuccess && st == COR_OK) {
        he = hipEventRecord(e[0], s);
        for (int r = 0; r < reps && he == hipSuccess; r++) he = run_sketch(P, P->skAX, false, 0, s);
        if (he == hipSuccess) he = hipEventRecord(e[1], s);
        for (int r = 0; r < reps && he == hipSuccess; r++) he = run_sketch(P, P->skATX, true, 0, s);
        if (he == hipSuccess) he = hipEventRecord(e[2], s);
        if (he == hipSuccess) he = hipEventSynchronize(e[2]);
        float a = 0.0f, b = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&a, e[0], e[1]);
        if (he == hipSuccess) he = hipEventElapsedTime(&b, e[1], e[2]);
        *us_ax = 1e3 * a / reps;
        *us_atx = 1e3 * b / reps;
    }
    for (int i = 0; i < 3; i++)
        if (e[i]) (void)hipEventDestroy(e[i]);
    (void)hipStreamSynchronize(s);
    plan_destroy(P, nullptr);
    if (he != hipSuccess) return hip_fail(he, "tuning runs");
    return st;
}

static cor_status tune_problem(const cor_problem& p, int reps, hipStream_t s, int32_t* s_ax,
                               int32_t* s_atx) {
    cor_status st = validate(p);
    if (st != COR_OK) return st;
    reps = std::max(1, std::min(reps, 100));
    const int l = p.k + p.p, lp = (int)roundup(l, 16), nt = lp / 16;
    const int bk = sketch_k_tile(p.prec);
    const int64_t nrb_ax = cdiv(p.m, sketch_rows_per_block(p.prec, nt, false));
    const int64_t nrb_atx = cdiv(p.n, sketch_rows_per_block(p.prec, nt, true));
    const int cand[] = {1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 56, 64};
    auto list = [&](int64_t K, int64_t nrb) {
        std::vector<int32_t> out;
        for (int c : cand) {
            int32_t sp = 0;
            int64_t kc = 0;
            apply_splits(K, bk, c, &sp, &kc);
            if (nrb * sp > 4096) break;
            if (std::find(out.begin(), out.end(), sp) == out.end()) out.push_back(sp);
        }
        return out;
    };
    double best_ax = 1e30, best_atx = 1e30, u_ax = 0, u_atx = 0;
    int32_t b_ax = 0, b_atx = 0, g_ax = 0, g_atx = 0;
    for (int32_t c : list(p.n, nrb_ax)) {
        st = tune_measure(p, c, 0, reps, s, &u_ax, &u_atx, &g_ax, &g_atx);
        if (st != COR_OK) return st;
        if (u_ax < best_ax) { best_ax = u_ax; b_ax = g_ax; }
    }
    for (int32_t c : list(p.m, nrb_atx)) {
        st = tune_measure(p, b_ax, c, reps, s, &u_ax, &u_atx, &g_ax, &g_atx);
        if (st != COR_OK) return st;
        if (u_atx < best_atx) { best_atx = u_atx; b_atx = g_atx; }
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[TuneKey{p.m, p.n, l, p.prec}] = TuneVal{b_ax, b_atx, best_ax, best_atx};
    }
    release_all();  // cached plans of this shape carry the old splits
    if (s_ax) *s_ax = b_ax;
    if (s_atx) *s_atx = b_atx;
    return COR_OK;
}

// JSON: {"version": 1, "entries": [{"m": .., "n": .., "l": .., "prec": ..,
// "s_ax": .., "s_atx": .., "us_ax": .., "us_atx": ..}, ...]}
static cor_status tune_save_file(const char* path) {
    FILE* f = fopen(path, "w");
    if (!f) return fail(COR_E_INVAL, std::string("cannot write ") + path);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    fprintf(f, "{\"version\": 1, \"entries\": [");
    bool first = true;
    for (const auto& kv : g_tune) {
        fprintf(f, "%s\n {\"m\": %lld, \"n\": %lld, \"l\": %d, \"prec\": %d, \"s_ax\": %d, "
                   "\"s_atx\": %d, \"us_ax\": %.3f, \"us_atx\": %.3f}",
                first ? "" : ",", (long long)kv.first.m, (long long)kv.first.n, kv.first.l,
                kv.first.prec, kv.second.s_ax, kv.second.s_atx, kv.second.us_ax,
                kv.second.us_atx);
        first = false;
    }
    fprintf(f, "\n]}\n");
    const bool ok = fclose(f) == 0;
    return ok ? COR_OK : fail(COR_E_INVAL, std::string("cannot write ") + path);
}

static bool json_num(const std::string& obj, const char* key, double* v) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char* end = nullptr;
    *v = strtod(obj.c_str() + p + 1, &end);
    return end != obj.c_str() + p + 1;
}

cor_status tune_load_file(const char* path) {
    FILE* f = fopen(path, "r");
    if (!f) return fail(COR_E_INVAL, std::string("cannot read ") + path);
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) txt.append(buf, got);
    fclose(f);
    const size_t arr = txt.find("\"entries\"");
    if (arr == std::string::npos) return fail(COR_E_INVAL, "no entries in the tuning file");
    std::vector<std::pair<TuneKey, TuneVal>> add;
    size_t pos = txt.find('[', arr);
    while (pos != std::string::npos) {
        const size_t a = txt.find('{', pos), b = txt.find('}', a == std::string::npos ? pos : a);
        if (a == std::string::npos || b == std::string::npos) break;
        const std::string obj = txt.substr(a, b - a + 1);
        double m, n, l, pr, sa, st, ua = 0, ut = 0;
        if (!json_num(obj, "m", &m) || !json_num(obj, "n", &n) || !json_num(obj, "l", &l) ||
            !json_num(obj, "prec", &pr) || !json_num(obj, "s_ax", &sa) ||
            !json_num(obj, "s_atx", &st))
            return fail(COR_E_INVAL, "malformed tuning entry");
        (void)json_num(obj, "us_ax", &ua);
        (void)json_num(obj, "us_atx", &ut);
        if (sa < 1 || sa > 64 || st < 1 || st > 64 || m < 1 || n < 1 || l < 2 || l > LMAX ||
            !valid_prec((int)pr))
            return fail(COR_E_INVAL, "tuning entry out of range");
        add.push_back({TuneKey{(int64_t)m, (int64_t)n, (int32_t)l, (int32_t)pr},
                       TuneVal{(int32_t)sa, (int32_t)st, ua, ut}});
        pos = b + 1;
    }
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (auto& kv : add) g_tune[kv.first] = kv.second;
    }
    release_all();
    return COR_OK;
}

}  // namespace cor

// ===========================================================================
// C ABI
// ===========================================================================
using namespace cor;

extern "C" {

cor_status cor_utv(const void* A, int64_t m, int64_t n, int32_t k, int32_t p, int32_t q,
                   uint64_t seed, int32_t prec, double* U, double* T, double* V, cor_info* info,
                   void* stream) {
    if (prec == COR_FP8) return fail(COR_E_INVAL, "COR_FP8 needs a column scale: use cor_utv_ex");
    cor_problem pr{};
    pr.A = A;
    pr.m = m; pr.n = n; pr.lda = n;
    pr.k = k; pr.p = p; pr.q = q;
    pr.prec = prec;
    pr.seed = seed;
    pr.U = U; pr.T = T; pr.V = V;
    return run_single(pr, nullptr, info, (hipStream_t)stream);
}

cor_status cor_utv_ex(const cor_problem* prob, const cor_opts* opts, cor_info* info,
                      void* stream) {
    if (!prob) return fail(COR_E_INVAL, "null problem");
    return run_single(*prob, opts, info, (hipStream_t)stream);
}

cor_status cor_tune(const cor_problem* prob, int32_t reps, int32_t* s_ax, int32_t* s_atx,
                    void* stream) {
    if (!prob) return fail(COR_E_INVAL, "null problem");
    return tune_problem(*prob, reps, (hipStream_t)stream, s_ax, s_atx);
}

cor_status cor_tune_save(const char* path) {
    if (!path) return fail(COR_E_INVAL, "null path");
    return tune_save_file(path);
}

cor_status cor_tune_load(const char* path) {
    if (!path) return fail(COR_E_INVAL, "null path");
    return tune_load_file(path);
}

cor_status cor_tune_clear(void) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune.clear();
    }
    release_all();
    return COR_OK;
}

cor_status cor_utv_host(const cor_problem* prob, const cor_opts* opts, int64_t panel_rows,
                        cor_info* info, void* stream) {
    if (!prob) return fail(COR_E_INVAL, "null problem");
    return run_host(*prob, opts, panel_rows, info, (hipStream_t)stream);
}

cor_status cor_utv_batched(const cor_problem* probs, int32_t count, const cor_opts* opts,
                           cor_info* infos, void* stream) {
    if (count == 0) return COR_OK;
    Plan* P = nullptr;
    cor_status st = plan_create(probs, count, opts, &P, nullptr, false);
    if (st != COR_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        plan_destroy(P, nullptr);
        return fail(COR_E_DEVICE, "event creation failed");
    }
    (void)hipEventRecord(e0, s);
    st = plan_run(P, s);
    (void)hipEventRecord(e1, s);
    if (st == COR_OK) st = plan_info(P, infos, s);
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (infos)
        for (int i = 0; i < count; i++) infos[i].device_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    plan_destroy(P, nullptr);
    return st;
}

cor_status cor_plan_create(const cor_problem* probs, int32_t count, const cor_opts* opts,
                           cor_plan** plan) {
    if (!plan) return fail(COR_E_INVAL, "null plan pointer");
    Plan* P = nullptr;
    cor_status st = plan_create(probs, count, opts, &P, nullptr, false);
    if (st == COR_OK) *plan = reinterpret_cast<cor_plan*>(P);
    return st;
}

cor_status cor_plan_run(cor_plan* plan, void* stream) {
    if (!plan) return fail(COR_E_INVAL, "null plan");
    return plan_run(reinterpret_cast<Plan*>(plan), (hipStream_t)stream);
}

cor_status cor_plan_capture(cor_plan* plan, void* stream) {
    if (!plan) return fail(COR_E_INVAL, "null plan");
    return plan_capture(reinterpret_cast<Plan*>(plan), (hipStream_t)stream);
}

cor_status cor_plan_info(cor_plan* plan, cor_info* infos, void* stream) {
    if (!plan) return fail(COR_E_INVAL, "null plan");
    return plan_info(reinterpret_cast<Plan*>(plan), infos, (hipStream_t)stream);
}

cor_status cor_plan_destroy(cor_plan* plan) {
    plan_destroy(reinterpret_cast<Plan*>(plan), nullptr);
    return COR_OK;
}

size_t cor_workspace_bytes(int64_t m, int64_t n, int32_t l, int32_t prec) {
    if (m < 1 || n < 1 || l < 2 || l > LMAX || !valid_prec(prec)) return 0;
    return workspace_bytes(m, n, l, prec);
}

cor_status cor_quantize(const float* A32, int64_t m, int64_t n, int64_t lda, int32_t to,
                        void* out, float* colscale, void* stream) {
    if (!A32 || !out || m < 0 || n < 0 || lda < n) return fail(COR_E_INVAL, "bad arguments");
    if (to != COR_BF16 && to != COR_FP8) return fail(COR_E_INVAL, "target must be BF16 or FP8");
    if (to == COR_FP8 && !colscale) return fail(COR_E_INVAL, "FP8 needs colscale");
    hipError_t e = launch_quantize(A32, m, n, lda, to, out, colscale, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "quantize");
    return COR_OK;
}

cor_status cor_omega(uint64_t seed, int64_t n, int32_t l, double* out, void* stream) {
    if (!out || n < 0 || l < 0) return fail(COR_E_INVAL, "bad arguments");
    hipError_t e = launch_omega_raw(seed, n, l, out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "omega");
    return COR_OK;
}

cor_status cor_profile_enable(int32_t on) {
    std::lock_guard<std::mutex> lk(g_prof.mu);
    g_prof.on = on & 3;
    return COR_OK;
}

cor_status cor_profile_read(double* ms, int64_t* launches, double* bytes, double* flops) {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pend;
    double b, f;
    int64_t n;
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        pend.swap(g_prof.pending);
        b = g_prof.bytes; f = g_prof.flops; n = g_prof.launches;
        g_prof.bytes = g_prof.flops = 0.0;
        g_prof.launches = 0;
    }
    double tot = 0.0;
    for (auto& pr : pend) {
        hipError_t e = hipEventSynchronize(pr.second);
        if (e != hipSuccess) return hip_fail(e, "profile events");
        float x = 0.0f;
        e = hipEventElapsedTime(&x, pr.first, pr.second);
        if (e != hipSuccess) return hip_fail(e, "profile events");
        tot += x;
    }
    {
        std::lock_guard<std::mutex> lk(g_prof.mu);
        for (auto& pr : pend) g_prof.free_ev.push_back(pr);
    }
    if (ms) *ms = tot;
    if (launches) *launches = n;
    if (bytes) *bytes = b;
    if (flops) *flops = f;
    return COR_OK;
}

const char* cor_status_string(int32_t st) {
    switch (st) {
        case COR_OK: return "ok";
        case COR_E_INVAL: return "invalid argument";
        case COR_E_NOMEM: return "out of memory";
        case COR_E_DEVICE: return "device error";
        case COR_E_NUMERIC: return "numerical failure";
        case COR_E_BUSY: return "busy";
        case COR_E_NOTFOUND: return "not found";
    }
    return "unknown status";
}

const char* cor_last_error(void) { return g_last_error.c_str(); }

cor_status cor_release(void) {
    release_all();
    return COR_OK;
}

}  // extern "C"

