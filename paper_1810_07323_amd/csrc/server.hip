// Served CoR-UTV decompositions with continuous batching.
//
// A server thread owns a pool of non-blocking HIP streams and a slot table of
// pinned host records.  Each loop iteration
//   1. admits queued requests, in arrival order, while a slot is free and the
//      request's workspace fits the remaining HBM budget;
//   2. turns the requests admitted together into one grouped plan (one launch
//      per stage covers all of them) and enqueues it on a free stream, with
//      stream-ordered allocation, so it overlaps with the rounds already on
//      the device;
//   3. retires every round whose completion event has fired: results are read
//      from the slot records, workspace returns to the budget, waiters wake.
// Requests that arrive while others run are admitted as soon as slots and
// memory free up; none waits for the whole device to drain.  Reductions have
// a fixed order per problem, so a request's result is the same alone and in
// any mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/cor_utv.h"
#include "common.h"
#include "kernels.h"
#include "runtime.h"

namespace cor {

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct SlotRec {  // pinned host record written back by the device
    int32_t flags;
    int32_t pad;
    double rep[8];
};

struct Request {
    uint64_t ticket = 0;
    cor_problem prob{};
    cor_opts opts{};
    size_t footprint = 0;
    bool convert = false;
    double t_submit = 0.0, t_done = 0.0;
    bool done = false;
    cor_status st = COR_OK;
    cor_info info{};
    void* conv = nullptr;  // BF16 copy of an FP32 A
    int slot = -1;
};

struct Round {
    std::vector<Request*> reqs;
    Plan* plan = nullptr;
    int stream = -1;
    hipEvent_t done_ev = nullptr;
};

struct Server {
    cor_server_cfg cfg{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> queue;
    std::map<uint64_t, Request*> reqs;
    std::vector<Round*> active;
    std::vector<hipStream_t> streams;
    std::vector<int> stream_busy;
    SlotRec* slots = nullptr;  // pinned, max_slots records
    std::vector<int> free_slots;
    size_t in_use = 0, high_water = 0;
    int active_reqs = 0;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread th;
    std::vector<double> lat_ms;
    double t_first = -1.0, t_last = 0.0;
    int64_t completed = 0, rejected = 0;
};

static size_t request_footprint(const cor_problem& p, const cor_opts& o, bool convert) {
    const int prec = convert ? COR_BF16 : p.prec;
    size_t b = workspace_bytes(p.m, p.n, p.k + p.p, prec, &o);
    if (convert) b += (size_t)p.m * p.n * 2 + 256;
    return b;
}

// Enqueue one round on a free stream.  Called by the server thread only.
static void launch_round(Server* S, std::vector<Request*>& adm) {
    int si = -1;
    for (size_t i = 0; i < S->streams.size(); i++)
        if (!S->stream_busy[i]) { si = (int)i; break; }
    if (si < 0) {
        hipStream_t s;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess) {
            S->streams.push_back(s);
            S->stream_busy.push_back(0);
            si = (int)S->streams.size() - 1;
        } else {
            si = 0;
        }
    }
    hipStream_t s = S->streams[si];
    Round* R = new Round();
    R->stream = si;
    std::vector<cor_problem> probs;
    std::vector<Request*> ok;
    for (Request* r : adm) {
        cor_problem p = r->prob;
        if (r->convert) {
            hipError_t e = hipMallocAsync(&r->conv, (size_t)p.m * p.n * 2, s);
            if (e == hipSuccess)
                e = launch_quantize((const float*)p.A, p.m, p.n, p.lda, COR_BF16, r->conv, nullptr, s);
            if (e != hipSuccess) {
                // Only the status is recorded here: the request stays in the
                // round and is retired (done, slot and budget returned) by
                // finish_round under the server lock.
                r->st = COR_E_DEVICE;
                continue;
            }
            p.A = r->conv;
            p.lda = p.n;
            p.prec = COR_BF16;
        }
        probs.push_back(p);
        ok.push_back(r);
    }
    cor_opts o{};
    for (Request* r : ok) o.report = std::max(o.report, r->opts.report);
    if (!ok.empty()) {  // uniform within a round
        o.cholqr2_all = ok[0]->opts.cholqr2_all;
        o.compress = ok[0]->opts.compress;
        o.orient = ok[0]->opts.orient;
        o.fused_power = ok[0]->opts.fused_power;
    }
    cor_status st = COR_OK;
    if (!ok.empty()) st = plan_create(probs.data(), (int32_t)probs.size(), &o, &R->plan, s, true);
    if (st == COR_OK && R->plan) st = plan_run(R->plan, s);
    if (st == COR_OK && R->plan) {
        for (size_t i = 0; i < ok.size(); i++) {
            const Prob& d = plan_desc(R->plan, (int)i);
            SlotRec* rec = S->slots + ok[i]->slot;
            (void)hipMemcpyAsync(&rec->flags, d.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s);
            (void)hipMemcpyAsync(rec->rep, d.rep, sizeof(rec->rep), hipMemcpyDeviceToHost, s);
        }
    } else {
        for (Request* r : ok) r->st = st == COR_OK ? COR_E_DEVICE : st;
    }
    (void)hipEventCreateWithFlags(&R->done_ev, hipEventDisableTiming);
    (void)hipEventRecord(R->done_ev, s);
    R->reqs = adm;
    S->stream_busy[si] = 1;
    S->active.push_back(R);
}

static void finish_round(Server* S, Round* R) {
    hipStream_t s = S->streams[R->stream];
    if (R->plan) plan_destroy(R->plan, s);
    const double t = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    for (Request* r : R->reqs) {
        if (r->conv) (void)hipFreeAsync(r->conv, s);
        r->conv = nullptr;
        if (r->st == COR_OK) {
            const SlotRec* rec = S->slots + r->slot;
            r->info.flags = rec->flags;
            r->info.err_l = rec->rep[0];
            r->info.err_k = rec->rep[1];
            r->info.orth_u = rec->rep[2];
            r->info.orth_v = rec->rep[3];
            if (rec->flags & FLAG_NONFINITE) r->st = COR_E_NUMERIC;
        }
        r->info.l = r->prob.k + r->prob.p;
        r->t_done = t;
        r->info.device_ms = (t - r->t_submit) * 1e3;
        r->done = true;
        S->in_use -= r->footprint;
        S->active_reqs--;
        S->free_slots.push_back(r->slot);
        S->lat_ms.push_back(r->info.device_ms);
        S->completed++;
        S->t_last = t;
    }
    S->stream_busy[R->stream] = 0;
    (void)hipEventDestroy(R->done_ev);
    delete R;
    S->cv_done.notify_all();
}

static void server_loop(Server* S) {
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<Request*> adm;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->active.empty())
                S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            if (S->stop && S->queue.empty() && S->active.empty()) break;
            while (!S->queue.empty() && !S->free_slots.empty()) {
                Request* r = S->queue.front();
                if (S->in_use + r->footprint > S->cfg.hbm_budget) break;
                S->queue.pop_front();
                r->slot = S->free_slots.back();
                S->free_slots.pop_back();
                S->in_use += r->footprint;
                S->active_reqs++;
                adm.push_back(r);
            }
            S->high_water = std::max(S->high_water, S->in_use);
        }
        if (!adm.empty()) {
            // one round per combination of the options that change the
            // stage sequence (orthonormalisation, compression, orientation,
            // the fused power step, which also needs one q per round); the
            // report option does not change the results
            std::map<int, std::vector<Request*>> part;
            for (Request* r : adm) {
                const int f = r->opts.fused_power ? 1 : 0;
                part[(r->opts.cholqr2_all ? 1 : 0) + 2 * r->opts.compress + 8 * r->opts.orient +
                     16 * f + 32 * f * r->prob.q]
                    .push_back(r);
            }
            for (auto& kv : part) launch_round(S, kv.second);
        }
        bool progressed = !adm.empty();
        for (size_t i = 0; i < S->active.size();) {
            Round* R = S->active[i];
            if (hipEventQuery(R->done_ev) == hipSuccess) {
                S->active.erase(S->active.begin() + i);
                finish_round(S, R);
                progressed = true;
            } else {
                i++;
            }
        }
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace cor

using namespace cor;

extern "C" {

cor_status cor_server_create(const cor_server_cfg* cfg, cor_server** server) {
    if (!server) return fail(COR_E_INVAL, "null server pointer");
    Server* S = new Server();
    if (cfg) S->cfg = *cfg;
    if (S->cfg.hbm_budget == 0) S->cfg.hbm_budget = (size_t)64 << 30;
    if (S->cfg.max_slots <= 0) S->cfg.max_slots = 32;
    if (S->cfg.convert_f32_to != 0 && S->cfg.convert_f32_to != COR_F32 &&
        S->cfg.convert_f32_to != COR_BF16) {
        delete S;
        return fail(COR_E_INVAL, "convert_f32_to must be COR_F32 or COR_BF16");
    }
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return fail(COR_E_DEVICE, "no device");
    }
    if (hipHostMalloc((void**)&S->slots, sizeof(SlotRec) * S->cfg.max_slots, hipHostMallocDefault) !=
        hipSuccess) {
        delete S;
        return fail(COR_E_NOMEM, "pinned slot table");
    }
    for (int i = S->cfg.max_slots - 1; i >= 0; i--) S->free_slots.push_back(i);
    S->th = std::thread(server_loop, S);
    *server = reinterpret_cast<cor_server*>(S);
    return COR_OK;
}

cor_status cor_server_submit(cor_server* server, const cor_problem* prob, const cor_opts* opts,
                             uint64_t* ticket) {
    Server* S = reinterpret_cast<Server*>(server);
    if (!S || !prob || !ticket) return fail(COR_E_INVAL, "null argument");
    const cor_problem& p = *prob;
    // Shape checks mirror the single call.
    const int64_t l = (int64_t)p.k + p.p;
    if (!p.A || !p.U || !p.T || !p.V || p.k < 1 || p.p < 0 || p.q < 0 || p.q > 16 || l < 2 ||
        l >= std::min(p.m, p.n) || l > LMAX || p.lda < p.n || p.prec < COR_F64 ||
        p.prec > COR_FP8 || (p.prec == COR_FP8 && !p.colscale) ||
        (opts && (opts->compress < COR_M_R2T || opts->compress > COR_M_APPROX ||
                  (opts->orient != COR_URV && opts->orient != COR_ULV) ||
                  (opts->orient == COR_ULV && p.prec == COR_FP8)))) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->rejected++;
        return fail(COR_E_INVAL, "malformed request");
    }
    const bool convert = S->cfg.convert_f32_to == COR_BF16 && p.prec == COR_F32;
    if (opts && opts->fused_power &&
        (convert || fused_check(p, opts->orient == COR_ULV ? 1 : 0) != COR_OK)) {
        std::lock_guard<std::mutex> lk(S->mu);
        S->rejected++;
        return fail(COR_E_INVAL, "the fused power step cannot run this request (FP32 or FP64 "
                                 "passes, l <= 64, n within the limits of cor_opts)");
    }
    Request* r = new Request();
    r->prob = p;
    if (opts) r->opts = *opts;
    r->convert = convert;
    r->footprint = request_footprint(p, r->opts, r->convert);
    if (r->footprint > S->cfg.hbm_budget) {
        delete r;
        std::lock_guard<std::mutex> lk(S->mu);
        S->rejected++;
        return fail(COR_E_INVAL, "request can never fit the HBM budget");
    }
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        if (S->t_first < 0) S->t_first = r->t_submit;
        S->reqs[r->ticket] = r;
        S->queue.push_back(r);
        *ticket = r->ticket;
    }
    S->cv_work.notify_one();
    return COR_OK;
}

static cor_status take_result(Server* S, std::map<uint64_t, Request*>::iterator it,
                              cor_info* info) {
    Request* r = it->second;
    if (info) *info = r->info;
    cor_status st = r->st;
    S->reqs.erase(it);
    delete r;
    return st;
}

cor_status cor_server_poll(cor_server* server, uint64_t ticket, cor_info* info) {
    Server* S = reinterpret_cast<Server*>(server);
    if (!S) return fail(COR_E_INVAL, "null server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return COR_E_NOTFOUND;
    if (!it->second->done) return COR_E_BUSY;
    return take_result(S, it, info);
}

cor_status cor_server_wait(cor_server* server, uint64_t ticket, cor_info* info) {
    Server* S = reinterpret_cast<Server*>(server);
    if (!S) return fail(COR_E_INVAL, "null server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return COR_E_NOTFOUND;
    Request* r = it->second;
    S->cv_done.wait(lk, [&] { return r->done; });
    return take_result(S, S->reqs.find(ticket), info);
}

cor_status cor_server_stats_get(cor_server* server, cor_server_stats* st) {
    Server* S = reinterpret_cast<Server*>(server);
    if (!S || !st) return fail(COR_E_INVAL, "null argument");
    std::lock_guard<std::mutex> lk(S->mu);
    cor_server_stats o{};
    std::vector<double> v = S->lat_ms;
    std::sort(v.begin(), v.end());
    auto pct = [&](double p) {
        if (v.empty()) return 0.0;
        size_t i = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * v.size()) - 1);
        return v[i];
    };
    o.p50_ms = pct(0.50);
    o.p99_ms = pct(0.99);
    double sum = 0.0;
    for (double x : v) sum += x;
    o.mean_ms = v.empty() ? 0.0 : sum / v.size();
    o.completed = S->completed;
    o.queued = (int64_t)S->queue.size();
    o.active = S->active_reqs;
    o.rejected = S->rejected;
    o.hbm_in_use = S->in_use;
    o.hbm_high_water = S->high_water;
    const double span = S->t_last - S->t_first;
    o.decomps_per_s = (span > 0.0 && S->completed > 0) ? S->completed / span : 0.0;
    *st = o;
    return COR_OK;
}

cor_status cor_server_destroy(cor_server* server) {
    Server* S = reinterpret_cast<Server*>(server);
    if (!S) return COR_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->th.joinable()) S->th.join();
    for (hipStream_t s : S->streams) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
    }
    for (auto& kv : S->reqs) delete kv.second;
    if (S->slots) (void)hipHostFree(S->slots);
    delete S;
    return COR_OK;
}

}  // extern "C"
