// Serving: continuous batching of independent requests (pms_stream_*).
//
// Requests are validated and copied on submit, with their device-memory
// bound (the batch plan's per-instance bytes) and an estimate of their work:
// the Appendix D cost model at its best stack size plus the Appendix C
// expected number of motifs (the output the search must emit and check).
//
// Device memory is one pool of device_mem_cap bytes, allocated on the first
// pass.  Several worker threads (pms_stream_config.workers) each form a
// device pass from the queue whenever they are free: requests that have
// waited longer than kAgeLimitS first (oldest first), then the cheapest,
// admitting a request while the pass's memory bound fits in the pool next to
// the passes already on the device, and without mixing requests whose
// estimates differ by more than kMixRatio (a pass lasts as long as its
// heaviest member).  Each worker runs its pass on its own non-blocking
// stream in its pool block (a caller workspace of pms_batch_create), so
// passes overlap on the device: a request that arrives while others run is
// admitted by the next free worker as soon as memory allows, and its
// kernels run beside theirs.  Instances in a pass never share data, so each
// ticket's result is the set the instance has alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/pms.h"
#include "pms_internal.h"

namespace {

struct Request {
    uint64_t ticket = 0;
    std::vector<std::string> seqs;
    std::vector<const char*> ptrs;
    std::string alphabet;
    pms_instance inst{};
    size_t bytes = 0;     // device bytes this request adds to a pass (upper bound)
    int status = PMS_E_AGAIN;
    pms_result result{};
    double est = 0;       // estimated work (arbitrary units, for ordering)
    bool wide = false;    // l > 32 (two 64-bit planes)
    bool letters5 = false;  // alphabet of more than 4 letters (five 32-bit planes)
    std::chrono::steady_clock::time_point t_submit;
};

constexpr double kAgeLimitS = 30.0;  // waited longer: admitted first, oldest first
constexpr double kMixRatio = 16.0;   // largest / smallest estimate within one pass
constexpr size_t kAlign = 256;

// |{x : Hd(x, u) <= d}| for one l-mer u over sigma letters (Appendix C).
double ball(int l, int d, int sigma) {
    double s = 0, c = 1;  // c = C(l, i)
    for (int i = 0; i <= d && i <= l; i++) {
        s += c * std::pow((double)(sigma - 1), i);
        c = c * (l - i) / (i + 1);
    }
    return s;
}

// Appendix D cost model at its best stack size plus the Appendix C expected
// number of l-mers within d of some window of every string, weighted by l.
double estimate(int n, int m, int l, int d, int sigma) {
    const int r = m - l + 1;
    if (r <= 0) return 0;
    const double nd = ball(l, d, sigma), n2d = ball(l, 2 * d, sigma),
                 all = std::pow((double)sigma, l);
    const double p = std::min(1.0, n2d / all), q = nd / n2d;
    double best = INFINITY, ts = 0;
    for (int t = 1; t <= n; t++) {
        const double lt = t * std::log((double)r) + 0.5 * t * (t - 1) * std::log(p);
        ts += (double)n * l * std::exp(std::min(lt, 700.0));
        const double tp = std::exp(std::min(lt + std::log(nd) + (t - 1) * std::log(q), 700.0)) * l;
        best = std::min(best, ts + tp);
    }
    return best + pms_expected_motifs(n, m, l, d, sigma) * l * n * r;
}

// First-fit allocator over the stream's device pool (offsets, host-side).
struct Pool {
    std::map<size_t, size_t> free_;  // offset -> size
    void reset(size_t bytes) {
        free_.clear();
        if (bytes) free_[0] = bytes;
    }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + kAlign - 1) / kAlign * kAlign;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

struct pms_stream {
    pms_stream_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1;
    size_t fixed = 0;        // per-pass bytes independent of its requests
    void* pool = nullptr;    // device_mem_cap bytes, allocated on first use
    bool pool_failed = false;
    Pool alloc;
    int inflight = 0;        // instances in flight
    int running = 0;         // passes on the device
    bool stopping = false;
    std::vector<std::thread> workers;
};

namespace {

void worker(pms_stream* s) {
    const pms_tune* tune = &s->cfg.tune;
    hipStream_t hs = nullptr;
    if (hipStreamCreateWithFlags(&hs, hipStreamNonBlocking) != hipSuccess) hs = nullptr;
    for (;;) {
        std::vector<std::shared_ptr<Request>> pass;
        size_t bytes = 0, off = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
            if (s->queue.empty()) break;  // stopping and nothing queued
            if (!s->pool && !s->pool_failed) {
                if (hipMalloc(&s->pool, (size_t)s->cfg.device_mem_cap) != hipSuccess) {
                    s->pool = nullptr;
                    s->pool_failed = true;
                } else {
                    s->alloc.reset((size_t)s->cfg.device_mem_cap);
                }
            }
            if (!hs || s->pool_failed) {
                for (auto& r : s->queue) r->status = PMS_E_NOMEM;
                s->queue.clear();
                s->cv_done.notify_all();
                continue;
            }
            // order: aged requests (oldest first), then the cheapest
            const auto now = std::chrono::steady_clock::now();
            std::vector<std::shared_ptr<Request>> order(s->queue.begin(), s->queue.end());
            auto aged = [&](const std::shared_ptr<Request>& r) {
                return std::chrono::duration<double>(now - r->t_submit).count() > kAgeLimitS;
            };
            std::stable_sort(order.begin(), order.end(),
                             [&](const std::shared_ptr<Request>& a, const std::shared_ptr<Request>& b) {
                                 const bool xa = aged(a), xb = aged(b);
                                 if (xa != xb) return xa;
                                 if (xa) return a->ticket < b->ticket;
                                 return a->est < b->est;
                             });
            // admit in that order while the pass's bound fits in the pool
            double lo_est = 0;
            size_t want = s->fixed;
            bool has_wide = false, has_letters5 = false;
            for (auto& r : order) {
                if ((int)pass.size() >= s->cfg.max_wave ||
                    s->inflight + (int)pass.size() >= s->cfg.max_inflight)
                    break;
                if (!pass.empty() && !aged(r) && r->est > kMixRatio * std::max(lo_est, 1.0)) continue;
                // one batch holds one l-mer class: l > 32 and large alphabets never meet
                if ((r->wide && has_letters5) || (r->letters5 && has_wide)) continue;
                size_t o = 0;
                if (!s->alloc.alloc(want + r->bytes, &o)) {
                    if (pass.empty()) break;  // the first choice does not fit now
                    continue;
                }
                s->alloc.release(o, want + r->bytes);
                pass.push_back(r);
                has_wide |= r->wide;
                has_letters5 |= r->letters5;
                want += r->bytes;
                if (pass.size() == 1) lo_est = r->est;
            }
            if (pass.empty()) {
                // the first request in admission order does not fit next to
                // what is running: wait for a pass to finish, or fail it if
                // nothing runs (it is larger than the whole pool)
                if (s->running == 0) {
                    auto r = order.front();
                    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
                    r->status = PMS_E_NOMEM;
                    s->cv_done.notify_all();
                } else {
                    s->cv_work.wait(lk);
                }
                continue;
            }
            if (!s->alloc.alloc(want, &off)) {  // cannot fail: just probed under the lock
                s->cv_work.wait(lk);
                continue;
            }
            bytes = want;
            for (auto& r : pass) s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
            s->inflight += (int)pass.size();
            s->running++;
        }
        std::vector<pms_instance> v;
        for (auto& r : pass) v.push_back(r->inst);
        std::vector<pms_result> outs(pass.size());
        pms_batch* b = nullptr;
        int rc = pms_batch_create(v.data(), (int32_t)v.size(), tune, (char*)s->pool + off, bytes, &b);
        if (!rc) rc = pms_batch_run(b, hs, 0);
        if (!rc) rc = pms_batch_results(b, outs.data());
        if (b) pms_batch_destroy(b);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < pass.size(); i++) {
                pass[i]->status = rc;
                if (rc == PMS_OK) pass[i]->result = outs[i];
            }
            s->alloc.release(off, bytes);
            s->inflight -= (int)pass.size();
            s->running--;
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
    if (hs) (void)hipStreamDestroy(hs);
}

int copy_request(const pms_instance* in, Request* r) {
    if (!in || !in->seqs || !in->alphabet || in->n < 1 || in->m < 0) return PMS_E_INVAL;
    r->seqs.resize(in->n);
    for (int i = 0; i < in->n; i++) {
        if (!in->seqs[i]) return PMS_E_INVAL;
        r->seqs[i].assign(in->seqs[i], strnlen(in->seqs[i], (size_t)in->m + 1));
        if ((int)r->seqs[i].size() != in->m) return PMS_E_INVAL;
    }
    r->ptrs.resize(in->n);
    for (int i = 0; i < in->n; i++) r->ptrs[i] = r->seqs[i].c_str();
    r->alphabet = in->alphabet;
    r->inst = pms_instance{r->ptrs.data(), in->n, in->m, r->alphabet.c_str(), in->l, in->d};
    return PMS_OK;
}

int take_result(pms_stream* s, std::map<uint64_t, std::shared_ptr<Request>>::iterator it,
                pms_result* out) {
    auto r = it->second;
    int st = r->status;
    if (out) *out = r->result;
    else pms_result_free(&r->result);
    r->result = pms_result{};
    s->all.erase(it);
    return st;
}

}  // namespace

extern "C" {

int pms_stream_create(const pms_stream_config* cfg, pms_stream** out) {
    if (!out) return PMS_E_INVAL;
    pms_stream* s = new (std::nothrow) pms_stream();
    if (!s) return PMS_E_NOMEM;
    if (cfg) s->cfg = *cfg;
    if (s->cfg.device_mem_cap <= 0) s->cfg.device_mem_cap = (int64_t)32 << 30;
    if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 256;
    if (s->cfg.max_wave <= 0) s->cfg.max_wave = 64;
    if (s->cfg.workers <= 0) s->cfg.workers = 3;
    s->cfg.workers = std::min(s->cfg.workers, 16);
    s->fixed = pms::fixed_bytes(&s->cfg.tune);
    for (int i = 0; i < s->cfg.workers; i++) s->workers.emplace_back(worker, s);
    *out = s;
    return PMS_OK;
}

int pms_stream_submit(pms_stream* s, const pms_instance* inst, uint64_t* ticket) {
    if (!s || !inst || !ticket) return PMS_E_INVAL;
    auto r = std::make_shared<Request>();
    int rc = copy_request(inst, r.get());
    if (rc) return rc;
    // host-side validation (the request's own plan)
    size_t b = 0;
    rc = pms_batch_workspace_size(&r->inst, 1, &s->cfg.tune, &b);
    if (rc) return rc;
    // letters of the (validated: distinct characters) alphabet
    const int sigma = (int)r->alphabet.size();
    r->bytes = pms::inst_bytes(inst->n, inst->m, inst->l, inst->d, sigma, &s->cfg.tune);
    if (s->fixed + r->bytes > (size_t)s->cfg.device_mem_cap) return PMS_E_NOMEM;
    r->est = estimate(r->inst.n, r->inst.m, r->inst.l, r->inst.d, sigma);
    r->wide = inst->l > 32;
    r->letters5 = sigma > 4;
    r->t_submit = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stopping) return PMS_E_ABORTED;
    r->ticket = s->next_ticket++;
    s->all[r->ticket] = r;
    s->queue.push_back(r);
    *ticket = r->ticket;
    s->cv_work.notify_one();
    return PMS_OK;
}

int pms_stream_poll(pms_stream* s, uint64_t ticket, pms_result* out) {
    if (!s) return PMS_E_INVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return PMS_E_INVAL;
    if (it->second->status == PMS_E_AGAIN) return PMS_E_AGAIN;
    return take_result(s, it, out);
}

int pms_stream_wait(pms_stream* s, uint64_t ticket, pms_result* out, int64_t timeout_us) {
    if (!s) return PMS_E_INVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return PMS_E_INVAL;
    auto r = it->second;
    auto ready = [&] { return r->status != PMS_E_AGAIN; };
    if (timeout_us < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return PMS_E_TIMEOUT;
    }
    it = s->all.find(ticket);
    if (it == s->all.end()) return PMS_E_INVAL;
    return take_result(s, it, out);
}

int pms_stream_destroy(pms_stream* s) {
    if (!s) return PMS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        for (auto& r : s->queue) r->status = PMS_E_ABORTED;
        s->queue.clear();
    }
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->all) pms_result_free(&kv.second->result);
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return PMS_OK;
}

}  // extern "C"
