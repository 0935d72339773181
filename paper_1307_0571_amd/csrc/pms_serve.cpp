// Serving: continuous batching of independent requests (pms_stream_*).
//
// Requests are validated and copied on submit, with an estimate of their
// work: the Appendix D cost model at its best stack size plus the Appendix C
// expected number of spurious motifs (the output the search must emit and
// check).  Worker threads repeatedly form a device pass from the queue:
// requests that have waited longer than kAgeLimit first (oldest first), then
// the cheapest, admitting a request while the pass's planned device memory
// plus what other passes hold stays within the stream's cap, and without
// mixing requests whose estimates differ by more than kMixRatio (a pass lasts
// as long as its heaviest member).  The pass runs with the batched pipeline
// (one launch per phase for all its instances).  A request that arrives while
// a pass is on the device joins a later pass; with more than one worker,
// passes overlap on the device.  Each ticket's result is the set the instance
// has alone: instances in a pass never share data.
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

namespace {

struct Request {
    uint64_t ticket = 0;
    std::vector<std::string> seqs;
    std::vector<const char*> ptrs;
    std::string alphabet;
    pms_instance inst{};
    size_t bytes = 0;     // planned device bytes when run alone
    int status = PMS_E_AGAIN;
    pms_result result{};
    bool taken = false;   // result handed to the caller
    double est = 0;       // estimated work (arbitrary units, for ordering)
    std::chrono::steady_clock::time_point t_submit;
};

constexpr double kAgeLimitS = 30.0;  // waited longer: admitted first, oldest first
constexpr double kMixRatio = 16.0;   // largest / smallest estimate within one pass

// |{x : Hd(x, u) <= d}| for one l-mer u over a 4-letter alphabet (Appendix C).
double ball(int l, int d) {
    double s = 0, c = 1;  // c = C(l, i)
    for (int i = 0; i <= d && i <= l; i++) {
        s += c * std::pow(3.0, i);
        c = c * (l - i) / (i + 1);
    }
    return s;
}

// Appendix D cost model at its best stack size plus the Appendix C expected
// number of l-mers within d of some window of every string, weighted by l.
double estimate(int n, int m, int l, int d) {
    const int r = m - l + 1;
    if (r <= 0) return 0;
    const double nd = ball(l, d), n2d = ball(l, 2 * d), all = std::pow(4.0, l);
    const double p = std::min(1.0, n2d / all), q = nd / n2d;
    double best = INFINITY, ts = 0;
    for (int t = 1; t <= n; t++) {
        const double lt = t * std::log((double)r) + 0.5 * t * (t - 1) * std::log(p);
        ts += (double)n * l * std::exp(std::min(lt, 700.0));
        const double tp = std::exp(std::min(lt + std::log(nd) + (t - 1) * std::log(q), 700.0)) * l;
        best = std::min(best, ts + tp);
    }
    const double hit = 1.0 - std::pow(1.0 - std::min(1.0, nd / all), (double)r);
    const double spurious = all * std::pow(hit, (double)n);
    return best + spurious * l * n * r;
}

}  // namespace

struct pms_stream {
    pms_stream_config cfg{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> all;
    uint64_t next_ticket = 1;
    size_t held = 0;       // device bytes of passes in flight
    int inflight = 0;      // instances in flight
    bool stopping = false;
    std::vector<std::thread> workers;
};

namespace {

size_t pass_bytes(const std::vector<std::shared_ptr<Request>>& reqs, const pms_tune* tune) {
    std::vector<pms_instance> v;
    v.reserve(reqs.size());
    for (auto& r : reqs) v.push_back(r->inst);
    size_t b = 0;
    if (pms_batch_workspace_size(v.data(), (int32_t)v.size(), tune, &b) != PMS_OK) return SIZE_MAX;
    return b;
}

void worker(pms_stream* s) {
    const pms_tune* tune = &s->cfg.tune;
    for (;;) {
        std::vector<std::shared_ptr<Request>> pass;
        size_t bytes = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
            if (s->queue.empty()) return;  // stopping and nothing queued
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
            // admit in that order while the pass fits the memory cap
            const size_t cap = (size_t)s->cfg.device_mem_cap;
            double lo_est = 0;
            for (auto& r : order) {
                if ((int)pass.size() >= s->cfg.max_wave ||
                    s->inflight + (int)pass.size() >= s->cfg.max_inflight)
                    break;
                if (!pass.empty() && !aged(r) && r->est > kMixRatio * std::max(lo_est, 1.0)) continue;
                pass.push_back(r);
                size_t b = pass_bytes(pass, tune);
                if (b == SIZE_MAX || s->held + b > cap) {
                    pass.pop_back();
                    if (pass.empty()) break;  // the first choice does not fit now
                    continue;
                }
                bytes = b;
                if (pass.size() == 1) lo_est = r->est;
            }
            for (auto& r : pass) s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
            if (pass.empty()) {
                // the first request in admission order does not fit next to
                // what is running: wait for a pass to finish (or fail it if
                // nothing runs)
                if (s->held == 0) {
                    auto r = order.front();
                    s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
                    r->status = PMS_E_NOMEM;
                    s->cv_done.notify_all();
                } else {
                    s->cv_work.wait(lk);
                }
                continue;
            }
            s->held += bytes;
            s->inflight += (int)pass.size();
        }
        std::vector<pms_instance> v;
        for (auto& r : pass) v.push_back(r->inst);
        std::vector<pms_result> outs(pass.size());
        int rc = pms_solve_batch(v.data(), (int32_t)v.size(), outs.data(), tune, nullptr);
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < pass.size(); i++) {
                pass[i]->status = rc;
                if (rc == PMS_OK) pass[i]->result = outs[i];
            }
            s->held -= bytes;
            s->inflight -= (int)pass.size();
        }
        s->cv_done.notify_all();
        s->cv_work.notify_all();
    }
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
    if (s->cfg.device_mem_cap <= 0) s->cfg.device_mem_cap = (int64_t)64 << 30;
    if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 256;
    if (s->cfg.max_wave <= 0) s->cfg.max_wave = 64;
    // one device pass at a time by default; PMS_STREAM_WORKERS raises it
    int workers = 1;
    if (const char* e = getenv("PMS_STREAM_WORKERS")) workers = std::max(1, std::min(8, atoi(e)));
    for (int i = 0; i < workers; i++) s->workers.emplace_back(worker, s);
    *out = s;
    return PMS_OK;
}

int pms_stream_submit(pms_stream* s, const pms_instance* inst, uint64_t* ticket) {
    if (!s || !inst || !ticket) return PMS_E_INVAL;
    auto r = std::make_shared<Request>();
    int rc = copy_request(inst, r.get());
    if (rc) return rc;
    // host-side validation and the instance's own memory plan
    size_t b = 0;
    rc = pms_batch_workspace_size(&r->inst, 1, &s->cfg.tune, &b);
    if (rc) return rc;
    if (b > (size_t)s->cfg.device_mem_cap) return PMS_E_NOMEM;
    r->bytes = b;
    r->est = estimate(r->inst.n, r->inst.m, r->inst.l, r->inst.d);
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
    for (auto& t : s->workers) t.join();
    for (auto& kv : s->all) pms_result_free(&kv.second->result);
    delete s;
    return PMS_OK;
}

}  // extern "C"
