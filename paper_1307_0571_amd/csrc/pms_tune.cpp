// Autotuner for the search parameters (pms_autotune, include/pms.h).
//
// Every setting of pms_tune except the S_1 window range gives the same motif
// sets, so the fastest one can be chosen by measurement, in this order: the
// staged survivors per tail batch (LDS per wave, hence resident waves), the
// part size, the persistent waves per CU, the threshold t (Section 2.2 and
// Appendix D leave it to be set empirically), the Theorem 1 survivor filter
// and the l-mer width.  The tuner times the whole device pipeline on a sample of the
// caller's instances and walks the parameters one at a time (coordinate
// descent from the library's defaults), keeping a change only when it is at
// least 2% faster.  A candidate whose motif counts differ from the first
// run's is rejected (a guard: the method is exact for every setting).
//
// Results are cached by the batch's shape -- the distinct (l, d, n/8,
// m/256) of its instances and log2 of their number -- in the process and,
// when PMS_TUNE_CACHE names a file, in that file (one line per shape).
// pms_solve_batch and pms_batch_create with tune == NULL use a cached entry
// for their shape when there is one.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pms.h"
#include "pms_internal.h"

namespace {

std::mutex g_mu;
std::map<std::string, pms_tune> g_cache;
bool g_loaded = false;

std::string shape_key(const pms_instance* inst, int count) {
    std::set<std::tuple<int, int, int, int, int>> shapes;
    for (int i = 0; i < count; i++)
        shapes.insert(std::make_tuple(inst[i].l, inst[i].d, inst[i].n / 8, inst[i].m / 256,
                                      inst[i].alphabet ? (int)strlen(inst[i].alphabet) : 0));
    std::string k;
    char buf[80];
    for (const auto& s : shapes) {
        // the alphabet's size is part of the key only when it is not 4
        if (std::get<4>(s) == 4)
            snprintf(buf, sizeof buf, "%d,%d,%d,%d;", std::get<0>(s), std::get<1>(s),
                     std::get<2>(s), std::get<3>(s));
        else
            snprintf(buf, sizeof buf, "%d,%d,%d,%d,a%d;", std::get<0>(s), std::get<1>(s),
                     std::get<2>(s), std::get<3>(s), std::get<4>(s));
        k += buf;
    }
    int lg = 0;
    while ((1 << (lg + 1)) <= count) lg++;
    snprintf(buf, sizeof buf, "c%d", lg);
    return k + buf;
}

void load_file_locked() {
    if (g_loaded) return;
    g_loaded = true;
    const char* path = getenv("PMS_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "r");
    if (!f) return;
    char line[8192];
    while (fgets(line, sizeof line, f)) {
        char* tab = strchr(line, '\t');
        if (!tab) continue;
        *tab = 0;
        pms_tune t{};
        int th, lw, tr, wpc, sp, sc;
        if (sscanf(tab + 1, "%d %d %d %d %d %d", &th, &lw, &tr, &wpc, &sp, &sc) != 6) continue;
        t.threshold = th;
        t.lmer_words = lw;
        t.triple_filter = tr;
        t.waves_per_cu = wpc;
        t.split = sp;
        t.stage_cap = sc;
        g_cache[line] = t;
    }
    fclose(f);
}

void store(const std::string& key, const pms_tune& t) {
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_locked();
    g_cache[key] = t;
    const char* path = getenv("PMS_TUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s\t%d %d %d %d %d %d\n", key.c_str(), t.threshold, t.lmer_words, t.triple_filter,
            t.waves_per_cu, t.split, t.stage_cap);
    fclose(f);
}

// Device time of one pipeline run (ms) and the motif counts; +inf on error.
double time_run(const std::vector<pms_instance>& s, const pms_tune& t, std::vector<int64_t>* counts) {
    pms_batch* b = nullptr;
    if (pms_batch_create(s.data(), (int32_t)s.size(), &t, nullptr, 0, &b) != PMS_OK) return INFINITY;
    std::vector<pms_result> r(s.size());
    double ms = INFINITY;
    int rc = pms_batch_run(b, nullptr, 0);  // warm-up (code objects, caches)
    if (!rc) rc = pms_batch_results(b, r.data());
    for (auto& x : r) pms_result_free(&x);
    if (!rc) rc = pms_batch_run(b, nullptr, 0);
    if (!rc) rc = pms_batch_results(b, r.data());
    float ph[5];
    if (!rc && pms_batch_timings(b, ph) == PMS_OK) {
        ms = 0;
        for (float p : ph) ms += p;
        if (counts) {
            counts->resize(s.size());
            for (size_t i = 0; i < s.size(); i++) (*counts)[i] = r[i].count;
        }
    }
    for (auto& x : r) pms_result_free(&x);
    pms_batch_destroy(b);
    return ms;
}

}  // namespace

namespace pms {

// Cached tuning for this shape of batch, if any (tune == NULL callers).
bool tuned_for(const pms_instance* inst, int count, pms_tune* out) {
    if (count <= 0 || !inst) return false;
    const std::string key = shape_key(inst, count);
    std::lock_guard<std::mutex> lk(g_mu);
    load_file_locked();
    auto it = g_cache.find(key);
    if (it == g_cache.end()) return false;
    *out = it->second;
    return true;
}

}  // namespace pms

extern "C" int pms_autotune(const pms_instance* inst, int32_t count, const pms_tune* base,
                            int32_t max_runs, int32_t sample, pms_tune* out) {
    if (!out || count < 0 || (count > 0 && !inst)) return PMS_E_INVAL;
    pms_tune cur{};
    if (base) cur = *base;
    cur.s1_begin = cur.s1_end = 0;  // tuning covers whole instances
    if (count == 0) {
        *out = cur;
        return PMS_OK;
    }
    if (max_runs <= 0) max_runs = 16;
    if (sample <= 0) sample = 32;
    // an evenly spread sample of the instances
    std::vector<pms_instance> s;
    const int ns = std::min<int>(count, sample);
    for (int i = 0; i < ns; i++) s.push_back(inst[(int64_t)i * count / ns]);
    std::vector<int64_t> ref;
    double best = time_run(s, cur, &ref);
    if (!std::isfinite(best)) {
        // the base itself does not run (bad input): report it as pms_batch_create would
        pms_batch* b = nullptr;
        int rc = pms_batch_create(s.data(), (int32_t)s.size(), &cur, nullptr, 0, &b);
        if (b) pms_batch_destroy(b);
        return rc ? rc : PMS_E_DEVICE;
    }
    int runs = 1;
    struct Dim {
        int32_t pms_tune::*field;
        std::vector<int32_t> values;
    };
    // the threshold after the launch parameters: it changes the work itself
    // (a stack of 4 instead of 3 is 30% faster on protein batches and 4x
    // slower on the DNA mix), and taken first from a sample it can lock the
    // descent into a stack size the whole batch does not favour
    const std::vector<Dim> dims = {
        {&pms_tune::stage_cap, {256, 384, 512, 768, 1024, 2048}},
        {&pms_tune::split, {16, 24, 48, 64}},
        {&pms_tune::waves_per_cu, {8, 12, 16, 24}},
        {&pms_tune::threshold, {3, 4, 2}},
        {&pms_tune::triple_filter, {-1}},
        {&pms_tune::lmer_words, {2}},
    };
    bool wide = false;  // l > 32, or an alphabet of more than 4 letters: one l-mer class
    for (const auto& x : s) wide |= x.l > 32 || (x.alphabet && strlen(x.alphabet) > 4);
    for (int pass = 0; pass < 2 && runs < max_runs; pass++) {
        bool improved = false;
        for (const Dim& dim : dims) {
            if (dim.field == &pms_tune::lmer_words && wide) continue;
            for (int32_t v : dim.values) {
                if (runs >= max_runs) break;
                if (cur.*dim.field == v) continue;
                pms_tune cand = cur;
                cand.*dim.field = v;
                std::vector<int64_t> cnt;
                const double ms = time_run(s, cand, &cnt);
                runs++;
                if (!std::isfinite(ms)) continue;
                if (cnt != ref) {
                    fprintf(stderr, "pms_autotune: a candidate setting changed the motif counts; "
                                    "rejected\n");
                    continue;
                }
                if (ms < 0.98 * best) {
                    best = ms;
                    cur = cand;
                    improved = true;
                }
            }
        }
        if (!improved) break;
    }
    *out = cur;
    store(shape_key(inst, count), cur);
    return PMS_OK;
}
