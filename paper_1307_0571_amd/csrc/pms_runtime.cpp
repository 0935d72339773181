// Host runtime of libpms: validation, memory planning, launches, results.
// The C ABI is declared in include/pms.h.
//
// Streams: every stream the library creates is non-blocking, and every copy
// is asynchronous on the batch's own stream followed by a wait on that
// stream only, so batches on different streams (serving workers) overlap on
// the device and never wait for each other.  The phases of one run are
// launched back to back on the run's stream; stream order alone sequences
// them (each phase reads only what earlier phases wrote).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pms.h"
#include "pms_internal.h"

using namespace pms;

namespace {

inline int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }
inline int64_t next_pow2(int64_t x) {
    int64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

int device_cus() {
    static std::atomic<int> cus{0};
    int c = cus.load();
    if (c > 0) return c;
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return 256;
    c = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    cus.store(c);
    return c;
}

int device_lds_per_block() {
    static std::atomic<int> lds{0};
    int v = lds.load();
    if (v > 0) return v;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
        return 65536;
    lds.store(v);
    return v;
}

// |N_d| for an l-mer over an alphabet of sigma letters:
// sum_{i<=d} C(l,i) (sigma-1)^i (Appendix C).
double ball_size(int l, int d, int sigma) {
    double s = 0, c = 1;
    for (int i = 0; i <= d && i <= l; i++) {
        s += c * std::pow((double)(sigma - 1), i);
        c = c * (l - i) / (i + 1);
    }
    return s;
}

int sigma_or_dna(int sigma) { return sigma < 2 ? 4 : sigma; }

}  // namespace

// Stack size t at which the search switches to generation: minimise the
// Appendix D cost model Time_s(t) + Time_p(t) over t, with
// p = N_2d / sigma^l and q = N_d / N_2d.  On the device a stack of three is never worse than two
// once the model asks for more than one level (Theorem 1 makes the
// three-l-mer tree free of dead ends), measured on MI355X for (9,2) .. (17,6);
// the result is clamped to [2, 8].
extern "C" int pms_default_threshold(int n, int m, int l, int d, int sigma) {
    const int r = m - l + 1;
    if (r <= 0 || n <= 1) return 2;
    sigma = sigma_or_dna(sigma);
    const double nd = ball_size(l, d, sigma), n2d = ball_size(l, 2 * d, sigma);
    const double p = std::min(1.0, n2d / std::pow((double)sigma, l));
    const double q = nd / n2d;
    int best = 1;
    double best_cost = INFINITY, ts = 0;
    for (int t = 1; t <= n; t++) {
        const double lt = t * std::log((double)r) + 0.5 * t * (t - 1) * std::log(p);
        ts += (double)n * l * std::exp(std::min(lt, 700.0));
        const double tp = std::exp(std::min(lt + std::log(nd) + (t - 1) * std::log(q), 700.0)) * l;
        if (ts + tp < best_cost) {
            best_cost = ts + tp;
            best = t;
        }
    }
    const int t = best <= 1 ? 2 : std::max(3, best);
    return std::max(2, std::min(kMaxT, t));
}

// Appendix C: the expected number of l-mers within d of some window of each
// of n random strings, sigma^l (1 - (1 - N_d / sigma^l)^(m-l+1))^n.  Used to
// pre-size an instance's output buffer (the planted motif plus the spurious
// ones).
extern "C" double pms_expected_motifs(int n, int m, int l, int d, int sigma) {
    const int r = m - l + 1;
    if (r <= 0 || n < 1 || l < 1 || d < 0) return 0.0;
    sigma = sigma_or_dna(sigma);
    const double all = std::pow((double)sigma, l);
    const double p = std::min(1.0, ball_size(l, d, sigma) / all);
    // 1 - (1 - p)^r without cancellation for tiny p
    const double hit = -std::expm1((double)r * std::log1p(-std::min(p, 1.0 - 1e-300)));
    return all * std::pow(hit, (double)n);
}

namespace {

constexpr int64_t kOutCapMin = 256;
constexpr int64_t kOutCapMax = int64_t(1) << 23;  // pre-sized slots; larger sets re-run alone
// Emitted keys per distinct motif: a motif is emitted once per stack that
// generates it (several S_1 windows and several second and third members
// lie within d of it); about 2-4 on the heavy-output instances of the
// benchmark mixes, measured with the oracle's counts.
constexpr double kEmitPerMotif = 4.0;

int64_t presized_out_cap(int n, int m, int l, int d, int sigma) {
    const double e = pms_expected_motifs(n, m, l, d, sigma);
    const double want = kEmitPerMotif * e + 64.0;
    const int64_t c = want >= (double)kOutCapMax ? kOutCapMax : (int64_t)want;
    return next_pow2(std::max(kOutCapMin, c));
}

// An instance whose whole compat matrix would exceed this keeps only the
// rows of S_1's l-mers (n times smaller); its pushes test Hd <= 2d directly.
constexpr int64_t kCompatBudget = int64_t(1) << 30;

struct HostInst {
    int n, m, l, d, t, triple, s1_lo, s1_hi, c1only;
    int asize, abits;   // letters; key bits per character
    std::string alpha;  // sorted
};

// Key bits per character: 2 for alphabets of up to 4 letters (the planar
// DNA class), else ceil(log2 letters).
int key_bits(int letters) {
    if (letters <= 4) return 2;
    int b = 0;
    while ((1 << b) < letters) b++;
    return b;
}

int validate(const pms_instance& in, HostInst& h, std::vector<uint8_t>& chars,
             std::vector<uint8_t>& lut) {
    if (!in.seqs || !in.alphabet || in.n < 1 || in.m < 0 || in.l < 1 || in.d < 0 || in.d >= in.l)
        return PMS_E_INVAL;
    const size_t alen = strlen(in.alphabet);
    std::string a(in.alphabet, alen);
    std::sort(a.begin(), a.end());
    for (size_t i = 1; i < a.size(); i++)
        if (a[i] == a[i - 1]) return PMS_E_ALPHABET;
    if (a.size() < 2) return PMS_E_ALPHABET;
    uint8_t tab[256];
    memset(tab, 0xFF, sizeof(tab));
    for (size_t i = 0; i < a.size(); i++) tab[(uint8_t)a[i]] = (uint8_t)i;
    const size_t base = chars.size();
    chars.resize(base + (size_t)in.n * in.m);
    for (int i = 0; i < in.n; i++) {
        const char* s = in.seqs[i];
        if (!s) return PMS_E_INVAL;
        for (int j = 0; j < in.m; j++) {
            if (s[j] == '\0') return PMS_E_INVAL;
            if (tab[(uint8_t)s[j]] == 0xFF) return PMS_E_ALPHABET;
        }
        if (s[in.m] != '\0') return PMS_E_INVAL;
        memcpy(&chars[base + (size_t)i * in.m], s, (size_t)in.m);
    }
    const int letters = (int)a.size();
    if (letters > kMaxAlpha) return PMS_E_UNSUPPORTED;
    if (in.l > kMaxL || in.n > kMaxN || in.m - in.l + 1 > kMaxR) return PMS_E_UNSUPPORTED;
    // larger alphabets: five 32-bit planes, and keys of two words
    if (letters > 4 && (in.l > kMaxLWide || in.l > 2 * (64 / key_bits(letters))))
        return PMS_E_UNSUPPORTED;
    lut.insert(lut.end(), tab, tab + 256);
    h.n = in.n;
    h.m = in.m;
    h.l = in.l;
    h.d = in.d;
    h.asize = letters;
    h.abits = key_bits(letters);
    h.alpha = a;
    return PMS_OK;
}

// One cached arena for pms_solve / pms_solve_batch (one call at a time holds
// it; a concurrent call allocates its own).
struct DevCache {
    std::mutex mu;
    void* ptr = nullptr;
    size_t bytes = 0;
    bool busy = false;
};
DevCache g_cache;

void* cache_take(size_t bytes, bool* from_cache) {
    std::lock_guard<std::mutex> lk(g_cache.mu);
    *from_cache = false;
    if (g_cache.busy) return nullptr;
    if (g_cache.bytes < bytes) {
        if (g_cache.ptr) (void)hipFree(g_cache.ptr);
        g_cache.ptr = nullptr;
        g_cache.bytes = 0;
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        g_cache.ptr = p;
        g_cache.bytes = bytes;
    }
    g_cache.busy = true;
    *from_cache = true;
    return g_cache.ptr;
}

void cache_give(void* p) {
    std::lock_guard<std::mutex> lk(g_cache.mu);
    if (p == g_cache.ptr) g_cache.busy = false;
}

hipError_t make_stream(hipStream_t* s) { return hipStreamCreateWithFlags(s, hipStreamNonBlocking); }

}  // namespace

struct pms_batch {
    std::vector<HostInst> hin;
    std::vector<InstDev> dinst;
    std::vector<uint8_t> chars, lut;
    std::vector<int64_t> out_cap;
    LaunchPlan plan{};
    DevBufs b{};
    void* arena = nullptr;
    size_t arena_bytes = 0;
    bool own_arena = false;
    bool cached_arena = false;
    void* ext_ws = nullptr;
    size_t ext_ws_bytes = 0;
    unsigned long long item_cap = 0;
    unsigned long long part_cap = 0;
    pms_tune tune{};
    hipStream_t own_stream = nullptr;  // uploads, and runs given no stream
    hipEvent_t uploaded = nullptr;     // recorded on own_stream after the uploads
    hipStream_t last = nullptr;        // stream of the last run
    hipGraphExec_t gexec = nullptr;
    hipStream_t graph_stream = nullptr;  // stream the graph was captured on
    hipEvent_t ev[6] = {};
    bool timed = false;
    bool ran = false;
    int plan_status = PMS_OK;  // PMS_E_UNSUPPORTED when the search's LDS does not fit
    int failed = PMS_OK;  // sticky error: the batch's device state is unusable
    int words = 1;   // l-mer class (1, 2, or 3 for alphabets of more than 4 letters)
    int kwords = 1;  // u64 words per key
    std::vector<uint8_t> sort_cands;     // multi-block sort candidate records (uploaded)
    std::vector<InstCounters> last_ctr;  // counters read back by the last results call
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? PMS_OK : PMS_E_DEVICE; }

// Plan offsets and sizes; returns total device bytes.
size_t plan_layout(pms_batch* bt) {
    const int ni = (int)bt->hin.size();
    LaunchPlan& p = bt->plan;
    p.n_inst = ni;
    p.words = bt->words;
    p.kwords = bt->kwords;
    p.max_n_lmers = 0;
    p.max_r = 0;
    p.max_n = 0;
    p.level_words = 1;
    p.tmax = 2;
    int64_t chars_off = 0, lmer_off = 0, compat_off = 0, out_off = 0;
    unsigned long long items = 0;
    bt->dinst.resize(ni);
    for (int i = 0; i < ni; i++) {
        const HostInst& h = bt->hin[i];
        InstDev& d = bt->dinst[i];
        d.n = h.n;
        d.m = h.m;
        d.l = h.l;
        d.d = h.d;
        d.r = h.m >= h.l ? h.m - h.l + 1 : 0;
        d.bw = (d.r + 63) / 64;
        d.t = h.t;
        d.triple = h.triple;
        d.s1_lo = h.s1_lo;
        d.s1_hi = h.s1_hi;
        d.c1only = h.c1only;
        d.asize = h.asize;
        d.abits = h.abits;
        d.amask = h.asize >= 32 ? 0xFFFFFFFFu : (1u << h.asize) - 1u;
        d.pad = 0;
        d.chars_off = chars_off;
        d.lmer_off = lmer_off;
        d.compat_off = compat_off;
        d.out_off = out_off;
        d.out_cap = bt->out_cap[i];
        const int64_t N = (int64_t)d.n * d.r;
        chars_off += (int64_t)h.n * h.m;
        lmer_off += N;
        compat_off += (d.c1only ? (int64_t)d.r : N) * d.n * d.bw;
        out_off += d.out_cap;
        items += (unsigned long long)d.r * (unsigned long long)std::max(d.r, 1);
        p.max_n_lmers = std::max<int64_t>(p.max_n_lmers, N);
        p.max_r = std::max(p.max_r, d.r);
        p.max_n = std::max(p.max_n, d.n);
        p.level_words = std::max(p.level_words, d.n * d.bw);
        p.tmax = std::max(p.tmax, d.t);
    }
    bt->item_cap = std::max<unsigned long long>(items, 1);
    // part items: a full part queue only makes waves keep their whole item
    bt->part_cap = std::max<unsigned long long>(std::min<unsigned long long>(items, 1ull << 22), 1024);
    const int wpc = bt->tune.waves_per_cu > 0 ? bt->tune.waves_per_cu : 20;
    p.search_blocks = device_cus() * wpc;
    // the MFMA builder where the one-hot vectors are 4 bytes per character
    // (17.7 vs 27.6 ms on the batched DNA mix); the VALU one for larger
    // alphabets (32.5 ms vs 382 ms on the protein batch)
    p.compat_kernel = bt->tune.compat_kernel > 0 ? (int)bt->tune.compat_kernel
                                                 : (bt->words == 3 ? 1 : 2);
    // part size: 32 for instances up to about 12000 l-mers (the plain
    // n = 20, m = 600 ones), 64 for larger ones (the batched mix: 80 vs 68
    // instances/s, the autotuner's choice there)
    p.split = bt->tune.split > 0 ? (int)bt->tune.split : (p.max_n_lmers > 12000 ? 64 : kSplitDefault);
    // staged survivors per tail batch (LDS per wave grows with it, so it
    // trades resident waves against checks from HBM): measured on MI355X,
    // 1024 suits n*(m-l+1) up to about 12000 l-mers per instance, 256 the
    // batched mix of larger instances (with four resident waves per SIMD:
    // 78.2 instances/s, 73.4 at 512)
    if (bt->tune.stage_cap > 0)
        p.s2cap = std::max(kStageCapMin, std::min(kStageCapMax, (int)(bt->tune.stage_cap + 63) / 64 * 64));
    else
        p.s2cap = p.max_n_lmers > 12000 ? 256 : 1024;
    while (p.s2cap > kStageCapMin && search_lds_bytes(p) > (size_t)device_lds_per_block())
        p.s2cap = std::max(kStageCapMin, p.s2cap / 2 / 64 * 64);
    bt->plan_status = search_lds_bytes(p) > (size_t)device_lds_per_block() ? PMS_E_UNSUPPORTED : PMS_OK;
    const int64_t lmer_size = (int64_t)lmer_bytes(bt->words);
    size_t off = 0;
    auto take = [&](int64_t bytes) {
        size_t o = off;
        off = (size_t)align_up((int64_t)off + std::max<int64_t>(bytes, 1), 256);
        return o;
    };
    size_t o_inst = take((int64_t)ni * sizeof(InstDev));
    size_t o_chars = take(chars_off);
    size_t o_lut = take((int64_t)ni * 256);
    size_t o_lmers = take(lmer_off * lmer_size);
    size_t o_compat = take(compat_off * 8);
    size_t o_items = take((int64_t)bt->item_cap * 8);
    size_t o_parts = take((int64_t)bt->part_cap * 8);
    // deep items: searches at stack size 3 and up split across waves
    // (only when some instance's threshold exceeds 3)
    p.deep_phases = p.tmax > 3 ? p.tmax - 3 : 0;
    unsigned long long deep_items = 0;  // work items of the instances that can split deeper
    for (const InstDev& d : bt->dinst)
        if (d.t > 3) deep_items += (unsigned long long)d.r * (unsigned long long)std::max(d.r, 1);
    p.deep_cap = p.deep_phases > 0
                     ? std::min<unsigned long long>(std::max<unsigned long long>(deep_items, 1024) * 2,
                                                    1ull << 20)
                     : 1;
    size_t o_deep0 = take((int64_t)p.deep_cap * (int64_t)sizeof(DeepItem));
    size_t o_deep1 = take((int64_t)p.deep_cap * (int64_t)sizeof(DeepItem));
    size_t o_keys = take(out_off * 8 * bt->kwords);
    // multi-block sort: instances whose key area exceeds one LDS chunk get a
    // compaction area as large as their key area and one record per chunk
    const int64_t chunk = sort_chunk_keys(bt->kwords);
    int ncand = 0;
    int64_t tmp_words = 0, side_words = 0;
    p.sort_pmax = 0;
    for (const InstDev& d : bt->dinst)
        if (d.out_cap > chunk) ncand++;
    bt->sort_cands.assign((size_t)ncand * sort_cand_bytes(), 0);
    ncand = 0;
    for (int i = 0; i < ni; i++) {
        const InstDev& d = bt->dinst[i];
        if (d.out_cap <= chunk) continue;
        sort_cand_fill(bt->sort_cands.data(), ncand++, i, tmp_words, side_words);
        tmp_words += d.out_cap * bt->kwords;
        side_words += (d.out_cap / chunk) * (2 * bt->kwords + 1);
        p.sort_pmax = std::max<long long>(p.sort_pmax, d.out_cap);
    }
    p.sort_cands = ncand;
    size_t o_scand = take((int64_t)bt->sort_cands.size());
    size_t o_stmp = take(tmp_words * 8);
    size_t o_sside = take(side_words * 8);
    size_t o_ctr = take((int64_t)ni * sizeof(InstCounters));
    size_t o_q = take(kQueues * sizeof(QueueCounters));
    // offsets are stored relative to the arena; resolve later
    bt->b.inst = (InstDev*)o_inst;
    bt->b.chars = (uint8_t*)o_chars;
    bt->b.lut = (uint8_t*)o_lut;
    bt->b.lmers = (void*)o_lmers;
    bt->b.compat = (uint64_t*)o_compat;
    bt->b.items = (uint64_t*)o_items;
    bt->b.parts = (uint64_t*)o_parts;
    bt->b.deep[0] = (DeepItem*)o_deep0;
    bt->b.deep[1] = (DeepItem*)o_deep1;
    bt->b.keys = (uint64_t*)o_keys;
    bt->b.ctr = (InstCounters*)o_ctr;
    bt->b.q = (QueueCounters*)o_q;
    bt->b.sort_cand = (void*)o_scand;
    bt->b.sort_tmp = (uint64_t*)o_stmp;
    bt->b.sort_side = (uint64_t*)o_sside;
    return off;
}

}  // namespace

namespace pms {

// Upper bound of the device bytes an instance adds to a batch (20-byte
// l-mers and 2-word keys, whatever the batch's class; its work items and
// at most as many part items).
size_t inst_bytes(int n, int m, int l, int d, int sigma, const pms_tune* tune) {
    const int64_t r = m >= l ? m - l + 1 : 0;
    const int64_t N = (int64_t)n * r, bw = (r + 63) / 64;
    const int64_t cap = (tune && tune->out_capacity > 0) ? next_pow2(tune->out_capacity)
                                                          : presized_out_cap(n, m, l, d, sigma);
    const int t = (tune && tune->threshold > 0) ? std::max(2, std::min(kMaxT, (int)tune->threshold))
                                                : pms_default_threshold(n, m, l, d, sigma);
    // deep-item queues exist only in batches with a threshold above 3; two
    // queues of at most 2 * (sum of r^2, at least 1024) entries
    const int64_t deep = t > 3 ? 2 * (2 * r * std::max<int64_t>(r, 1) + 2048) * (int64_t)sizeof(DeepItem) : 0;
    // keys (2 words) plus the multi-block sort's compaction area and records
    return (size_t)((int64_t)sizeof(InstDev) + (int64_t)n * m + 256 + cap * 17 +
                    (int64_t)sort_cand_bytes() + 256 +
                    N * (int64_t)lmer_bytes(3) + N * n * bw * 8 +
                    2 * r * std::max<int64_t>(r, 1) * 8 + cap * 16 + (int64_t)sizeof(InstCounters) +
                    deep);
}

// Device bytes of a batch that do not depend on its instances (the part
// queue's minimum, queue counters, region alignment).
size_t fixed_bytes(const pms_tune* tune) {
    (void)tune;
    return (size_t)(1024 * 8 + kQueues * (int64_t)sizeof(QueueCounters) +
                    2 * (int64_t)sizeof(DeepItem) + 16 * 256);
}

}  // namespace pms

namespace {

void resolve(pms_batch* bt) {
    char* a = (char*)bt->arena;
    bt->b.inst = (InstDev*)(a + (size_t)bt->b.inst);
    bt->b.chars = (uint8_t*)(a + (size_t)bt->b.chars);
    bt->b.lut = (uint8_t*)(a + (size_t)bt->b.lut);
    bt->b.lmers = (void*)(a + (size_t)bt->b.lmers);
    bt->b.compat = (uint64_t*)(a + (size_t)bt->b.compat);
    bt->b.items = (uint64_t*)(a + (size_t)bt->b.items);
    bt->b.parts = (uint64_t*)(a + (size_t)bt->b.parts);
    bt->b.deep[0] = (DeepItem*)(a + (size_t)bt->b.deep[0]);
    bt->b.deep[1] = (DeepItem*)(a + (size_t)bt->b.deep[1]);
    bt->b.keys = (uint64_t*)(a + (size_t)bt->b.keys);
    bt->b.ctr = (InstCounters*)(a + (size_t)bt->b.ctr);
    bt->b.q = (QueueCounters*)(a + (size_t)bt->b.q);
    bt->b.sort_cand = (void*)(a + (size_t)bt->b.sort_cand);
    bt->b.sort_tmp = (uint64_t*)(a + (size_t)bt->b.sort_tmp);
    bt->b.sort_side = (uint64_t*)(a + (size_t)bt->b.sort_side);
}

void release_arena(pms_batch* bt) {
    if (bt->gexec) (void)hipGraphExecDestroy(bt->gexec);
    bt->gexec = nullptr;
    if (bt->arena) {
        if (bt->cached_arena) cache_give(bt->arena);
        else if (bt->own_arena) (void)hipFree(bt->arena);
    }
    bt->arena = nullptr;
    bt->own_arena = bt->cached_arena = false;
}

// Allocate (or adopt the workspace), then upload the inputs on the batch's
// own stream; `uploaded` marks their completion for whichever stream runs.
int materialise(pms_batch* bt, bool use_cache) {
    const size_t need = plan_layout(bt);
    if (bt->plan_status) return bt->plan_status;
    bt->arena_bytes = need;
    if (bt->ext_ws) {
        if (bt->ext_ws_bytes < need) return PMS_E_NOMEM;
        bt->arena = bt->ext_ws;
    } else {
        void* p = nullptr;
        bool fc = false;
        if (use_cache) p = cache_take(need, &fc);
        if (!p) {
            if (hipMalloc(&p, need) != hipSuccess) return PMS_E_NOMEM;
            bt->own_arena = true;
        }
        bt->cached_arena = fc;
        bt->arena = p;
    }
    resolve(bt);
    hipError_t e = hipSuccess;
    if (!bt->own_stream) e = make_stream(&bt->own_stream);
    if (e == hipSuccess && !bt->uploaded) e = hipEventCreateWithFlags(&bt->uploaded, hipEventDisableTiming);
    hipStream_t s = bt->own_stream;
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->b.inst, bt->dinst.data(), bt->dinst.size() * sizeof(InstDev),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !bt->chars.empty())
        e = hipMemcpyAsync(bt->b.chars, bt->chars.data(), bt->chars.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(bt->b.lut, bt->lut.data(), bt->lut.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && !bt->sort_cands.empty())
        e = hipMemcpyAsync(bt->b.sort_cand, bt->sort_cands.data(), bt->sort_cands.size(),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(bt->uploaded, s);
    return hip_status(e);
}

// The whole device pipeline on stream s, launched back to back.  With
// `timed`, events between the phases give per-phase device times.
int enqueue(pms_batch* bt, hipStream_t s, bool timed) {
    hipError_t e = hipSuccess;
    auto rec = [&](int i) {
        if (timed && e == hipSuccess) e = hipEventRecord(bt->ev[i], s);
    };
    rec(0);
    if (e == hipSuccess) e = launch_reset(bt->plan, bt->b, bt->item_cap, bt->part_cap, s);
    if (e == hipSuccess) e = launch_pack(bt->plan, bt->b, s);
    rec(1);
    if (e == hipSuccess) e = launch_compat(bt->plan, bt->b, s);
    rec(2);
    if (e == hipSuccess) e = launch_expand(bt->plan, bt->b, s);
    rec(3);
    if (e == hipSuccess) e = launch_search(bt->plan, bt->b, s);
    rec(4);
    if (e == hipSuccess) e = launch_sort(bt->plan, bt->b, s);
    rec(5);
    if (e != hipSuccess) {
        fprintf(stderr, "pms: launch failed: %s\n", hipGetErrorString(e));
        return PMS_E_DEVICE;
    }
    return PMS_OK;
}

int make_batch(const pms_instance* inst, int32_t count, const pms_tune* tune, pms_batch** out) {
    if (!out || count < 0 || (count > 0 && !inst)) return PMS_E_INVAL;
    if (count > kMaxInst) return PMS_E_UNSUPPORTED;
    if (tune) {
        if (tune->compat_kernel > 2) return PMS_E_INVAL;
        if (tune->split > 2047) return PMS_E_INVAL;
        if (tune->s1_begin < 0 || tune->s1_end < 0 ||
            (tune->s1_end > 0 && tune->s1_begin > tune->s1_end))
            return PMS_E_INVAL;
        if (tune->out_capacity < 0 || tune->out_capacity > (int64_t(1) << 30)) return PMS_E_INVAL;
        if (tune->stage_cap < 0 || tune->stage_cap > kStageCapMax) return PMS_E_INVAL;
        if (tune->compat_mode < 0 || tune->compat_mode > 2) return PMS_E_INVAL;
    }
    pms_batch* bt = new (std::nothrow) pms_batch();
    if (!bt) return PMS_E_NOMEM;
    if (tune) bt->tune = *tune;
    else (void)pms::tuned_for(inst, count, &bt->tune);  // the autotuner's choice for this shape
    bt->hin.resize(count);
    bt->out_cap.assign(count, kOutCapMin);
    bool wide = bt->tune.lmer_words == 2;
    bool letters5 = false;  // some alphabet has more than 4 letters
    for (int i = 0; i < count; i++) {
        int rc = validate(inst[i], bt->hin[i], bt->chars, bt->lut);
        if (rc) {
            delete bt;
            return rc;
        }
        HostInst& h = bt->hin[i];
        h.t = bt->tune.threshold > 0 ? std::max(2, std::min(kMaxT, (int)bt->tune.threshold))
                                     : pms_default_threshold(h.n, h.m, h.l, h.d, h.asize);
        h.triple = bt->tune.triple_filter < 0 ? 0 : 1;  // 0 = automatic = on
        const int r = h.m >= h.l ? h.m - h.l + 1 : 0;
        const bool all = bt->tune.s1_begin == 0 && bt->tune.s1_end == 0;
        h.s1_hi = all ? r : std::min(r, (int)bt->tune.s1_end);
        h.s1_lo = all ? 0 : std::min(h.s1_hi, (int)bt->tune.s1_begin);
        if (h.l > 32) wide = true;
        if (h.asize > 4) letters5 = true;
        const int64_t full = (int64_t)h.n * r * h.n * ((r + 63) / 64) * 8;
        h.c1only = bt->tune.compat_mode == 2 || (bt->tune.compat_mode == 0 && full > kCompatBudget);
        bt->out_cap[i] = bt->tune.out_capacity > 0 ? next_pow2(bt->tune.out_capacity)
                                                   : presized_out_cap(h.n, h.m, h.l, h.d, h.asize);
    }
    if (letters5 && wide) {  // l > 32 and a large alphabet in one batch: no l-mer class fits
        delete bt;
        return PMS_E_UNSUPPORTED;
    }
    if (!letters5 && bt->tune.lmer_words == 1 && wide) {
        delete bt;
        return PMS_E_UNSUPPORTED;
    }
    bt->words = letters5 ? 3 : wide ? 2 : 1;
    bt->kwords = bt->words == 1 ? 1 : 2;
    *out = bt;
    return PMS_OK;
}

void fill_result(const HostInst& h, const uint64_t* keys, int64_t cnt, int kw, pms_result* r) {
    const int B = h.abits, cpw = 64 / B;
    const uint64_t cmask = (1ull << B) - 1ull;
    r->count = cnt;
    r->l = h.l;
    r->words = (h.l + cpw - 1) / cpw;
    r->motifs = nullptr;
    r->packed = nullptr;
    if (cnt == 0) return;
    r->motifs = (char*)malloc((size_t)cnt * h.l);
    r->packed = (uint64_t*)malloc((size_t)cnt * r->words * 8);
    for (int64_t i = 0; i < cnt; i++) {
        const uint64_t* k = keys + i * kw;
        for (int p = 0; p < h.l; p++) {
            const int q = p / cpw;
            const int c = (int)((k[q] >> (64 - B * (p - q * cpw + 1))) & cmask);
            r->motifs[i * h.l + p] = h.alpha[c];
        }
        for (int q = 0; q < r->words; q++) r->packed[i * r->words + q] = k[q];
    }
}

int batch_create_impl(const pms_instance* inst, int32_t count, const pms_tune* tune, void* ws,
                      size_t ws_bytes, bool use_cache, const std::vector<int64_t>* caps,
                      pms_batch** out);

// Instances whose output overflowed their slots are solved again in a batch
// of their own, with slots for every motif they emitted; the others keep
// the first run's result.
int rerun_overflowed(pms_batch* bt, const std::vector<int>& idx,
                     const std::vector<InstCounters>& ctr, hipStream_t s, pms_result* outs) {
    std::vector<std::vector<std::string>> strs(idx.size());
    std::vector<std::vector<const char*>> ptrs(idx.size());
    std::vector<std::string> alphas(idx.size());
    std::vector<pms_instance> sub(idx.size());
    std::vector<int64_t> caps(idx.size());
    for (size_t k = 0; k < idx.size(); k++) {
        const int i = idx[k];
        const HostInst& h = bt->hin[i];
        const InstDev& d = bt->dinst[i];
        strs[k].resize(h.n);
        ptrs[k].resize(h.n);
        for (int j = 0; j < h.n; j++) {
            strs[k][j].assign((const char*)&bt->chars[(size_t)d.chars_off + (size_t)j * h.m],
                              (size_t)h.m);
            ptrs[k][j] = strs[k][j].c_str();
        }
        alphas[k] = h.alpha;
        sub[k] = pms_instance{ptrs[k].data(), h.n, h.m, alphas[k].c_str(), h.l, h.d};
        if (ctr[i].out_count > (1ull << 30)) return PMS_E_NOMEM;  // beyond the sort's index range
        caps[k] = next_pow2(std::max<int64_t>((int64_t)ctr[i].out_count, 1));
    }
    pms_tune t = bt->tune;  // same threshold, width and S_1 window range
    pms_batch* sb = nullptr;
    int rc = batch_create_impl(sub.data(), (int32_t)sub.size(), &t, nullptr, 0, false, &caps, &sb);
    if (rc) return rc;
    rc = pms_batch_run(sb, s, 0);
    std::vector<pms_result> r(idx.size());
    if (!rc) rc = pms_batch_results(sb, r.data());
    pms_batch_destroy(sb);
    if (rc) return rc;
    for (size_t k = 0; k < idx.size(); k++) outs[idx[k]] = r[k];
    return PMS_OK;
}

int batch_create_impl(const pms_instance* inst, int32_t count, const pms_tune* tune, void* ws,
                      size_t ws_bytes, bool use_cache, const std::vector<int64_t>* caps,
                      pms_batch** out) {
    pms_batch* bt = nullptr;
    int rc = make_batch(inst, count, tune, &bt);
    if (rc) return rc;
    if (caps)
        for (int i = 0; i < count; i++) bt->out_cap[i] = (*caps)[i];
    bt->ext_ws = ws;
    bt->ext_ws_bytes = ws_bytes;
    rc = materialise(bt, use_cache);
    if (rc == PMS_OK) {
        for (int i = 0; i < 6 && rc == PMS_OK; i++) rc = hip_status(hipEventCreate(&bt->ev[i]));
    }
    if (rc) {
        pms_batch_destroy(bt);
        return rc;
    }
    *out = bt;
    return PMS_OK;
}

}  // namespace

extern "C" {

const char* pms_version(void) { return "pms-mi355x 0.2 (gfx950)"; }

int pms_device_count(int32_t* count) {
    if (!count) return PMS_E_INVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess) n = 0;
    *count = n;
    return PMS_OK;
}

int pms_device_synchronize(void) { return hip_status(hipDeviceSynchronize()); }

const char* pms_strerror(int s) {
    switch (s) {
        case PMS_OK: return "ok";
        case PMS_E_INVAL: return "invalid argument";
        case PMS_E_ALPHABET: return "character outside the alphabet or repeated alphabet character";
        case PMS_E_UNSUPPORTED: return "outside the GPU path's limits";
        case PMS_E_NOMEM: return "out of memory or above the admission cap";
        case PMS_E_DEVICE: return "HIP runtime error";
        case PMS_E_AGAIN: return "not finished yet";
        case PMS_E_ABORTED: return "aborted";
        case PMS_E_TIMEOUT: return "timed out";
        default: return "unknown status";
    }
}

void pms_result_free(pms_result* r) {
    if (!r) return;
    free(r->motifs);
    free(r->packed);
    r->motifs = nullptr;
    r->packed = nullptr;
    r->count = 0;
}

int pms_batch_workspace_size(const pms_instance* inst, int32_t count, const pms_tune* tune,
                             size_t* bytes) {
    if (!bytes) return PMS_E_INVAL;
    pms_batch* bt = nullptr;
    int rc = make_batch(inst, count, tune, &bt);
    if (rc) return rc;
    *bytes = plan_layout(bt);
    rc = bt->plan_status;
    delete bt;
    return rc;
}

int pms_batch_create(const pms_instance* inst, int32_t count, const pms_tune* tune,
                     void* workspace, size_t workspace_bytes, pms_batch** out) {
    return batch_create_impl(inst, count, tune, workspace, workspace_bytes, false, nullptr, out);
}

int pms_batch_run(pms_batch* bt, void* hip_stream, int32_t use_graph) {
    if (!bt) return PMS_E_INVAL;
    if (bt->failed) return bt->failed;
    if (!bt->arena) return PMS_E_INVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    if (!s) s = bt->own_stream;
    // the uploads (own stream) precede every run, whichever stream it is on
    if (hipStreamWaitEvent(s, bt->uploaded, 0) != hipSuccess) return PMS_E_DEVICE;
    bt->last = s;
    bt->ran = true;
    if (!use_graph) {
        bt->timed = true;
        const int rc = enqueue(bt, s, true);
        if (rc) bt->failed = rc;
        return rc;
    }
    bt->timed = false;
    if (bt->gexec && bt->graph_stream != s) {
        (void)hipGraphExecDestroy(bt->gexec);
        bt->gexec = nullptr;
    }
    if (!bt->gexec) {
        hipGraph_t g = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return PMS_E_DEVICE;
        const int rc = enqueue(bt, s, false);
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return rc ? rc : PMS_E_DEVICE;
        }
        e = hipGraphInstantiate(&bt->gexec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            bt->gexec = nullptr;
            return PMS_E_DEVICE;
        }
        bt->graph_stream = s;
    }
    return hip_status(hipGraphLaunch(bt->gexec, s));
}

int pms_batch_timings(pms_batch* bt, float* ms5) {
    if (!bt || !ms5) return PMS_E_INVAL;
    if (!bt->timed) return PMS_E_AGAIN;
    if (hipEventSynchronize(bt->ev[5]) != hipSuccess) return PMS_E_DEVICE;
    for (int i = 0; i < 5; i++)
        if (hipEventElapsedTime(&ms5[i], bt->ev[i], bt->ev[i + 1]) != hipSuccess) return PMS_E_DEVICE;
    return PMS_OK;
}

int pms_batch_results(pms_batch* bt, pms_result* outs) {
    if (!bt || (!outs && !bt->hin.empty())) return PMS_E_INVAL;
    if (bt->failed) return bt->failed;
    if (!bt->arena || !bt->ran) return PMS_E_INVAL;
    hipStream_t s = bt->last;
    const int ni = (int)bt->hin.size();
    for (int i = 0; i < ni; i++) outs[i] = pms_result{};
    std::vector<InstCounters> ctr(ni);
    if (ni && hipMemcpyAsync(ctr.data(), bt->b.ctr, ni * sizeof(InstCounters),
                             hipMemcpyDeviceToHost, s) != hipSuccess)
        return PMS_E_DEVICE;
    if (hipStreamSynchronize(s) != hipSuccess) {
        bt->failed = PMS_E_DEVICE;
        return PMS_E_DEVICE;
    }
    std::vector<int> over;
    for (int i = 0; i < ni; i++) {
        if (ctr[i].flags & (kFlagItemOverflow | kFlagNodeOverflow)) return PMS_E_NOMEM;
        if ((ctr[i].flags & kFlagOutOverflow) || ctr[i].out_count > (unsigned long long)bt->out_cap[i])
            over.push_back(i);
    }
    bt->last_ctr = ctr;
    const int kw = bt->kwords;
    std::vector<std::vector<uint64_t>> keys(ni);
    for (int i = 0; i < ni; i++) {
        if (std::find(over.begin(), over.end(), i) != over.end()) continue;
        const int64_t u = (int64_t)ctr[i].uniq;
        keys[i].resize((size_t)u * kw);
        if (u > 0 && hipMemcpyAsync(keys[i].data(), bt->b.keys + bt->dinst[i].out_off * kw,
                                    (size_t)u * kw * 8, hipMemcpyDeviceToHost, s) != hipSuccess)
            return PMS_E_DEVICE;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return PMS_E_DEVICE;
    for (int i = 0; i < ni; i++)
        if (std::find(over.begin(), over.end(), i) == over.end())
            fill_result(bt->hin[i], keys[i].data(), (int64_t)ctr[i].uniq, kw, &outs[i]);
    if (!over.empty()) {
        // the run's other results stand; only these instances run again
        int rc = rerun_overflowed(bt, over, ctr, s, outs);
        if (rc) {
            for (int i = 0; i < ni; i++) pms_result_free(&outs[i]);
            return rc;
        }
    }
    return PMS_OK;
}

int pms_batch_work(pms_batch* bt, int32_t i, pms_work* w) {
    if (!bt || !w || i < 0 || i >= (int)bt->hin.size()) return PMS_E_INVAL;
    if (bt->last_ctr.size() != bt->hin.size()) return PMS_E_AGAIN;
    const InstCounters& c = bt->last_ctr[i];
    const InstDev& d = bt->dinst[i];
    const int64_t r = d.r;
    *w = pms_work{};
    // counted on the host: the compat matrix tests every unordered pair of
    // l-mers from different strings; the device reports work items and
    // emitted motifs (search-side work counters are not in this version)
    w->compat_pairs = (int64_t)d.n * (d.n - 1) / 2 * r * r;
    w->items = (int64_t)c.items;
    w->pushes = w->filter_words = w->triple_tests = w->tuples = -1;
    w->gen_evals = w->candidates = w->verify_tests = -1;
    w->motifs_emitted = (int64_t)c.out_count;
    w->done_ticks = (int64_t)c.done_at;
    return PMS_OK;
}

int pms_batch_destroy(pms_batch* bt) {
    if (!bt) return PMS_OK;
    if (bt->last) (void)hipStreamSynchronize(bt->last);
    if (bt->own_stream) (void)hipStreamSynchronize(bt->own_stream);
    release_arena(bt);
    for (int i = 0; i < 6; i++)
        if (bt->ev[i]) (void)hipEventDestroy(bt->ev[i]);
    if (bt->uploaded) (void)hipEventDestroy(bt->uploaded);
    if (bt->own_stream) (void)hipStreamDestroy(bt->own_stream);
    delete bt;
    return PMS_OK;
}

int pms_solve_batch(const pms_instance* inst, int32_t count, pms_result* outs,
                    const pms_tune* tune, void* hip_stream) {
    if (count < 0 || (count > 0 && (!inst || !outs))) return PMS_E_INVAL;
    for (int i = 0; i < count; i++) outs[i] = pms_result{};
    if (count == 0) return PMS_OK;
    pms_batch* bt = nullptr;
    int rc = batch_create_impl(inst, count, tune, nullptr, 0, true, nullptr, &bt);
    if (rc) return rc;
    rc = pms_batch_run(bt, hip_stream, 0);
    if (!rc) rc = pms_batch_results(bt, outs);
    pms_batch_destroy(bt);
    if (rc)
        for (int i = 0; i < count; i++) pms_result_free(&outs[i]);
    return rc;
}

int pms_solve(const char* const* seqs, int32_t n, int32_t m, const char* alphabet, int32_t l,
              int32_t d, pms_result* out) {
    if (!out) return PMS_E_INVAL;
    pms_instance in{seqs, n, m, alphabet, l, d};
    return pms_solve_batch(&in, 1, out, nullptr, nullptr);
}

}  // extern "C"
