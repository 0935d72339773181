// Allocation-free entry point: pms_solve_device_noalloc (include/pms.h).
//
// The same device pipeline as pms_solve_batch on one instance, with every
// intermediate buffer (instance descriptor, character table, packed l-mers,
// compat bit-matrix, work and part queues, emitted keys, counters) carved out of `scratch`, a fixed device array of this
// library that each GPU holds until the process ends.  Inputs and outputs
// are the caller's device buffers; the host side only validates sizes and
// enqueues kernels on the caller's stream (no hipMalloc, no hipFree, no
// memset or copy nodes, no host allocation), so it can run under hipGraph
// capture.  Calls that overlap on one GPU share its scratch and race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>

#include "../../include/pms.h"
#include "pms_internal.h"

namespace pms {

constexpr size_t kScratchBytes = size_t(256) << 20;  // PMS_NOALLOC_SCRATCH_BYTES
constexpr int kNoallocWavesPerCu = 20;                 // persistent search waves per CU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_mu;
void* g_ptr[kMaxDevices];  // scratch's device address, per device (set once)
int g_cus[kMaxDevices];

// hipGetSymbolAddress once per device, with that device current.
int scratch_of(int dev, void** ptr, int* cus) {
    if (dev < 0 || dev >= kMaxDevices) return PMS_E_UNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PMS_E_DEVICE;
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            c <= 0)
            return PMS_E_DEVICE;
        g_ptr[dev] = p;
        g_cus[dev] = c;
    }
    *ptr = g_ptr[dev];
    *cus = g_cus[dev];
    return PMS_OK;
}

inline size_t up256(size_t x) { return (x + 255) / 256 * 256; }

// Instance descriptor and character table, written from kernel arguments.
__global__ void k_noalloc_setup(InstDev* inst, InstDev v, uint8_t* lut, uint32_t alpha4) {
    const int i = threadIdx.x;
    if (i == 0) *inst = v;
    if (i < 256) {
        uint8_t code = 0xFF;
        for (int k = 0; k < 4; k++)
            if (((alpha4 >> (8 * k)) & 0xFFu) == (uint32_t)i) code = (uint8_t)k;
        lut[i] = code;
    }
}

// Copy the sorted, de-duplicated keys out and write the count, or a
// negative pms_status: PMS_E_ALPHABET for a character outside the
// alphabet, PMS_E_NOMEM when the motifs (or the internal queues) exceed
// their slots.
__global__ void k_noalloc_finish(const InstCounters* ctr, const uint64_t* keys, int words,
                                 uint64_t* out, int64_t out_cap, int64_t* count) {
    const InstCounters c = ctr[0];
    int64_t status = (int64_t)c.uniq;
    if (c.flags & kFlagBadChar) status = PMS_E_ALPHABET;
    else if (c.flags & (kFlagOutOverflow | kFlagItemOverflow | kFlagNodeOverflow)) status = PMS_E_NOMEM;
    else if ((int64_t)c.uniq > out_cap) status = PMS_E_NOMEM;
    if (blockIdx.x == 0 && threadIdx.x == 0) *count = status;
    if (status <= 0) return;
    const int64_t n = status * words;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = keys[i];
}

}  // namespace
}  // namespace pms

using namespace pms;

extern "C" size_t pms_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" int pms_solve_device_noalloc(const uint8_t* chars, int32_t n, int32_t m,
                                        const char* alphabet, int32_t l, int32_t d,
                                        uint64_t* keys_out, int64_t keys_cap, int64_t* count_out,
                                        void* hip_stream) {
    if (!alphabet || !count_out || n < 1 || m < 0 || l < 1 || d < 0 || d >= l || keys_cap < 0)
        return PMS_E_INVAL;
    if (m > 0 && !chars) return PMS_E_INVAL;
    if (keys_cap > 0 && !keys_out) return PMS_E_INVAL;
    // alphabet: exactly 4 distinct characters, codes by ascending byte value
    char a[4];
    size_t alen = 0;
    while (alphabet[alen] && alen < 5) alen++;
    if (alen != 4) return alen < 2 ? PMS_E_ALPHABET : PMS_E_UNSUPPORTED;
    memcpy(a, alphabet, 4);
    std::sort(a, a + 4, [](char x, char y) { return (uint8_t)x < (uint8_t)y; });
    for (int i = 1; i < 4; i++)
        if (a[i] == a[i - 1]) return PMS_E_ALPHABET;
    if (l > kMaxL || n > kMaxN || m - l + 1 > kMaxR) return PMS_E_UNSUPPORTED;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return PMS_E_DEVICE;
    void* base = nullptr;
    int cus = 0;
    int rc = scratch_of(dev, &base, &cus);
    if (rc) return rc;

    // plan (one instance) inside the scratch array
    const int words = l > 32 ? 2 : 1;
    const int r = m >= l ? m - l + 1 : 0;
    const int bw = (r + 63) / 64;
    const int64_t N = (int64_t)n * r;
    const int t = pms_default_threshold(n, m, l, d, 4);
    const unsigned long long items = std::max<unsigned long long>((unsigned long long)r * r, 1);
    const unsigned long long parts =
        std::max<unsigned long long>(std::min<unsigned long long>(items, 1ull << 22), 1024);
    const int blocks = cus * kNoallocWavesPerCu;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = up256(off + std::max<size_t>(bytes, 1));
        return o;
    };
    const size_t o_inst = take(sizeof(InstDev));
    const size_t o_lut = take(256);
    const size_t o_lmers = take((size_t)N * (words == 1 ? 8 : 16));
    // the whole compat matrix when it takes at most a quarter of the scratch,
    // else only the rows of S_1's l-mers (pushes test Hd <= 2d directly)
    const int c1only = (size_t)N * n * bw * 8 > kScratchBytes / 4 ? 1 : 0;
    const size_t o_compat = take((size_t)(c1only ? r : N) * n * bw * 8);
    const size_t o_items = take((size_t)items * 8);
    const size_t o_parts = take((size_t)parts * 8);
    const int tmax = std::max(2, t);
    const int deep_phases = tmax > 3 ? tmax - 3 : 0;
    const unsigned long long deep_cap = deep_phases > 0 ? (1ull << 16) : 1;
    const size_t o_deep0 = take((size_t)deep_cap * sizeof(DeepItem));
    const size_t o_deep1 = take((size_t)deep_cap * sizeof(DeepItem));
    const size_t o_ctr = take(sizeof(InstCounters));
    const size_t o_q = take(kQueues * sizeof(QueueCounters));
    if (off >= kScratchBytes) return PMS_E_NOMEM;
    // key slots: the rest of the scratch, a power of two (the sort's size)
    int64_t out_cap = 1;
    while ((size_t)(out_cap * 2) * 8 * words <= kScratchBytes - off) out_cap *= 2;
    if (out_cap < 64) return PMS_E_NOMEM;
    const size_t o_keys = off;

    char* s = (char*)base;
    DevBufs b{};
    b.inst = (InstDev*)(s + o_inst);
    b.chars = (uint8_t*)chars;
    b.lut = (uint8_t*)(s + o_lut);
    b.lmers = (void*)(s + o_lmers);
    b.compat = (uint64_t*)(s + o_compat);
    b.items = (uint64_t*)(s + o_items);
    b.parts = (uint64_t*)(s + o_parts);
    b.deep[0] = (DeepItem*)(s + o_deep0);
    b.deep[1] = (DeepItem*)(s + o_deep1);
    b.keys = (uint64_t*)(s + o_keys);
    b.ctr = (InstCounters*)(s + o_ctr);
    b.q = (QueueCounters*)(s + o_q);

    InstDev v{};
    v.n = n;
    v.m = m;
    v.l = l;
    v.d = d;
    v.r = r;
    v.bw = bw;
    v.t = t;
    v.triple = 1;
    v.s1_lo = 0;
    v.s1_hi = r;
    v.c1only = c1only;
    v.asize = 4;
    v.abits = 2;
    v.amask = 0xFu;
    v.chars_off = 0;
    v.lmer_off = 0;
    v.compat_off = 0;
    v.out_off = 0;
    v.out_cap = out_cap;

    LaunchPlan p{};
    p.n_inst = 1;
    p.max_n_lmers = (int)N;
    p.max_r = r;
    p.max_n = n;
    p.level_words = std::max(1, n * bw);
    p.tmax = tmax;
    p.deep_phases = deep_phases;
    p.deep_cap = deep_cap;
    p.words = words;
    p.kwords = words;
    p.search_blocks = blocks;
    p.compat_kernel = 1;
    p.split = kSplitDefault;
    p.s2cap = 1024;
    int lds_max = 0;
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return PMS_E_DEVICE;
    while (p.s2cap > kStageCapMin && search_lds_bytes(p) > (size_t)lds_max) p.s2cap /= 2;
    if (search_lds_bytes(p) > (size_t)lds_max) return PMS_E_UNSUPPORTED;

    uint32_t alpha4 = 0;
    for (int k = 0; k < 4; k++) alpha4 |= (uint32_t)(uint8_t)a[k] << (8 * k);
    hipStream_t st = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_noalloc_setup, dim3(1), dim3(256), 0, st, b.inst, v, b.lut, alpha4);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = launch_reset(p, b, items, parts, st);
    if (e == hipSuccess) e = launch_pack(p, b, st);
    if (e == hipSuccess) e = launch_compat(p, b, st);
    if (e == hipSuccess) e = launch_expand(p, b, st);
    if (e == hipSuccess) e = launch_search(p, b, st);
    if (e == hipSuccess) e = launch_sort(p, b, st);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_noalloc_finish, dim3(64), dim3(256), 0, st, b.ctr, b.keys, words,
                           keys_out, keys_cap, count_out);
        e = hipGetLastError();
    }
    return e == hipSuccess ? PMS_OK : PMS_E_DEVICE;
}
