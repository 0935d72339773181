// Internal layout shared by the host runtime and the gfx950 kernels.
#pragma once
#include <stdint.h>

#include <hip/hip_runtime_api.h>

struct pms_tune;      // include/pms.h
struct pms_instance;

namespace pms {

// Limits of the device path.
constexpr int kMaxN = 32;        // strings per instance (row bit masks are 32-bit)
constexpr int kMaxR = 8192;      // windows per string (13-bit window index)
constexpr int kMaxL = 64;        // motif length (two 64-bit bit-planes; alphabets of up to 4 letters)
constexpr int kMaxLWide = 32;    // motif length over larger alphabets (five 32-bit planes)
constexpr int kMaxAlpha = 32;    // letters (5-bit codes)
constexpr int kMaxT = 8;         // stack size at which generation starts
constexpr int kSplitDefault = 32;  // third stack members one work item keeps (rest: part items)
constexpr int kStageCapMin = 256;   // staged survivors of one tail batch (LDS entries; also
                                    // the push filter's listing scratch)
constexpr int kStageCapMax = 4096;
constexpr int kMaxInst = (1 << 20) - 1;  // instances per batch (20-bit field of a work item)

// Work item (64 bits): inst << 44 | lo << 31 | u1 << 18 | p2 << 13 | x2.
// u1: window of string 0 (level 1); p2, x2: string and window of the second
// stack member (p2 == 0 marks n == 1); lo: first rank, among the survivors
// of the string chosen at stack size 2, that the item covers (0 for the
// items the expansion writes; part items cover `split` ranks from lo).
constexpr uint64_t make_item(uint64_t inst, uint64_t lo, uint64_t u1, uint64_t p2, uint64_t x2) {
    return (inst << 44) | (lo << 31) | (u1 << 18) | (p2 << 13) | x2;
}
constexpr int item_inst(uint64_t it) { return (int)(it >> 44); }
constexpr int item_lo(uint64_t it) { return (int)((it >> 31) & 0x1FFF); }
constexpr int item_u1(uint64_t it) { return (int)((it >> 18) & 0x1FFF); }
constexpr int item_p2(uint64_t it) { return (int)((it >> 13) & 31); }
constexpr int item_x2(uint64_t it) { return (int)(it & 0x1FFF); }
constexpr uint64_t kNoItem = ~0ull;  // part slot that was reserved but not written

// One instance as the kernels see it.
struct InstDev {
    int32_t n, m, l, d;
    int32_t r;        // windows per string, m - l + 1 (0 if m < l)
    int32_t bw;       // 64-bit words per row bitset, ceil(r / 64)
    int32_t t;        // stack size at which neighbourhood generation starts
    int32_t triple;   // Theorem 1 survivor filter on/off
    int32_t s1_lo, s1_hi;  // S_1 windows searched: [s1_lo, s1_hi)
    int32_t c1only;   // compat rows only for the l-mers of S_1; pushes test Hd <= 2d directly
    int32_t asize;    // letters of the alphabet (codes 0 .. asize-1)
    int32_t abits;    // key bits per character (2 up to 4 letters, else ceil(log2 asize))
    uint32_t amask;   // (1 << asize) - 1: every child of a generator node
    int32_t pad;
    int64_t chars_off;   // byte offset of the n*m characters
    int64_t lmer_off;    // l-mer offset (units of one packed l-mer)
    int64_t compat_off;  // u64 offset of the compat bit-matrix [N][n][bw] (c1only: [r][n][bw])
    int64_t out_off;     // key offset (units of one key)
    int64_t out_cap;     // key slots (power of two)
};

// Per-instance device counters.
struct InstCounters {
    unsigned long long out_count;    // motifs emitted (with repeats)
    unsigned long long uniq;         // distinct motifs after sort/unique
    unsigned int flags;              // kFlag* bits
    unsigned int pad;
    unsigned long long items;        // level-2 work items produced
    unsigned long long outstanding;  // items, parts and deep items not finished yet
    unsigned long long done_at;      // 100 MHz device clock when outstanding reached 0
};

// Deep item: a stack prefix of k members (string and window of each) and a
// rank range [ra, rb) of the survivors of string p at level k, searched by
// whichever wave takes it (it rebuilds the levels by pushing the prefix
// again).  Waves split an oversized string this way at any stack size >= 3.
struct DeepItem {
    uint32_t inst;
    uint8_t k, p, pad0, pad1;
    uint16_t ra, rb;
    uint16_t win[kMaxT];
    uint8_t row[kMaxT];
    uint32_t pad2;
};
constexpr int kQueues = 4;  // q[0] items, q[1] parts, q[2], q[3] deep items (alternating phases)

constexpr unsigned kFlagOutOverflow = 1u;
constexpr unsigned kFlagItemOverflow = 2u;
constexpr unsigned kFlagNodeOverflow = 4u;  // a search loop reached its step guard
constexpr unsigned kFlagBadChar = 8u;  // a window holds a character outside the alphabet

// Global queue counters.
struct QueueCounters {
    unsigned long long item_count;  // items appended
    unsigned long long item_next;   // next item to take
    unsigned long long item_cap;
    unsigned long long pad;
};

struct LaunchPlan {
    int n_inst;
    int max_n_lmers;     // max over instances of n*r
    int max_r;
    int max_n;
    int level_words;     // max over instances of n*bw (u64 words per search level)
    int tmax;            // max threshold in the batch (template selector)
    int words;           // l-mer class: 1, 2 (two 32- / 64-bit planes), 3 (five 32-bit planes)
    int kwords;          // u64 words per motif key (1 or 2)
    int search_blocks;   // persistent grid size
    int compat_kernel;   // 1 VALU xor/popcount, 2 int8 one-hot MFMA
    int split;           // survivors of one string a wave keeps (the rest: split items)
    int s2cap;           // staged survivors per tail batch (multiple of 64)
    int deep_phases;     // search launches for deep items (tmax - 3, at least 0)
    unsigned long long deep_cap;  // deep items per queue
    int sort_cands;      // instances whose key area exceeds one LDS sort chunk (multi-block sort)
    long long sort_pmax; // the largest key area among them (a power of two)
};

// Device buffers of one planned batch.
struct DevBufs {
    InstDev* inst;
    uint8_t* chars;
    uint8_t* lut;
    void* lmers;
    uint64_t* compat;
    uint64_t* items;
    uint64_t* parts;     // part items (second search launch)
    uint64_t* keys;
    InstCounters* ctr;
    QueueCounters* q;    // kQueues counter sets
    DeepItem* deep[2];   // deep-item queues
    void* sort_cand;     // multi-block sort: candidate list, compaction scratch, chunk records
    uint64_t* sort_tmp;
    uint64_t* sort_side;
};

// Kernel launchers (pms_kernels.hip).  All enqueue on `stream`.
hipError_t launch_reset(const LaunchPlan& p, const DevBufs& b, unsigned long long item_cap,
                        unsigned long long part_cap, hipStream_t stream);
hipError_t launch_pack(const LaunchPlan& p, const DevBufs& b, hipStream_t stream);
hipError_t launch_compat(const LaunchPlan& p, const DevBufs& b, hipStream_t stream);
hipError_t launch_expand(const LaunchPlan& p, const DevBufs& b, hipStream_t stream);
hipError_t launch_search(const LaunchPlan& p, const DevBufs& b, hipStream_t stream);
hipError_t launch_sort(const LaunchPlan& p, const DevBufs& b, hipStream_t stream);
size_t search_lds_bytes(const LaunchPlan& p);
// Multi-block sort candidate records (pms_kernels.hip).
size_t sort_cand_bytes();
void sort_cand_fill(void* dst, int i, int inst, long long tmp_off, long long side_off);
constexpr int sort_chunk_keys(int kwords) { return 4096 / kwords; }
size_t lmer_bytes(int words);

// Memory plan bounds (pms_runtime.cpp): a batch needs at most
// fixed_bytes(tune) + the sum of inst_bytes(...) over its instances.
size_t inst_bytes(int n, int m, int l, int d, int sigma, const ::pms_tune* tune);
size_t fixed_bytes(const ::pms_tune* tune);

// The autotuner's cached setting for a batch of this shape (pms_tune.cpp).
bool tuned_for(const ::pms_instance* inst, int count, ::pms_tune* out);

}  // namespace pms
