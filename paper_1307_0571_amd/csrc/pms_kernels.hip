// gfx950 kernels for exact (l,d) planted motif search (PMS8).
//
// Data layout (per instance, all in HBM):
//   chars   n*m bytes, row-major (string i at i*m)
//   lmers   N = n*r packed l-mers, id g = row*r + window.  Planar packing
//           (Section 2.1 stores l * ceil(log2 |alphabet|) bits per l-mer):
//           bit p of plane b is bit b of the code of character p, so
//           Hd(u,v) = popcount of the OR over the planes of u XOR v.
//           W = 1: two 32-bit planes (alphabets of up to 4 letters, l <= 32);
//           W = 2: two 64-bit planes (up to 4 letters, l <= 64); W = 3: five
//           32-bit planes (up to 32 letters, such as the 20 amino acids,
//           l <= 32).
//   compat  [N][n][bw] u64 bitsets: bit x of word (u, j, x/64) is set iff
//           Hd(u, window x of string j) <= 2d and u is not in string j
//           (the pair condition of Section 2.4, precomputed as Section 2.1
//           describes).
//   keys    motif keys, B bits per character (B = 2 up to 4 letters, else
//           ceil(log2 |alphabet|)), floor(64 / B) characters per word, first
//           character in the most significant bits; KW words per key (1 for
//           W = 1, else 2).
//
// Pipeline: pack -> compat -> expand (level 1, one wave per S_1 window;
// pushes level-2 work items to a device queue) -> search (persistent waves
// pop items and run the rest of Algorithm 2 depth-first with per-level row
// bitsets in LDS, the Theorem 1 survivor filter, Algorithm 1's pruned tree
// and the candidate check) -> sort/unique.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "pms_internal.h"

namespace pms {

template <int W> struct Lm;
template <> struct Lm<1> { uint32_t h, lo; };
template <> struct Lm<2> { uint64_t h, lo; };
// larger alphabets: plane lo holds bit 0 of every character's code, h bit 1,
// x2 .. x4 bits 2 .. 4
template <> struct Lm<3> { uint32_t h, lo, x2, x3, x4; };
template <int W> struct MaskOf { typedef uint64_t type; };
template <> struct MaskOf<1> { typedef uint32_t type; };
template <> struct MaskOf<3> { typedef uint32_t type; };
template <int W> struct KeyWords { static constexpr int value = W == 1 ? 1 : 2; };

__device__ __forceinline__ uint32_t dmask(const Lm<1>& a, const Lm<1>& b) {
    return (a.h ^ b.h) | (a.lo ^ b.lo);
}
__device__ __forceinline__ uint64_t dmask(const Lm<2>& a, const Lm<2>& b) {
    return (a.h ^ b.h) | (a.lo ^ b.lo);
}
__device__ __forceinline__ uint32_t dmask(const Lm<3>& a, const Lm<3>& b) {
    return (a.h ^ b.h) | (a.lo ^ b.lo) | (a.x2 ^ b.x2) | (a.x3 ^ b.x3) | (a.x4 ^ b.x4);
}
template <int W> __device__ __forceinline__ Lm<W> lm_zero() {
    Lm<W> v{};
    return v;
}
// code of character p
__device__ __forceinline__ uint32_t code_at(const Lm<1>& v, int p) {
    return ((v.h >> p) & 1u) << 1 | ((v.lo >> p) & 1u);
}
__device__ __forceinline__ uint32_t code_at(const Lm<2>& v, int p) {
    return (uint32_t)(((v.h >> p) & 1ull) << 1 | ((v.lo >> p) & 1ull));
}
__device__ __forceinline__ uint32_t code_at(const Lm<3>& v, int p) {
    return ((v.x4 >> p) & 1u) << 4 | ((v.x3 >> p) & 1u) << 3 | ((v.x2 >> p) & 1u) << 2 |
           ((v.h >> p) & 1u) << 1 | ((v.lo >> p) & 1u);
}
__device__ __forceinline__ int pc(uint32_t x) { return __popc(x); }
__device__ __forceinline__ int pc(uint64_t x) { return __popcll(x); }
// bits at positions >= s (s <= 64)
__device__ __forceinline__ uint32_t suf(uint32_t x, int s) { return s >= 32 ? 0u : x >> s; }
__device__ __forceinline__ uint64_t suf(uint64_t x, int s) { return s >= 64 ? 0ull : x >> s; }

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63); }
__device__ __forceinline__ unsigned long long ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int rank_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    return (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x) |
           (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32)) << 32;
}

__device__ __forceinline__ int wave_incl_scan(int x) {
    int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}
__device__ __forceinline__ int wave_min(int x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = min(x, __shfl_xor(x, o, 64));
    return x;
}

// --------------------------------------------------------------- reset

__global__ void k_reset(InstCounters* ctr, int n_inst, QueueCounters* q, unsigned long long item_cap,
                        unsigned long long part_cap, unsigned long long deep_cap) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_inst) {
        ctr[i].out_count = 0;
        ctr[i].uniq = 0;
        ctr[i].flags = 0;
        ctr[i].pad = 0;
        ctr[i].items = 0;
        ctr[i].outstanding = 0;
        ctr[i].done_at = 0;
    }
    if (i < kQueues) {
        q[i].item_count = 0;
        q[i].item_next = 0;
        q[i].item_cap = i == 0 ? item_cap : i == 1 ? part_cap : deep_cap;
        q[i].pad = 0;
    }
}

// Empty deep queue i before a phase appends to it again.
__global__ void k_reset_queue(QueueCounters* q, int i) {
    if (threadIdx.x == 0) {
        q[i].item_count = 0;
        q[i].item_next = 0;
    }
}

// Part slots start as kNoItem: a slot reserved by a search wave that then
// found the part queue full is skipped by the second search launch.
__global__ void k_fill_parts(uint64_t* parts, unsigned long long n) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += stride)
        parts[i] = kNoItem;
}

// ---------------------------------------------------------------- pack (a1)

// A character outside the alphabet (table entry 0xFF) sets kFlagBadChar;
// the host path has rejected those already, device-resident inputs have not.
template <int W>
__global__ __launch_bounds__(256) void k_pack(const InstDev* __restrict__ insts,
                                              const uint8_t* __restrict__ chars,
                                              const uint8_t* __restrict__ lut,
                                              Lm<W>* __restrict__ lmers,
                                              InstCounters* __restrict__ ctr) {
    typedef typename MaskOf<W>::type M;
    const InstDev I = insts[blockIdx.y];
    const int N = I.n * I.r;
    const int g = blockIdx.x * 256 + threadIdx.x;
    if (g >= N) return;
    const int row = g / I.r, w = g - row * I.r;
    const uint8_t* p = chars + I.chars_off + (int64_t)row * I.m + w;
    const uint8_t* tab = lut + (int64_t)blockIdx.y * 256;
    M h = 0, lo = 0, x2 = 0, x3 = 0, x4 = 0;
    bool bad = false;
    for (int i = 0; i < I.l; i++) {
        uint32_t c = tab[p[i]];
        bad |= c == 0xFFu;
        h |= (M)((c >> 1) & 1u) << i;
        lo |= (M)(c & 1u) << i;
        if constexpr (W == 3) {
            x2 |= (M)((c >> 2) & 1u) << i;
            x3 |= (M)((c >> 3) & 1u) << i;
            x4 |= (M)((c >> 4) & 1u) << i;
        }
    }
    if (bad) atomicOr(&ctr[blockIdx.y].flags, kFlagBadChar);
    Lm<W> v = lm_zero<W>();
    v.h = h;
    v.lo = lo;
    if constexpr (W == 3) {
        v.x2 = x2;
        v.x3 = x3;
        v.x4 = x4;
    }
    lmers[I.lmer_off + g] = v;
}

// ------------------------------------------------- compat bit-matrix (a2)
// One wave per (tile of 8 l-mers u, string j); lane x of word w tests window
// 64w+x of string j against the 8 u's; each test's wave ballot is one word.

constexpr int kCompatTile = 8;

template <int W>
__global__ __launch_bounds__(256) void k_compat(const InstDev* __restrict__ insts,
                                                const Lm<W>* __restrict__ lmers,
                                                uint64_t* __restrict__ compat) {
    const InstDev I = insts[blockIdx.y];
    const int N = I.n * I.r;
    if (N <= 0) return;
    const int Nu = I.c1only ? I.r : N;  // rows computed: every l-mer, or those of S_1
    const int ntile = (Nu + kCompatTile - 1) / kCompatTile;
    const int task = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (task >= ntile * I.n) return;
    const int lane = lane_id();
    const int tile = task / I.n, j = task - tile * I.n;
    const int u0 = tile * kCompatTile;
    const Lm<W>* L = lmers + I.lmer_off;
    Lm<W> u[kCompatTile];
    int urow[kCompatTile];
#pragma unroll
    for (int k = 0; k < kCompatTile; k++) {
        int g = u0 + k;
        if (g < Nu) {
            u[k] = L[g];
            urow[k] = g / I.r;
        } else {
            u[k] = lm_zero<W>();
            urow[k] = -1;
        }
    }
    const int thr = 2 * I.d;
    uint64_t* out = compat + I.compat_off;
    for (int w = 0; w < I.bw; w++) {
        const int x = w * 64 + lane;
        const bool valid = x < I.r;
        const Lm<W> v = valid ? L[j * I.r + x] : lm_zero<W>();
#pragma unroll
        for (int k = 0; k < kCompatTile; k++) {
            if (urow[k] < 0) continue;
            bool pred = valid && urow[k] != j && pc(dmask(u[k], v)) <= thr;
            unsigned long long b = ballot(pred);
            if (lane == 0) out[((int64_t)(u0 + k) * I.n + j) * I.bw + w] = b;
        }
    }
}

// Int8 MFMA builder of the same matrix.  Hd(u, v) <= 2d is matches(u, v) >=
// l - 2d, and matches(u, v) is the dot product of the one-hot codes of u and
// v (an l x A vector of 0/1 bytes, A = 4 letters, or the alphabet's size in
// the five-plane class).  One wave takes 32 rows u and walks every string j
// and 64-window word w: two 32x32 tiles of v_mfma_i32_32x32x16_i8 over the
// one-hot K dimension give the 32 x 64 match counts, a ballot per
// accumulator register turns them into row bits, and each of the first 32
// lanes writes one row's 64-bit word.
typedef int v16i __attribute__((ext_vector_type(16)));

// Bytes k0 .. k0+7 of l-mer x's one-hot code vector (byte k = [code of
// character k / AL equals k % AL]; 0 beyond the l-mer).
template <int W>
__device__ __forceinline__ long onehot8(const Lm<W>& x, int k0, int AL, int l) {
    uint64_t o = 0;
    if (AL == 4) {
        const int p0 = k0 >> 2;  // k0 is a multiple of 8: characters p0, p0 + 1
        if (p0 < l) o |= 1ull << (8 * code_at(x, p0));
        if (p0 + 1 < l) o |= 1ull << (32 + 8 * code_at(x, p0 + 1));
    } else {
        int p = k0 / AL, c = k0 - p * AL;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            if (p < l && (int)code_at(x, p) == c) o |= 1ull << (8 * i);
            if (++c == AL) {
                c = 0;
                p++;
            }
        }
    }
    return (long)o;
}

template <int W>
__global__ __launch_bounds__(64) void k_compat_mfma(const InstDev* __restrict__ insts,
                                                    const Lm<W>* __restrict__ lmers,
                                                    uint64_t* __restrict__ compat) {
    const InstDev I = insts[blockIdx.y];
    const int N = I.n * I.r;
    const int Nu = I.c1only ? I.r : N;
    const int u0 = blockIdx.x * 32;
    if (N <= 0 || u0 >= Nu) return;
    const int lane = lane_id();
    const int AL = W == 3 ? I.asize : 4;
    const int K = AL * I.l;
    const int steps = (K + 15) / 16;
    const int kb = (lane >> 5) * 8;
    const Lm<W>* L = lmers + I.lmer_off;
    const int ua = u0 + (lane & 31);  // this lane's row for the A operand
    const Lm<W> ux = ua < Nu ? L[ua] : lm_zero<W>();
    const int thr = I.l - 2 * I.d;
    // the row whose word this lane writes (lanes 0..31): accumulator
    // register r = (R / 8) * 4 + R % 4 holds it, in the ballot's low half
    // when (R / 4) is even
    const int R = lane & 31;
    const int myr = (R >> 3) * 4 + (R & 3);
    const bool hi_half = (R >> 2) & 1;
    const int urow = u0 + R;
    const int ustr = urow < Nu ? urow / I.r : -1;
    uint64_t* out = compat + I.compat_off;
    for (int j = 0; j < I.n; j++) {
        for (int w = 0; w < I.bw; w++) {
            const int x0 = w * 64 + (lane & 31), x1 = x0 + 32;
            const Lm<W> v0 = x0 < I.r ? L[j * I.r + x0] : lm_zero<W>();
            const Lm<W> v1 = x1 < I.r ? L[j * I.r + x1] : lm_zero<W>();
            v16i c0 = {0}, c1 = {0};
            for (int st = 0; st < steps; st++) {
                const int k0 = st * 16 + kb;
                const long a = onehot8<W>(ux, k0, AL, I.l);
                const long b0 = x0 < I.r ? onehot8<W>(v0, k0, AL, I.l) : 0l;
                const long b1 = x1 < I.r ? onehot8<W>(v1, k0, AL, I.l) : 0l;
                c0 = __builtin_amdgcn_mfma_i32_32x32x16_i8(a, b0, c0, 0, 0, 0);
                c1 = __builtin_amdgcn_mfma_i32_32x32x16_i8(a, b1, c1, 0, 0, 0);
            }
            uint64_t word = 0;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const uint64_t m0 = ballot(c0[r] >= thr);
                const uint64_t m1 = ballot(c1[r] >= thr);
                if (r == myr)
                    word = hi_half ? ((m0 >> 32) | (m1 & 0xFFFFFFFF00000000ull))
                                   : ((m0 & 0xFFFFFFFFull) | (m1 << 32));
            }
            if (lane < 32 && urow < Nu) {
                // no bits for the row's own string nor beyond the last window
                const int left = I.r - w * 64;
                const uint64_t valid = left >= 64 ? ~0ull : (left > 0 ? (1ull << left) - 1ull : 0ull);
                out[((int64_t)urow * I.n + j) * I.bw + w] = (j == ustr) ? 0ull : (word & valid);
            }
        }
    }
}

// ----------------------------------------------------- level-1 expansion
// One wave per (instance, window u1 of S_1): the level-1 survivors of string j
// are exactly the compat row C[u1][j] (Algorithm 2's first push and filter).
// Picks the smallest remaining string (ties: lowest index; Section 2.1) and
// appends one work item per survivor u2 of that string.
// Items as pms_internal.h lays them out, with lo = 0; p2 = 0 (string 0 is
// never a search row) marks n == 1, where the stack {u1} is already complete.

__global__ __launch_bounds__(256) void k_expand(const InstDev* __restrict__ insts,
                                                const uint64_t* __restrict__ compat,
                                                uint64_t* __restrict__ items,
                                                QueueCounters* __restrict__ q,
                                                InstCounters* __restrict__ ctr) {
    const int inst = blockIdx.y;
    const InstDev I = insts[inst];
    const int u1 = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
    if (u1 >= I.r || u1 < I.s1_lo || u1 >= I.s1_hi) return;
    const int lane = lane_id();
    const int n = I.n, bw = I.bw;
    if (n == 1) {
        if (lane == 0) {
            unsigned long long at = atomicAdd(&q->item_count, 1ull);
            if (at < q->item_cap)
                items[at] = make_item((uint64_t)inst, 0, (uint64_t)u1, 0, 0);
            else
                atomicOr(&ctr[inst].flags, kFlagItemOverflow);
            atomicAdd(&ctr[inst].items, 1ull);
            atomicAdd(&ctr[inst].outstanding, 1ull);
        }
        return;
    }
    const uint64_t* C = compat + I.compat_off + (int64_t)u1 * n * bw;
    // per-row popcounts: lanes over (row, word), rows 1..n-1
    int best = 0x7FFFFFFF;  // (count << 5) | row
    bool dead = false;
    for (int j = 1; j < n; j++) {
        int c = 0;
        for (int w = lane; w < bw; w += 64) c += pc(C[j * bw + w]);
        for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
        dead |= (c == 0);
        best = min(best, (c << 5) | j);
    }
    if (dead) return;
    const int p2 = best & 31;
    // items: one per set bit of C[u1][p2], compacted with ballot + prefix sum
    int total = best >> 5;
    unsigned long long base = 0;
    if (lane == 0) {
        base = atomicAdd(&q->item_count, (unsigned long long)total);
        atomicAdd(&ctr[inst].items, (unsigned long long)total);
        atomicAdd(&ctr[inst].outstanding, (unsigned long long)total);
    }
    base = __shfl(base, 0, 64);
    if (base + (unsigned long long)total > q->item_cap) {
        if (lane == 0) atomicOr(&ctr[inst].flags, kFlagItemOverflow);
        return;
    }
    int done = 0;
    for (int w0 = 0; w0 < bw; w0 += 64) {
        const int w = w0 + lane;
        uint64_t bits = (w < bw) ? C[p2 * bw + w] : 0ull;
        const int c = pc(bits);
        const int incl = wave_incl_scan(c);
        int o = done + incl - c;
        while (bits) {
            const int b = __builtin_ctzll(bits);
            bits &= bits - 1;
            const uint64_t x2 = (uint64_t)(w * 64 + b);
            items[base + o++] = make_item((uint64_t)inst, 0, (uint64_t)u1, (uint64_t)p2, x2);
        }
        done += uni(__shfl(incl, 63, 64));
    }
}

// --------------------------------------------------------------- search
//
// One persistent wave per work item runs Algorithm 2 depth-first from the
// item's stack {u1, u2}: per-level row bitsets in LDS, the pair bit and the
// Theorem 1 filter on every push, the smallest remaining string next.
//
// The last level is a "tail batch".  When the stack holds t-1 members and
// the next member comes from string p, every candidate of p (up to
// kTailSlots at a time) becomes a slot:
//   * the survivors of the other remaining strings are staged once in LDS
//     (one segment per string, fewest survivors first);
//   * the pruned trees of Algorithm 1 of all live slots are split into
//     subtrees at depth 2 or 3 and handed to lanes; each lane walks its
//     subtree depth-first on its own (no shared stack): a node's 4-bit mask
//     of valid children comes from the budgets of the prefix and the pair /
//     triple slacks of the suffix (the prune of Algorithm 1 with Theorem 1),
//     and the unvisited children of every depth on the path are kept as
//     nibbles in registers;
//   * complete l-mers go to an LDS buffer and are checked against the
//     survivors of every remaining string (Algorithm 2's isMotif on the
//     filtered rows), transposed: the lanes hold 64 survivors of a string,
//     and each buffered l-mer is tested against all of them in one wave
//     instruction.  The candidate's own push filter is not applied to the
//     survivors first: a survivor within d of a generated l-mer passes it
//     anyway (triangle inequality, and Theorem 1 for the common neighbour),
//     so the check finds the same hits without it.
// When the staged survivors do not fit the LDS area, the check loads each
// string's survivors (from the level bitsets) 64 at a time instead.  A
// complete stack (t reached at a push, no string left, or a single string)
// is a tail batch of one slot.

constexpr int kTailSlots = 16;  // candidates of one tail batch (<= 32: one bit each)
constexpr int kLeafCap = 256;   // generated l-mers awaiting the check
constexpr long long kStepLimit = 1ll << 32;  // guard on every loop of the tail batch

template <int W, int TMAX>
struct SearchLds {
    uint32_t rows[TMAX + 1];         // strings not on the stack at each level
    int prow[TMAX + 1];              // string whose survivors are pushed next
    int cursor[TMAX + 1];            // next window to try in that string
    Lm<W> st[TMAX];                  // the stack
    typename MaskOf<W>::type E[TMAX][TMAX];  // e(s_a, s_b) differing-position masks
    int HD[TMAX][TMAX];              // Hd(s_a, s_b)
    uint16_t segoff[kMaxN + 1];      // staged segment g: [segoff[g], segoff[g+1])
    uint8_t segrow[kMaxN];           // string of segment g
    int nseg;
    int item;
    int xs[kTailSlots];              // window of each slot's candidate
    int sv[256];                     // windows of the survivors a transposed check holds
    int lix[64];                     // l-mers a grouped check round takes, by group
    int aslot[kTailSlots];           // live slots, in order
    Lm<W> dq_v[64];                  // donated subtrees: prefix,
    uint8_t dq_d[64], dq_s[64];      // depth and slot
};

template <int W>
__device__ __forceinline__ uint64_t key_word(uint64_t h, uint64_t lo, int from, int to) {
    // characters from..to-1 (to - from <= 32), first one in bits 63..62
    uint64_t k = 0;
    for (int p = from; p < to; p++) {
        uint64_t c = (((h >> p) & 1ull) << 1) | ((lo >> p) & 1ull);
        k |= c << (62 - 2 * (p - from));
    }
    return k;
}

// bits at positions < s (s <= 64)
__device__ __forceinline__ uint32_t low_bits(uint32_t, int s) { return s >= 32 ? ~0u : ((1u << s) - 1u); }
__device__ __forceinline__ uint64_t low_bits(uint64_t, int s) { return s >= 64 ? ~0ull : ((1ull << s) - 1ull); }

// Prefix v with character ch at position q (positions after q cleared).
template <int W>
__device__ __forceinline__ Lm<W> with_char(const Lm<W>& v, int q, uint32_t ch) {
    typedef typename MaskOf<W>::type M;
    const M keep = low_bits((M)0, q);
    Lm<W> o = lm_zero<W>();
    o.h = (M)((v.h & keep) | ((M)((ch >> 1) & 1u) << q));
    o.lo = (M)((v.lo & keep) | ((M)(ch & 1u) << q));
    if constexpr (W == 3) {
        o.x2 = (v.x2 & keep) | (((ch >> 2) & 1u) << q);
        o.x3 = (v.x3 & keep) | (((ch >> 3) & 1u) << q);
        o.x4 = (v.x4 & keep) | (((ch >> 4) & 1u) << q);
    }
    return o;
}

// Child mask (bit c: character code c; `full` = every letter of the
// alphabet) from a pair's or triple's slack: child c is kept when
// slack >= (members) - (members whose character at the position is c).
__device__ __forceinline__ uint32_t slack2(int s, uint32_t oa, uint32_t ob, uint32_t full) {
    return s >= 2 ? full : s == 1 ? (oa | ob) : s == 0 ? (oa & ob) : 0u;
}
__device__ __forceinline__ uint32_t slack3(int s, uint32_t oa, uint32_t ob, uint32_t oc, uint32_t full) {
    return s >= 3 ? full
         : s == 2 ? (oa | ob | oc)
         : s == 1 ? ((oa & ob) | (oa & oc) | (ob & oc))
         : s == 0 ? (oa & ob & oc) : 0u;
}

template <int W, int TMAX>
struct Searcher {
    typedef typename MaskOf<W>::type M;
    // u64 words of child nibbles (16 depths each; alphabets of up to 4
    // letters); larger alphabets keep one 32-bit child mask per depth in LDS
    static constexpr int NW = W == 1 ? 2 : W == 2 ? 4 : 1;
    SearchLds<W, TMAX>& S;
    uint64_t* lv;  // LDS level bitsets: level k at lv + (k - 2) * level_words
    int level_words;
    const InstDev& I;
    int inst;
    const Lm<W>* L;       // this instance's l-mers
    const uint64_t* C;    // this instance's compat matrix
    uint64_t u1g;         // global id of the level-1 l-mer (string 0)
    uint64_t* keys;
    InstCounters* ctr;
    int lane;
    unsigned* cntw;
    uint32_t inv_bw;      // ceil(2^32 / bw) (bw >= 2)
    Lm<W>* s2;            // staged survivors (and the filter's listing scratch)
    Lm<W>* ut;            // [kTailSlots] candidate of each slot
    Lm<W>* leaf;          // [kLeafCap] generated l-mers
    int s2cap;            // staging area (entries of sizeof(Lm<W>))
    bool half;            // W == 1 and l <= 16: staged l-mers packed in 4 bytes
    int scap;             // staged l-mers that fit
    uint32_t* cm;         // W == 3: [32 depths][64 lanes] child masks

    __device__ __forceinline__ uint64_t* level(int k) { return lv + (k - 2) * level_words; }
    __device__ __forceinline__ unsigned& cnt_word(int k, int j) { return cntw[k * kMaxN + j]; }
    __device__ __forceinline__ unsigned cnt16(int k, int j) { return cntw[k * kMaxN + j]; }

    // string index of flattened row word i (i < n * bw <= 4096): an exact
    // reciprocal multiply instead of a division (i * bw < 2^32)
    __device__ __forceinline__ int row_of(int i) const {
        return I.bw == 1 ? i : (int)__umulhi((unsigned)i, inv_bw);
    }

    // Push the window px of string prow as stack member k (stack size becomes
    // k + 1) and filter every remaining string's survivors into level k + 1:
    // keep v iff Hd(top, v) <= 2d (compat bit) and, for every earlier member
    // s_a, Cd(s_a, top, v) <= 3d (Theorem 1 with d1 = d2 = d3 = d; its pair
    // conditions already hold).  Returns whether every remaining string still
    // has a survivor (Algorithm 2's R'.size > 0).
    __device__ __forceinline__ bool push_filter(int k, int prow, int px) {
        const int n = I.n, bw = I.bw, r = I.r;
        const int ug = prow * r + px;
        const Lm<W> top = L[ug];
        if (lane == 0) S.st[k] = top;
        if (lane < k) {
            M e = dmask(S.st[lane], top);
            S.E[lane][k] = e;
            S.HD[lane][k] = pc(e);
        }
        if (lane < kMaxN) cntw[(k + 1) * kMaxN + lane] = 0u;
        const uint32_t rows = S.rows[k] & ~(1u << prow);
        __syncthreads();
        const uint64_t* Cu = I.c1only ? C : C + (int64_t)ug * n * bw;  // unused when c1only
        if (k == 1)
            filter_body(C + (int64_t)u1g * n * bw, Cu, top, k, rows);
        else
            filter_body(level(k), Cu, top, k, rows);
        __syncthreads();
        const bool bad = lane < n && ((rows >> lane) & 1u) && cnt16(k + 1, lane) == 0;
        if (lane == 0) S.rows[k + 1] = rows;
        __syncthreads();
        return ballot(bad) == 0ull;
    }

    // Lanes over the row words of the remaining strings: child = parent AND
    // compat(top).  With the Theorem 1 filter, the set bits of each block of
    // 64 words are listed in LDS (s2cap entries per pass: l-mer index and
    // word/bit) by a wave prefix sum, lanes then test one listed survivor
    // each (independent l-mer loads) and clear the failures with an LDS
    // atomic AND.  Counts are taken afterwards.
    template <typename PP>
    __device__ __forceinline__ void filter_body(PP parent, const uint64_t* Cu, const Lm<W>& top,
                                                int k, uint32_t rows) {
        const int bw = I.bw, r = I.r;
        uint64_t* child = level(k + 1);
        const int total = I.n * bw;
        const int thr3 = 3 * I.d;
        Lm<W> sa[TMAX];
        M ea[TMAX];
        int ha[TMAX];
#pragma unroll
        for (int a = 0; a < TMAX; a++) {
            const int aa = a < k ? a : 0;
            sa[a] = S.st[aa];
            ea[a] = S.E[aa][k];
            ha[a] = S.HD[aa][k];
        }
        // without the compat rows of the other strings (c1only), every parent
        // survivor is listed and tested for Hd(top, v) <= 2d directly
        const bool fly = I.c1only != 0;
        const int d2 = 2 * I.d;
        for (int i0 = 0; i0 < total; i0 += 64) {
            const int i = i0 + lane;
            const int j = row_of(i);
            const bool act = i < total && ((rows >> j) & 1u);
            const uint64_t nb = act ? (fly ? parent[i] : (parent[i] & Cu[i])) : 0ull;
            if (act) child[i] = nb;
            if (!I.triple && !fly) continue;
            const int c = pc(nb);
            const int incl = wave_incl_scan(c);
            const int T = uni(__shfl(incl, 63, 64));
            const int w = i - j * bw;
            for (int lo = 0; lo < T; lo += s2cap) {
                // list the bits of rank [lo, lo + s2cap) of this block
                int rank = incl - c;
                uint64_t bits = nb;
                while (bits && rank < lo + s2cap) {
                    const int bb = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    if (rank >= lo) {
                        s2[rank - lo].h = (M)(j * r + w * 64 + bb);
                        s2[rank - lo].lo = (M)((i << 6) | bb);
                    }
                    rank++;
                }
                __syncthreads();
                const int cnt = T - lo < s2cap ? T - lo : s2cap;
                // four listed survivors per lane per round: their l-mer loads
                // are independent and in flight together
                for (int q0 = 0; q0 < cnt; q0 += 256) {
                    Lm<W> v[4];
                    int e[4];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        const int q = q0 + 64 * u + lane;
                        e[u] = -1;
                        v[u] = lm_zero<W>();
                        if (q < cnt) {
                            e[u] = (int)s2[q].lo;
                            v[u] = L[(int)s2[q].h];
                        }
                    }
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        if (e[u] < 0) continue;
                        const int hv = pc(dmask(top, v[u]));
                        bool ok = !fly || hv <= d2;
                        if (I.triple) {
#pragma unroll
                            for (int a = 0; a < TMAX; a++) {
                                if (a < k) {
                                    const M da = dmask(sa[a], v[u]);
                                    ok &= ha[a] + pc(da) + hv - pc((M)(ea[a] | da)) <= thr3;
                                }
                            }
                        }
                        if (!ok)
                            atomicAnd((unsigned long long*)&child[e[u] >> 6], ~(1ull << (e[u] & 63)));
                    }
                }
                __syncthreads();
            }
        }
        __syncthreads();
        for (int i0 = 0; i0 < total; i0 += 64) {
            const int i = i0 + lane;
            const int j = row_of(i);
            if (i < total && ((rows >> j) & 1u)) {
                const int c = pc(child[i]);
                if (c) atomicAdd(&cnt_word(k + 1, j), (unsigned)c);
            }
        }
    }

    __device__ __forceinline__ int choose_row(int k) {
        const uint32_t rows = S.rows[k];
        int v = 0x7FFFFFFF;
        if (lane < I.n && ((rows >> lane) & 1u)) v = (int)(cnt16(k, lane) << 5) | lane;
        v = wave_min(v);
        return v & 31;
    }

    // window of the survivor of rank nth (0-based) of string p at level k,
    // or -1 if the string has no more survivors; lanes hold one word each
    // per block of 64 words
    __device__ __forceinline__ int nth_bit(int k, int p, int nth) {
        const uint64_t* row = level(k) + p * I.bw;
        int done = 0;
        for (int w0 = 0; w0 < I.bw; w0 += 64) {
            const uint64_t w = w0 + lane < I.bw ? row[w0 + lane] : 0ull;
            const int c = pc(w);
            const int incl = done + wave_incl_scan(c);
            const unsigned long long m = ballot(incl - c <= nth && nth < incl);
            if (m != 0ull) {
                const int src = __builtin_ctzll(m);
                int res = -1;
                if (lane == src) {
                    uint64_t x = w;
                    for (int i = incl - c; i < nth; i++) x &= x - 1;
                    res = (w0 + lane) * 64 + __builtin_ctzll(x);
                }
                return __shfl(res, src, 64);
            }
            done = uni(__shfl(incl, 63, 64));
        }
        return -1;
    }

    // next survivor of string p at level k with window >= from, or -1
    __device__ __forceinline__ int next_bit(int k, int p, int from) {
        const uint64_t* row = level(k) + p * I.bw;
        int w = from >> 6;
        if (w >= I.bw) return -1;
        uint64_t bits = row[w] & (~0ull << (from & 63));
        while (true) {
            if (bits) return w * 64 + __builtin_ctzll(bits);
            if (++w >= I.bw) return -1;
            bits = row[w];
        }
    }

    // Append the motifs of the lanes with ok (their keys) to the instance's
    // output: one atomic per wave.
    __device__ __forceinline__ void emit(const Lm<W>& mv, bool ok) {
        const unsigned long long em = ballot(ok);
        if (em == 0ull) return;
        unsigned long long base = 0;
        if (lane == __builtin_ctzll(em)) base = atomicAdd(&ctr[inst].out_count, (unsigned long long)__popcll(em));
        base = __shfl(base, __builtin_ctzll(em), 64);
        if (!ok) return;
        const unsigned long long at = base + (unsigned long long)rank_below(em);
        if (at < (unsigned long long)I.out_cap) {
            constexpr int KW = KeyWords<W>::value;
            uint64_t* dst = keys + (I.out_off + (int64_t)at) * KW;
            if constexpr (W == 3) {
                // I.abits bits per character, floor(64 / I.abits) per word
                uint64_t k[2] = {0ull, 0ull};
                int wq = 0, sh = 64;
                for (int p = 0; p < I.l; p++) {
                    if (sh < I.abits) {
                        wq = 1;
                        sh = 64;
                    }
                    sh -= I.abits;
                    const uint64_t c = code_at(mv, p);
                    if (wq == 0) k[0] |= c << sh;
                    else k[1] |= c << sh;
                }
                dst[0] = k[0];
                dst[1] = k[1];
            } else {
                const uint64_t h = (uint64_t)mv.h, lo = (uint64_t)mv.lo;
                dst[0] = key_word<W>(h, lo, 0, I.l < 32 ? I.l : 32);
                if (W == 2) dst[1] = I.l > 32 ? key_word<W>(h, lo, 32, I.l) : 0ull;
            }
        } else {
            atomicOr(&ctr[inst].flags, kFlagOutOverflow);
        }
    }

    // Staged l-mer i: 4-byte packed (planes in the low and high 16 bits)
    // when l <= 16, else the plain l-mer.
    __device__ __forceinline__ uint32_t* s2h() const { return reinterpret_cast<uint32_t*>(s2); }
    __device__ __forceinline__ Lm<W> s2get(int i) const {
        if (W == 1 && half) {
            const uint32_t v = s2h()[i];
            Lm<W> x = lm_zero<W>();
            x.h = (M)(v & 0xFFFFu);
            x.lo = (M)(v >> 16);
            return x;
        }
        return s2[i];
    }

    // Segments of the strings in vrows at level k, fewest survivors first
    // (ties: lower string first), and, if their survivors fit the staging
    // area, the survivors themselves in that order.  Returns whether they
    // were staged.
    __device__ __forceinline__ bool stage_rows(int k, uint32_t vrows) {
        const int n = I.n;
        const bool mine = lane < n && ((vrows >> lane) & 1u);
        const int c = mine ? (int)cnt16(k, lane) : 0;
        const int incl = wave_incl_scan(c);
        const int tot = uni(__shfl(incl, 63, 64));
        int rank = 0;
        for (int j = 0; j < n; j++) {
            const int cj = __shfl(c, j, 64);
            const bool in = (vrows >> j) & 1u;
            rank += (in && (cj < c || (cj == c && j < lane))) ? 1 : 0;
        }
        const int R = __popcll(ballot(mine));
        __syncthreads();
        if (mine) {
            S.segoff[rank] = (uint16_t)c;  // count, turned into a start below
            S.segrow[rank] = (uint8_t)lane;
        }
        __syncthreads();
        const int cr = lane < R ? (int)S.segoff[lane] : 0;
        const int ir = wave_incl_scan(cr);
        __syncthreads();
        if (lane < R) S.segoff[lane] = (uint16_t)(ir - cr);
        if (lane == 0) {
            S.segoff[R] = (uint16_t)(tot < 65535 ? tot : 65535);
            S.nseg = R;
        }
        __syncthreads();
        if (tot > scap || R == 0) return R == 0;
        const int rowbase = mine ? (int)S.segoff[rank] : 0;
        const int natural = incl - c;  // start of this string in index order
        const uint64_t* lvk = level(k);
        const int total = n * I.bw;
        int done = 0;
        for (int i0 = 0; i0 < total; i0 += 64) {
            const int i = i0 + lane;
            const int j = row_of(i);
            uint64_t bits = (i < total && ((vrows >> j) & 1u)) ? lvk[i] : 0ull;
            const int cb = pc(bits);
            const int inc = wave_incl_scan(cb);
            const int jj = j < 64 ? j : 0;
            const int nat_j = __shfl(natural, jj, 64);
            const int base_j = __shfl(rowbase, jj, 64);
            int o = base_j + (done + inc - cb - nat_j);
            const int w = i - j * I.bw;
            while (bits) {
                const int b = __builtin_ctzll(bits);
                bits &= bits - 1;
                const int g = j * I.r + w * 64 + b;
                if (W == 1 && half) s2h()[o++] = (uint32_t)g;
                else s2[o++].h = (M)g;
            }
            done += uni(__shfl(inc, 63, 64));
        }
        __syncthreads();
        // four loads in flight per lane
        for (int q0 = 0; q0 < tot; q0 += 256) {
            Lm<W> x[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int q = q0 + 64 * u + lane;
                if (q < tot) x[u] = L[(W == 1 && half) ? (int)s2h()[q] : (int)s2[q].h];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int q = q0 + 64 * u + lane;
                if (q < tot) {
                    if (W == 1 && half) s2h()[q] = (uint32_t)x[u].h | ((uint32_t)x[u].lo << 16);
                    else s2[q] = x[u];
                }
            }
        }
        __syncthreads();
        return true;
    }

    // Windows of the survivors of string p at level k with rank in [a, b)
    // (b - a <= kTailSlots) into S.xs; returns how many.
    __device__ __forceinline__ int list_candidates(int k, int p, int a, int b) {
        const uint64_t* row = level(k) + p * I.bw;
        int done = 0;
        for (int w0 = 0; w0 < I.bw && done < b; w0 += 64) {
            const uint64_t w = w0 + lane < I.bw ? row[w0 + lane] : 0ull;
            const int c = pc(w);
            const int incl = done + wave_incl_scan(c);
            int rank = incl - c;
            uint64_t bits = w;
            while (bits && rank < b) {
                const int bb = __builtin_ctzll(bits);
                bits &= bits - 1;
                if (rank >= a) S.xs[rank - a] = (w0 + lane) * 64 + bb;
                rank++;
            }
            done = uni(__shfl(incl, 63, 64));
        }
        __syncthreads();
        const int hi = b < done ? b : done;
        return hi > a ? hi - a : 0;
    }

    // ---- the tail batch: generation over subtrees, check, emission ----

    // Valid children (4-bit mask) of the node at depth P whose prefix is mv
    // (characters 0..P-1), for members mh/ml[0..K) with pair masks e2:
    // Algorithm 1's prune with budgets d - Hd(prefix) and suffixes from P+1.
    __device__ __forceinline__ uint32_t expand(const Lm<W> (&mm)[TMAX], const M (&e2)[TMAX][TMAX],
                                               int K, const Lm<W>& v, int P) const {
        const M below = low_bits((M)0, P);
        const int d = I.d;
        // every letter: codes 0..3 in the two-plane class (a smaller
        // alphabet's codes are masked once at the end), I.amask otherwise
        const uint32_t full = W == 3 ? I.amask : 0xFu;
        int rb[TMAX];
        uint32_t oh[TMAX];
        uint32_t allowed = full;
#pragma unroll
        for (int a = 0; a < TMAX; a++) {
            if (a < K) {
                rb[a] = d - pc((M)(dmask(v, mm[a]) & below));
                oh[a] = 1u << code_at(mm[a], P);
                allowed &= rb[a] >= 1 ? full : rb[a] == 0 ? oh[a] : 0u;
            } else {
                rb[a] = 0;
                oh[a] = full;
            }
        }
        const int sfx = P + 1;
#pragma unroll
        for (int a = 0; a < TMAX; a++)
#pragma unroll
            for (int b = a + 1; b < TMAX; b++)
                if (b < K) allowed &= slack2(rb[a] + rb[b] - pc(suf(e2[a][b], sfx)), oh[a], oh[b], full);
#pragma unroll
        for (int a = 0; a < TMAX; a++)
#pragma unroll
            for (int b = a + 1; b < TMAX; b++)
#pragma unroll
                for (int c = b + 1; c < TMAX; c++)
                    if (c < K) {
                        const M u = (M)(e2[a][b] | e2[a][c]);
                        const M x = (M)(e2[a][b] & e2[a][c] & e2[b][c]);
                        const int cd = pc(suf(u, sfx)) + pc(suf(x, sfx));
                        allowed &= slack3(rb[a] + rb[b] + rb[c] - cd, oh[a], oh[b], oh[c], full);
                    }
        return W == 3 ? allowed : allowed & I.amask;
    }

    // Whether the node at depth P with prefix mv is in the pruned tree
    // (budgets >= 0, pair and triple conditions on suffixes from P).  A
    // valid node's ancestors are valid too (each condition only loosens
    // towards the root), so the valid nodes of one depth split the tree's
    // leaves into disjoint subtrees.
    __device__ __forceinline__ bool node_valid(const Lm<W> (&mm)[TMAX], const M (&e2)[TMAX][TMAX],
                                               int K, const Lm<W>& v, int P) const {
        const M below = low_bits((M)0, P);
        int rb[TMAX];
        bool ok = true;
#pragma unroll
        for (int a = 0; a < TMAX; a++) {
            rb[a] = a < K ? I.d - pc((M)(dmask(v, mm[a]) & below)) : 0;
            ok &= rb[a] >= 0;
        }
#pragma unroll
        for (int a = 0; a < TMAX; a++)
#pragma unroll
            for (int b = a + 1; b < TMAX; b++)
                if (b < K) ok &= pc(suf(e2[a][b], P)) <= rb[a] + rb[b];
#pragma unroll
        for (int a = 0; a < TMAX; a++)
#pragma unroll
            for (int b = a + 1; b < TMAX; b++)
#pragma unroll
                for (int c = b + 1; c < TMAX; c++)
                    if (c < K) {
                        const M u = (M)(e2[a][b] | e2[a][c]);
                        const M x = (M)(e2[a][b] & e2[a][c] & e2[b][c]);
                        ok &= pc(suf(u, P)) + pc(suf(x, P)) <= rb[a] + rb[b] + rb[c];
                    }
        return ok;
    }

    // Which buffered l-mers have a survivor of string `row` (level-k bitset
    // rw, not staged) within d, transposed: lanes hold up to 64 of the
    // survivors at a time (one load each) and the l-mers without a hit yet
    // are walked uniformly, each tested against all of them in one wave
    // instruction.  Bit i of hw[i / 64] is set for l-mer i with a hit.
    template <int V>
    __device__ __forceinline__ void walk_leaves(const Lm<W> (&v)[V], const bool (&mine)[V], int nl,
                                                uint64_t (&hw)[kLeafCap / 64], int& live) const {
        const int d = I.d;
#pragma unroll
        for (int q = 0; q < kLeafCap / 64; q++) {
            if (q * 64 < nl) {
                const int nq = nl - q * 64 < 64 ? nl - q * 64 : 64;
                // the loop state is wave-uniform: keep it in scalar registers
                uint64_t todo = uni64(~hw[q] & (nq == 64 ? ~0ull : ((1ull << nq) - 1ull)));
                uint64_t hit = 0ull;
                while (todo) {
                    // two l-mers per round
                    const int i0 = __builtin_ctzll(todo);
                    todo &= todo - 1;
                    const bool two = todo != 0ull;
                    const int i1 = two ? __builtin_ctzll(todo) : i0;
                    if (two) todo &= todo - 1;
                    const Lm<W> m0 = leaf[q * 64 + i0];
                    const Lm<W> m1 = leaf[q * 64 + i1];
                    bool h0 = false, h1 = false;
#pragma unroll
                    for (int u = 0; u < V; u++) {
                        h0 |= mine[u] && pc(dmask(m0, v[u])) <= d;
                        h1 |= mine[u] && pc(dmask(m1, v[u])) <= d;
                    }
                    const uint64_t b0 = ballot(h0) ? 1ull << i0 : 0ull;
                    const uint64_t b1 = (two && ballot(h1)) ? 1ull << i1 : 0ull;
                    hit = uni64(hit | b0 | b1);
                }
                hw[q] = uni64(hw[q] | hit);
                live -= __popcll(hit);
            }
        }
    }

    // Segments of at most 8 survivors: the wave splits into 64 / C groups of
    // C lanes (C the survivor count rounded up to a power of two), lane x of
    // every group holds survivor x, and each group tests a different
    // buffered l-mer, so one round takes 64 / C l-mers.
    __device__ __forceinline__ void walk_grouped(const Lm<W>& v, bool mine, int C, int nl,
                                                 uint64_t (&hw)[kLeafCap / 64], int& live) {
        const int d = I.d;
        const int G = 64 / C;
        const int j = lane / C;
        const unsigned long long cmask = C >= 64 ? ~0ull : ((1ull << C) - 1ull);
#pragma unroll
        for (int q = 0; q < kLeafCap / 64; q++) {
            if (q * 64 < nl) {
                const int nq = nl - q * 64 < 64 ? nl - q * 64 : 64;
                uint64_t todo = uni64(~hw[q] & (nq == 64 ? ~0ull : ((1ull << nq) - 1ull)));
                while (todo) {
                    // the round's l-mers: the G lowest pending ones, one per group
                    const bool set = (todo >> lane) & 1ull;
                    const int rk = rank_below(todo);
                    const bool sel = set && rk < G;
                    if (sel) S.lix[rk] = lane;
                    __syncthreads();
                    const int nsel = __popcll(todo) < G ? __popcll(todo) : G;
                    const bool act = j < nsel;
                    const Lm<W> m = act ? leaf[q * 64 + S.lix[j]] : lm_zero<W>();
                    const unsigned long long bm = ballot(act && mine && pc(dmask(m, v)) <= d);
                    const bool hit = sel && ((bm >> (rk * C)) & cmask) != 0ull;
                    const unsigned long long hb = ballot(hit);
                    hw[q] = uni64(hw[q] | hb);
                    live -= __popcll(hb);
                    todo = uni64(todo & ~ballot(sel));
                    __syncthreads();  // S.lix is rewritten by the next round
                }
            }
        }
    }

    // Survivors a lane holds per pass (V of them, 64 V per wave), by the
    // segment's size (V up to 4 for the 8-byte l-mers, 2 for the wider
    // ones, whose registers would cost resident waves): each buffered
    // l-mer's visit tests them all.
    template <int V>
    __device__ __forceinline__ void hits_staged_v(int a, int b, int nl,
                                                  uint64_t (&hw)[kLeafCap / 64]) {
        int live = nl;
        for (int c0 = a; c0 < b && live > 0; c0 += 64 * V) {
            Lm<W> v[V];
            bool mine[V];
#pragma unroll
            for (int u = 0; u < V; u++) {
                const int x = c0 + 64 * u + lane;
                mine[u] = x < b;
                v[u] = s2get(mine[u] ? x : a);
            }
            walk_leaves<V>(v, mine, nl, hw, live);
        }
    }

    // The same for a staged segment [a, b) of the staging area.
    __device__ __forceinline__ void hits_staged(int a, int b, int nl,
                                                uint64_t (&hw)[kLeafCap / 64]) {
        const int sz = b - a;
        if (sz <= 8) {
            int C = 1;
            while (C < sz) C <<= 1;
            const int x = lane & (C - 1);
            const bool mine = x < sz;
            const Lm<W> v = s2get(mine ? a + x : a);
            int live = nl;
            walk_grouped(v, mine, C, nl, hw, live);
            return;
        }
        if (W == 1 && sz > 128) hits_staged_v<W == 1 ? 4 : 2>(a, b, nl, hw);
        else if (sz > 64) hits_staged_v<2>(a, b, nl, hw);
        else hits_staged_v<1>(a, b, nl, hw);
    }

    template <int V>
    __device__ __forceinline__ void hits_unstaged_v(const uint64_t* rw, int row, int nl,
                                                    uint64_t (&hw)[kLeafCap / 64]) {
        const int bw = I.bw;
        int w = 0;
        uint64_t rest = uni64(rw[0]);
        int live = nl;  // l-mers without a hit yet
        while (live > 0) {
            // the next (up to) 64 V survivors, in window order, into S.sv
            int cnt = 0;
            while (cnt < 64 * V) {
                if (rest == 0ull) {
                    if (++w >= bw) break;
                    rest = uni64(rw[w]);
                    continue;
                }
                const int pcnt = __popcll(rest);
                const int take = pcnt < 64 * V - cnt ? pcnt : 64 * V - cnt;
                const bool set = (rest >> lane) & 1ull;
                const int rk = rank_below(rest);
                if (set && rk < take) S.sv[cnt + rk] = w * 64 + lane;
                if (take == pcnt) {
                    rest = 0ull;
                } else {
                    // keep the bits from the take-th set bit on
                    const unsigned long long first = ballot(set && rk == take);
                    rest &= ~0ull << __builtin_ctzll(first);
                }
                cnt += take;
            }
            if (cnt == 0) break;
            __syncthreads();
            Lm<W> v[V];
            bool mine[V];
#pragma unroll
            for (int u = 0; u < V; u++) {
                mine[u] = 64 * u + lane < cnt;
                v[u] = mine[u] ? L[row * I.r + S.sv[64 * u + lane]] : lm_zero<W>();
            }
            walk_leaves<V>(v, mine, nl, hw, live);
            __syncthreads();  // S.sv is rewritten by the next pass
        }
    }

    __device__ __forceinline__ void hits_unstaged(const uint64_t* rw, int row, int nl, int sz,
                                                  uint64_t (&hw)[kLeafCap / 64]) {
        if (sz <= 8) {
            // list the (at most 8) survivors, then the grouped walk
            int cnt = 0;
            for (int w = 0; w < I.bw && cnt < sz; w++) {
                const uint64_t bits = uni64(rw[w]);
                if (bits == 0ull) continue;
                const bool set = (bits >> lane) & 1ull;
                const int rk = cnt + rank_below(bits);
                if (set && rk < 8) S.sv[rk] = w * 64 + lane;
                cnt += __popcll(bits);
            }
            if (cnt > 8) cnt = 8;
            __syncthreads();
            int C = 1;
            while (C < cnt) C <<= 1;
            const int x = lane & (C - 1);
            const bool mine = x < cnt;
            const Lm<W> v = mine ? L[row * I.r + S.sv[x]] : lm_zero<W>();
            int live = nl;
            walk_grouped(v, mine, C, nl, hw, live);
            __syncthreads();
            return;
        }
        if (W == 1 && sz > 128) hits_unstaged_v<W == 1 ? 4 : 2>(rw, row, nl, hw);
        else if (sz > 64) hits_unstaged_v<2>(rw, row, nl, hw);
        else hits_unstaged_v<1>(rw, row, nl, hw);
    }

    // Check the buffered l-mers against every remaining string, one string
    // (segment) at a time, fewest survivors first; the l-mers that have a
    // survivor of that string within d are compacted in place and go on to
    // the next string, the rest are motifs.  The survivors come from the
    // staging area, or from the string's level-k bitset when not staged.
    __device__ __forceinline__ void check_leaves(int k, int nl, bool staged) {
        const int nseg = S.nseg, bw = I.bw;
        const uint64_t* lvk = k >= 2 ? level(k) : nullptr;
        for (int g = 0; g < nseg && nl > 0; g++) {
            uint64_t hw[kLeafCap / 64];
#pragma unroll
            for (int q = 0; q < kLeafCap / 64; q++) hw[q] = 0ull;
            if (staged) {
                hits_staged(S.segoff[g], S.segoff[g + 1], nl, hw);
            } else {
                const int row = S.segrow[g];
                hits_unstaged(lvk + row * bw, row, nl, (int)cnt16(k, row), hw);
            }
            // keep the l-mers with a hit, in order
            int keep_n = 0;
#pragma unroll
            for (int q = 0; q < kLeafCap / 64; q++) {
                if (q * 64 < nl) {
                    const int i = q * 64 + lane;
                    const bool act = i < nl;
                    const Lm<W> mv = act ? leaf[i] : lm_zero<W>();
                    const bool hit = act && ((hw[q] >> lane) & 1ull);
                    const unsigned long long hm = ballot(hit);
                    __syncthreads();  // every lane has read its l-mer before the compaction
                    if (hit) leaf[keep_n + rank_below(hm)] = mv;
                    keep_n += __popcll(hm);
                    __syncthreads();
                }
            }
            nl = keep_n;
        }
        for (int c0 = 0; c0 < nl; c0 += 64) {
            const int i = c0 + lane;
            Lm<W> mv = lm_zero<W>();
            const bool ok = i < nl;
            if (ok) mv = leaf[i];
            emit(mv, ok);
        }
        __syncthreads();
    }

    // Member K-1 is the slot's candidate (compile-time indices only: K is
    // uniform but not a constant).
    __device__ __forceinline__ void load_slot(Lm<W> (&mm)[TMAX], M (&e2)[TMAX][TMAX], int K,
                                              int sl) const {
        const Lm<W> c = ut[sl];
#pragma unroll
        for (int a = 0; a < TMAX; a++)
            if (a == K - 1) mm[a] = c;
#pragma unroll
        for (int a = 0; a < TMAX; a++)
#pragma unroll
            for (int b = a + 1; b < TMAX; b++)
                if (b == K - 1) e2[a][b] = (M)dmask(mm[a], c);
    }

    // Unvisited children of depth q on a lane's path: 4-bit nibbles in
    // registers (alphabets of up to 4 letters) or a 32-bit mask in LDS.
    __device__ __forceinline__ uint32_t kids_get(const uint64_t (&av)[NW], int q) const {
        if constexpr (W == 3) {
            return cm[q * 64 + lane];
        } else {
            uint32_t nib = 0;
#pragma unroll
            for (int i = 0; i < NW; i++)
                if (i == (q >> 4)) nib = (uint32_t)(av[i] >> (4 * (q & 15))) & 0xFu;
            return nib;
        }
    }
    __device__ __forceinline__ void kids_put(uint64_t (&av)[NW], int q, uint32_t m) const {
        if constexpr (W == 3) {
            cm[q * 64 + lane] = m;
        } else {
#pragma unroll
            for (int i = 0; i < NW; i++)
                if (i == (q >> 4)) {
                    const int sh = 4 * (q & 15);
                    av[i] = (av[i] & ~(0xFull << sh)) | ((uint64_t)m << sh);
                }
        }
    }
    // depth q's entry is empty (every deeper depth is exhausted first)
    __device__ __forceinline__ void kids_fresh(uint64_t (&av)[NW], int q, uint32_t m) const {
        if constexpr (W == 3) {
            cm[q * 64 + lane] = m;
        } else {
#pragma unroll
            for (int i = 0; i < NW; i++)
                if (i == (q >> 4)) av[i] |= (uint64_t)m << (4 * (q & 15));
        }
    }

    // Start a walk at the valid node (vh, vl) of depth P: its child nibble,
    // or a leaf when P == l (returned).
    __device__ __forceinline__ bool start(const Lm<W> (&mm)[TMAX], const M (&e2)[TMAX][TMAX],
                                          int K, const Lm<W>& v, int P, uint64_t (&av)[NW],
                                          uint64_t& nz, bool& has) const {
#pragma unroll
        for (int i = 0; i < NW; i++) av[i] = 0ull;
        nz = 0;
        if (P == I.l) return true;
        const uint32_t nb = expand(mm, e2, K, v, P);
        if (nb) {
            kids_fresh(av, P, nb);
            nz = 1ull << P;
            has = true;
        }
        return false;
    }

    // Generate the common d-neighbourhoods of the live slots' stacks
    // (shared members st[0..K-2], last member ut[slot]) and check them.
    // Lanes walk subtrees on their own; the first subtrees are the valid
    // nodes at depth D of every live slot's tree, and when those are handed
    // out, idle lanes take the shallowest pending child of a busy lane
    // (which drops it from its own walk), so every node is visited once.
    __device__ __forceinline__ void tail_generate(int k, int K, uint32_t alive, bool staged) {
        const int l = I.l;
        const int nalive = __popc(alive);
        if (nalive == 0) return;
        if (lane == 0) {
            int q = 0;
            for (int s = 0; s < kTailSlots; s++)
                if ((alive >> s) & 1u) S.aslot[q++] = s;
        }
        __syncthreads();
        // shared members and their pair masks (uniform)
        Lm<W> mm[TMAX];
        M e2[TMAX][TMAX];
#pragma unroll
        for (int a = 0; a < TMAX; a++) {
            const int aa = a < K - 1 ? a : 0;
            mm[a] = S.st[aa];
#pragma unroll
            for (int b = 0; b < TMAX; b++) e2[a][b] = (a < b && b < K - 1) ? (M)S.E[a][b] : (M)0;
        }
        // first subtrees: every prefix of D characters of every live slot
        // (alphabets of up to 4 letters: D = 2 or 3, base-4 digits; larger
        // alphabets: D = 1)
        const int A = I.asize;
        int D = W == 3 ? 1 : nalive >= 4 ? 2 : 3;
        if (D > l) D = l;
        const int per = W == 3 ? A : 1 << (2 * D);
        const int units = nalive * per;
        int next = 0;
        int nl = 0;
        bool has = false;
        int slot = 0;
        Lm<W> v = lm_zero<W>();
        uint64_t av[NW];
#pragma unroll
        for (int i = 0; i < NW; i++) av[i] = 0ull;
        uint64_t nz = 0;  // depths whose nibble is not zero
        long long guard = 0;
        for (;;) {
            if (++guard > kStepLimit) {
                if (lane == 0) atomicOr(&ctr[inst].flags, kFlagNodeOverflow);
                break;
            }
            bool isleaf = false;
            const unsigned long long need = ballot(!has);
            const int nidle = __popcll(need);
            if (next < units) {
                // hand out the depth-D subtrees (batched: at least 8 idle lanes)
                if (nidle >= 8 || need == ~0ull) {
                    if (!has) {
                        const int u = next + rank_below(need);
                        if (u < units) {
                            const int su = W == 3 ? u / A : u >> (2 * D);
                            slot = S.aslot[su];
                            load_slot(mm, e2, K, slot);
                            const int pre = u - su * per;
                            v = lm_zero<W>();
                            bool in_alpha = true;
                            if constexpr (W == 3) {
                                v = with_char<W>(v, 0, (uint32_t)pre);
                            } else {
                                for (int q = 0; q < D; q++) {
                                    const int ch = (pre >> (2 * (D - 1 - q))) & 3;
                                    in_alpha &= ch < A;
                                    v = with_char<W>(v, q, (uint32_t)ch);
                                }
                            }
                            if (in_alpha && node_valid(mm, e2, K, v, D))
                                isleaf = start(mm, e2, K, v, D, av, nz, has);
                        }
                    }
                    next += nidle;
                }
            } else if (nidle >= 4) {
                // donation: busy lanes with two or more pending children give
                // away the shallowest one
                int q0 = 0;
                uint32_t nib0 = 0;
                bool donor = false;
                if (has) {
                    q0 = __builtin_ctzll(nz);
                    nib0 = kids_get(av, q0);
                    donor = __popcll(nz) >= 2 || __popc(nib0) >= 2;
                }
                const unsigned long long dm = ballot(donor);
                const int ndon = __popcll(dm) < nidle ? __popcll(dm) : nidle;
                if (ndon > 0) {
                    if (donor && rank_below(dm) < ndon) {
                        const int ch = __builtin_ctz(nib0);
                        nib0 &= nib0 - 1;
                        kids_put(av, q0, nib0);
                        if (!nib0) nz &= ~(1ull << q0);
                        const int at = rank_below(dm);
                        S.dq_v[at] = with_char<W>(v, q0, (uint32_t)ch);
                        S.dq_d[at] = (uint8_t)(q0 + 1);
                        S.dq_s[at] = (uint8_t)slot;
                    }
                    __syncthreads();
                    if (!has && rank_below(need) < ndon) {
                        const int at = rank_below(need);
                        slot = S.dq_s[at];
                        load_slot(mm, e2, K, slot);
                        v = S.dq_v[at];
                        isleaf = start(mm, e2, K, v, (int)S.dq_d[at], av, nz, has);
                    }
                    __syncthreads();
                }
            }
            if (has && !isleaf) {
                // deepest depth with an unvisited child
                const int q = 63 - __builtin_clzll(nz);
                uint32_t nib = kids_get(av, q);
                const int ch = __builtin_ctz(nib);
                nib &= nib - 1;
                kids_put(av, q, nib);
                if (!nib) nz &= ~(1ull << q);
                v = with_char<W>(v, q, (uint32_t)ch);
                if (q + 1 == l) {
                    isleaf = true;
                } else {
                    const uint32_t nb = expand(mm, e2, K, v, q + 1);
                    if (nb) {
                        kids_fresh(av, q + 1, nb);
                        nz |= 1ull << (q + 1);
                    }
                }
                if (nz == 0ull) has = false;
            }
            const unsigned long long lm = ballot(isleaf);
            if (isleaf) leaf[nl + rank_below(lm)] = v;
            nl += __popcll(lm);
            const bool done = ballot(has) == 0ull && next >= units;
            if (nl > kLeafCap - 64 || (done && nl > 0)) {
                __syncthreads();
                check_leaves(k, nl, staged);
                nl = 0;
            }
            if (done) break;
        }
        __syncthreads();
    }

    // Whether every staged segment has a survivor within 2d of slot s's
    // candidate (else no l-mer of its tree can be a motif: the pair
    // condition of Section 2.4).  Used for alphabets of more than 4 letters,
    // where it removes many slots; on DNA nearly every slot passes.
    __device__ __forceinline__ bool slot_alive(int s) {
        const Lm<W> cand = ut[s];
        const int d2 = 2 * I.d;
        for (int g = 0; g < S.nseg; g++) {
            const int a = S.segoff[g], b = S.segoff[g + 1];
            bool any = false;
            for (int c0 = a; c0 < b && !any; c0 += 64) {
                const int x = c0 + lane;
                const bool ok = x < b && pc(dmask(cand, s2get(x < b ? x : a))) <= d2;
                any = ballot(ok) != 0ull;
            }
            if (!any) return false;
        }
        return true;
    }

    // Tail batch.  p >= 0: the stack st[0..k) is followed by each survivor
    // of string p at level k with rank in [ra, rb).  p < 0: the stack
    // st[0..k) is complete (one slot).
    __device__ __forceinline__ void tail(int k, int p, int ra, int rb) {
        const uint32_t vrows = p >= 0 ? (S.rows[k] & ~(1u << p)) : S.rows[k];
        const bool staged = stage_rows(k, vrows);
        if (p < 0) {
            if (lane == 0) ut[0] = S.st[k - 1];
            __syncthreads();
            ra = 0;
            rb = 1;
        }
        for (int a = ra; a < rb; a += kTailSlots) {
            const int b = rb - a > kTailSlots ? a + kTailSlots : rb;
            int T = 1;
            uint32_t alive = 1u;
            if (p >= 0) {
                T = list_candidates(k, p, a, b);
                if (T <= 0) break;
                if (lane < T) ut[lane] = L[p * I.r + S.xs[lane]];
                __syncthreads();
                alive = (1u << T) - 1u;
                if (I.asize > 4 && staged)
                    for (int s = 0; s < T; s++)
                        if (!slot_alive(s)) alive &= ~(1u << s);
            }
            tail_generate(k, p >= 0 ? k + 1 : k, alive, staged);
            if (T < b - a) break;
        }
    }
};

// Persistent search over one queue.  phase 0 takes the expansion's items
// (the stack {u1, u2}), phase 1 the part items (the same stack and a rank
// range of the next member's string), phase >= 2 the deep items (a longer
// stack prefix and a rank range).  When the string chosen next has more
// than `split` survivors, the wave keeps ranks [0, split) and queues the
// rest in ranges of `split`: at stack size 2 (phase 0) as part items, at
// stack size 3 and up as deep items for the next phase (deep queues
// alternate between phases).  Each launch drains its queue: every wave
// leaves when it is empty and nothing waits on another wave.  An
// instance's outstanding count is raised for every queued item before the
// item that queues it finishes, so it reaches zero exactly when the
// instance's search is complete; that wave stamps the completion time.
// Four resident waves per SIMD (at most 128 VGPRs; 12 bytes of spills) for
// the 8-byte l-mers up to a stack of three, the batched DNA mix's case:
// 78.2 vs 74.6 instances/s with 256 staged survivors; the others keep the
// registers they need.
template <int W, int TMAX>
__global__ __launch_bounds__(64, (W == 1 && TMAX <= 3) ? 4 : 1) void k_search(const InstDev* __restrict__ insts,
                                               const Lm<W>* __restrict__ lmers,
                                               const uint64_t* __restrict__ compat,
                                               const uint64_t* __restrict__ items,
                                               uint64_t* __restrict__ parts,
                                               DeepItem* __restrict__ deep0,
                                               DeepItem* __restrict__ deep1,
                                               QueueCounters* __restrict__ qs,
                                               uint64_t* __restrict__ keys,
                                               InstCounters* __restrict__ ctr,
                                               int level_words, int lv_words, int s2cap,
                                               int phase, int last_phase, int split) {
    extern __shared__ uint64_t dyn[];
    __shared__ SearchLds<W, TMAX> S;
    __shared__ unsigned cntw[(TMAX + 1) * kMaxN];
    __shared__ int rct[TMAX + 1], rhi[TMAX + 1];  // rank taken next / rank limit, per level
    const int lane = lane_id();
    QueueCounters* q = qs + (phase < 2 ? phase : 2 + (phase & 1));
    QueueCounters* qp = qs + 1;
    const DeepItem* dsrc = (phase & 1) ? deep1 : deep0;              // phase >= 2
    DeepItem* ddst = (phase < 2 || (phase & 1)) ? deep0 : deep1;     // next deep phase
    QueueCounters* qd = qs + ((phase < 2 || (phase & 1)) ? 2 : 3);
    const bool deep_ok = (phase < 2 ? 2 : phase + 1) <= last_phase;
    Lm<W>* s2 = reinterpret_cast<Lm<W>*>(dyn + lv_words);
    Lm<W>* ut = s2 + s2cap;
    Lm<W>* leaf = ut + kTailSlots;
    uint32_t* cm = W == 3 ? reinterpret_cast<uint32_t*>(leaf + kLeafCap) : nullptr;
    for (;;) {
        if (lane == 0) {
            unsigned long long it = atomicAdd(&q->item_next, 1ull);
            S.item = it < q->item_count && it < q->item_cap ? (int)it : -1;
        }
        __syncthreads();
        const int it = uni(S.item);
        __syncthreads();
        if (it < 0) break;
        int inst, u1, p2 = 0, x2 = 0, flev = -1, frlo = 0, frhi = 0;
        const DeepItem* di = dsrc + it;  // phase >= 2 (fields read in place: no local copy)
        if (phase < 2) {
            const uint64_t item = (phase == 0 ? items : parts)[it];
            if (item == kNoItem) continue;
            inst = uni(item_inst(item));
            const int lo = uni(item_lo(item));
            u1 = uni(item_u1(item));
            p2 = uni(item_p2(item));
            x2 = uni(item_x2(item));
            if (phase == 1) {
                flev = 2;
                frlo = lo;
                frhi = lo + split;
            }
        } else {
            inst = uni((int)di->inst);
            u1 = uni((int)di->win[0]);
            flev = uni((int)di->k);
            frlo = uni((int)di->ra);
            frhi = uni((int)di->rb);
        }
        const InstDev I = insts[inst];
        Searcher<W, TMAX> sr{S, dyn, level_words, I, inst, lmers + I.lmer_off,
                             compat + I.compat_off, (uint64_t)u1, keys, ctr, lane, cntw,
                             I.bw > 1 ? (uint32_t)((0xFFFFFFFFull + (uint64_t)I.bw) / (uint64_t)I.bw) : 0u,
                             s2, ut, leaf, s2cap, W == 1 && I.l <= 16,
                             (W == 1 && I.l <= 16) ? 2 * s2cap : s2cap, cm};
        if (lane == 0) {
            S.st[0] = sr.L[u1];
            S.rows[1] = (I.n >= 32 ? 0xFFFFFFFFu : ((1u << I.n) - 1u)) & ~1u;
        }
        if (lane <= TMAX) {
            rct[lane] = 0;
            rhi[lane] = 0x7FFFFFFF;
        }
        __syncthreads();
        const int t = I.t < TMAX ? I.t : TMAX;
        int k = 2, kmin = 2;
        bool run = true;
        if (phase < 2) {
            if (p2 == 0) {  // n == 1: the stack {u1} is complete, nothing to check
                if (lane == 0) S.rows[1] = 0;
                __syncthreads();
                k = 1;
            } else {
                if (lane == 0) {
                    S.prow[1] = p2;
                    S.cursor[1] = x2 + 1;
                }
                run = sr.push_filter(1, p2, x2);
            }
        } else {
            // rebuild the levels of the deep item's stack prefix
            for (int j = 1; j < flev && run; j++) {
                const int rj = uni((int)di->row[j]), wj = uni((int)di->win[j]);
                if (lane == 0) {
                    S.prow[j] = rj;
                    S.cursor[j] = wj + 1;
                }
                run = sr.push_filter(j, rj, wj);
            }
            k = kmin = flev;
        }
        bool descend = true;
        while (run) {
            if (descend) {
                int tp = -2, ra = 0, rb = 0;  // tail batch: string (-1: complete stack), ranks
                int p = 0, cur = 0;
                if (k >= t || S.rows[k] == 0u) {
                    tp = -1;
                } else {
                    p = uni(sr.choose_row(k));
                    const int c = uni((int)sr.cnt16(k, p));
                    int lo = 0, hi = 0x7FFFFFFF;
                    if (k == flev) {
                        // the range this part / deep item covers
                        lo = frlo;
                        hi = frhi;
                        flev = -1;
                        if (lo > 0) {
                            cur = uni(sr.nth_bit(k, p, lo));
                            if (cur < 0) cur = 64 * I.bw;
                        }
                    } else if (c > split && (k >= 3 ? deep_ok : phase == 0)) {
                        // keep ranks [0, split), queue the rest
                        const int extra = (c - 1) / split;
                        unsigned long long base = 0;
                        QueueCounters* qq = k == 2 ? qp : qd;
                        if (lane == 0) base = atomicAdd(&qq->item_count, (unsigned long long)extra);
                        base = __shfl(base, 0, 64);
                        if (base + (unsigned long long)extra <= qq->item_cap) {
                            if (k == 2) {
                                for (int e = lane; e < extra; e += 64)
                                    parts[base + e] = make_item((uint64_t)inst, (uint64_t)((e + 1) * split),
                                                                (uint64_t)u1, (uint64_t)p2, (uint64_t)x2);
                            } else {
                                for (int e = 0; e < extra; e++) {
                                    DeepItem* o = ddst + base + e;
                                    if (lane == 0) {
                                        o->inst = (uint32_t)inst;
                                        o->k = (uint8_t)k;
                                        o->p = (uint8_t)p;
                                        o->ra = (uint16_t)((e + 1) * split);
                                        o->rb = (uint16_t)min((e + 2) * split, 65535);
                                    }
                                    if (lane < k) {
                                        o->win[lane] = (uint16_t)(lane == 0 ? u1 : S.cursor[lane] - 1);
                                        o->row[lane] = (uint8_t)(lane == 0 ? 0 : S.prow[lane]);
                                    }
                                }
                            }
                            if (lane == 0) atomicAdd(&ctr[inst].outstanding, (unsigned long long)extra);
                            hi = split;
                        }
                    }
                    if (k == t - 1) {  // the last member: string p's survivors
                        tp = p;
                        ra = lo;
                        rb = hi;
                    } else if (lane == 0) {
                        S.prow[k] = p;
                        S.cursor[k] = cur;
                        rct[k] = lo;
                        rhi[k] = hi;
                    }
                }
                if (tp != -2) {
                    sr.tail(k, tp, ra, rb);
                    k--;
                    if (k < kmin) break;
                    descend = false;
                    continue;
                }
                __syncthreads();
            }
            const int p = uni(S.prow[k]);
            int x = uni(sr.next_bit(k, p, S.cursor[k]));
            if (x >= 0 && uni(rct[k]) >= uni(rhi[k])) x = -1;
            __syncthreads();
            if (x < 0) {
                k--;
                if (k < kmin) break;
                descend = false;
                continue;
            }
            if (lane == 0) {
                S.cursor[k] = x + 1;
                rct[k]++;
            }
            __syncthreads();
            if (sr.push_filter(k, p, x)) {
                k++;
                descend = true;
            } else {
                descend = false;
            }
        }
        // this item is done
        if (lane == 0) {
            const unsigned long long left = atomicSub(&ctr[inst].outstanding, 1ull);
            if (left == 1ull) ctr[inst].done_at = (unsigned long long)__builtin_amdgcn_s_memrealtime();
        }
    }
}

// ---------------------------------------------------------- sort / unique (a8)
// One block per instance: bitonic sort of the emitted keys (LDS when they fit,
// else in place in HBM), then drop repeats with a block prefix sum.  With a
// sort scratch planned, instances with more keys than one LDS chunk are left
// to the multi-block sort below instead.

template <int KW> struct Key { uint64_t w[KW]; };
template <int KW>
__device__ __forceinline__ bool key_less(const Key<KW>& a, const Key<KW>& b) {
    if (KW == 1) return a.w[0] < b.w[0];
    return a.w[0] < b.w[0] || (a.w[0] == b.w[0] && a.w[KW - 1] < b.w[KW - 1]);
}
template <int KW>
__device__ __forceinline__ bool key_eq(const Key<KW>& a, const Key<KW>& b) {
    bool e = true;
#pragma unroll
    for (int i = 0; i < KW; i++) e &= a.w[i] == b.w[i];
    return e;
}

constexpr int kSortThreads = 1024;

// One compare-exchange step of a bitonic network over P = 2^k keys; `a` is
// either the LDS copy or the HBM array (two separate instantiations, so LDS
// is only ever reached with ds_* instructions).
template <int KW, typename A>
__device__ __forceinline__ void bitonic_steps(A a, int P) {
    for (int size = 2; size <= P; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < P / 2; i += kSortThreads) {
                const int lo = 2 * i - (i & (stride - 1));
                const int hi = lo + stride;
                const bool up = ((lo & size) == 0);
                Key<KW> x = a.get(lo), y = a.get(hi);
                if (key_less(y, x) == up) {
                    a.put(lo, y);
                    a.put(hi, x);
                }
            }
            __syncthreads();
        }
    }
}

template <int KW> struct LdsKeys {
    Key<KW>* p;
    __device__ Key<KW> get(int i) const { return p[i]; }
    __device__ __forceinline__ void put(int i, const Key<KW>& v) const { p[i] = v; }
};
template <int KW> struct HbmKeys {
    Key<KW>* p;
    __device__ Key<KW> get(int i) const { return p[i]; }
    __device__ __forceinline__ void put(int i, const Key<KW>& v) const { p[i] = v; }
};

// Keep a[i] when i == 0 or a[i] != a[i-1]; compacted into g (block prefix sum).
template <int KW, typename A>
__device__ __forceinline__ int unique_into(A a, int n, Key<KW>* g, int* scan) {
    int written = 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c0 = 0; c0 < n; c0 += kSortThreads) {
        const int i = c0 + threadIdx.x;
        Key<KW> v;
        bool keep = false;
        if (i < n) {
            v = a.get(i);
            keep = (i == 0) || !key_eq(v, a.get(i - 1));
        }
        const unsigned long long bm = ballot(keep);
        __syncthreads();  // every read of this chunk precedes the writes below
        if (lane == 0) scan[wid] = __popcll(bm);
        __syncthreads();
        if (threadIdx.x == 0) {
            int acc = 0;
            for (int x = 0; x < kSortThreads / 64; x++) {
                int tmp = scan[x];
                scan[x] = acc;
                acc += tmp;
            }
            scan[kSortThreads / 64] = acc;
        }
        __syncthreads();
        if (keep) g[written + scan[wid] + rank_below(bm)] = v;
        written += scan[kSortThreads / 64];
        __syncthreads();
    }
    return written;
}

template <int KW>
__global__ __launch_bounds__(kSortThreads) void k_sort(const InstDev* __restrict__ insts,
                                                       uint64_t* __restrict__ keys,
                                                       InstCounters* __restrict__ ctr, int multi) {
    constexpr int kLdsKeys = 4096 / KW;
    __shared__ Key<KW> sk[kLdsKeys];
    __shared__ int scan[kSortThreads / 64 + 1];
    const int inst = blockIdx.x;
    const InstDev I = insts[inst];
    const unsigned long long cnt = ctr[inst].out_count;
    if (cnt > (unsigned long long)I.out_cap || (ctr[inst].flags & kFlagOutOverflow)) return;
    const int n = (int)cnt;
    if (n == 0) return;
    int P = 1;
    while (P < n) P <<= 1;
    if (multi && P > kLdsKeys) return;
    Key<KW>* g = reinterpret_cast<Key<KW>*>(keys + I.out_off * KW);
    int written;
    if (P <= kLdsKeys) {
        for (int i = threadIdx.x; i < P; i += kSortThreads) {
            if (i < n) {
                sk[i] = g[i];
            } else {
#pragma unroll
                for (int w = 0; w < KW; w++) sk[i].w[w] = ~0ull;
            }
        }
        __syncthreads();
        bitonic_steps<KW>(LdsKeys<KW>{sk}, P);
        written = unique_into<KW>(LdsKeys<KW>{sk}, n, g, scan);
    } else {
        // P <= out_cap (a power of two >= n): sort in place in HBM
        for (int i = n + threadIdx.x; i < P; i += kSortThreads) {
#pragma unroll
            for (int w = 0; w < KW; w++) g[i].w[w] = ~0ull;
        }
        __syncthreads();
        bitonic_steps<KW>(HbmKeys<KW>{g}, P);
        written = unique_into<KW>(HbmKeys<KW>{g}, n, g, scan);
    }
    if (threadIdx.x == 0) ctr[inst].uniq = (unsigned long long)written;
}

// Multi-block sort of the instances with more emitted keys than one LDS
// chunk (C = 4096 / KW keys): a bitonic network over P = 2^k >= n keys
// (padding slots n .. P-1 of the instance's key area hold the largest
// key), whose stages with a stride of at least C run as passes over HBM and
// whose other stages run per chunk in LDS; the last merge also records each
// chunk's distinct-key count and end keys, a scan turns them into output
// offsets, and the distinct keys are compacted into the sort scratch and
// copied back.  Every kernel walks the candidate list (the instances whose
// key area exceeds C); instances that emitted at most C keys, or whose
// network is shorter than a pass's size, skip it.

struct SortCand {
    int32_t inst;
    int32_t pad;
    int64_t tmp_off;   // u64 offset of its compaction area in the sort scratch
    int64_t side_off;  // u64 offset of its per-chunk records
};

template <int KW> struct SortCtx {
    int n, P, chunks;
    Key<KW>* g;
    Key<KW>* tmp;
    Key<KW>* first;  // [chunks] smallest key of each chunk after the last merge
    Key<KW>* last;   // [chunks] largest
    uint64_t* co;    // [chunks] distinct count (low 32 bits), output offset (high 32)
};

template <int KW>
__device__ __forceinline__ bool sort_ctx(const InstDev* insts, const InstCounters* ctr,
                                         uint64_t* keys, uint64_t* tmp, uint64_t* side,
                                         const SortCand& c, SortCtx<KW>& x) {
    constexpr int C = 4096 / KW;
    const InstDev I = insts[c.inst];
    const unsigned long long cnt = ctr[c.inst].out_count;
    if (cnt > (unsigned long long)I.out_cap || (ctr[c.inst].flags & kFlagOutOverflow)) return false;
    if (cnt <= (unsigned long long)C) return false;
    x.n = (int)cnt;
    x.P = 1;
    while (x.P < x.n) x.P <<= 1;
    x.chunks = x.P / C;
    x.g = reinterpret_cast<Key<KW>*>(keys + I.out_off * KW);
    x.tmp = reinterpret_cast<Key<KW>*>(tmp + c.tmp_off);
    x.first = reinterpret_cast<Key<KW>*>(side + c.side_off);
    x.last = x.first + x.chunks;
    x.co = reinterpret_cast<uint64_t*>(x.last + x.chunks);
    return true;
}

// stages of sizes 2 .. C of every chunk, the padding written first
template <int KW>
__global__ __launch_bounds__(kSortThreads) void k_msort_local(const InstDev* __restrict__ insts,
                                                              const InstCounters* __restrict__ ctr,
                                                              uint64_t* __restrict__ keys,
                                                              uint64_t* __restrict__ tmp,
                                                              uint64_t* __restrict__ side,
                                                              const SortCand* __restrict__ cand) {
    constexpr int C = 4096 / KW;
    __shared__ Key<KW> sk[C];
    SortCtx<KW> x;
    if (!sort_ctx<KW>(insts, ctr, keys, tmp, side, cand[blockIdx.y], x)) return;
    for (int ch = blockIdx.x; ch < x.chunks; ch += gridDim.x) {
        const int base = ch * C;
        for (int i = threadIdx.x; i < C; i += kSortThreads) {
            if (base + i < x.n) {
                sk[i] = x.g[base + i];
            } else {
#pragma unroll
                for (int w = 0; w < KW; w++) sk[i].w[w] = ~0ull;
            }
        }
        __syncthreads();
        for (int size = 2; size <= C; size <<= 1) {
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int j = threadIdx.x; j < C / 2; j += kSortThreads) {
                    const int lo = 2 * j - (j & (stride - 1));
                    const bool up = ((base + lo) & size) == 0;
                    const Key<KW> a = sk[lo], b = sk[lo + stride];
                    if (key_less(b, a) == up) {
                        sk[lo] = b;
                        sk[lo + stride] = a;
                    }
                }
                __syncthreads();
            }
        }
        for (int i = threadIdx.x; i < C; i += kSortThreads) x.g[base + i] = sk[i];
        __syncthreads();
    }
}

// one stage (size, stride >= C) over HBM
template <int KW>
__global__ __launch_bounds__(256) void k_msort_global(const InstDev* __restrict__ insts,
                                                      const InstCounters* __restrict__ ctr,
                                                      uint64_t* __restrict__ keys,
                                                      uint64_t* __restrict__ tmp,
                                                      uint64_t* __restrict__ side,
                                                      const SortCand* __restrict__ cand, int size,
                                                      int stride) {
    SortCtx<KW> x;
    if (!sort_ctx<KW>(insts, ctr, keys, tmp, side, cand[blockIdx.y], x)) return;
    if (size > x.P) return;
    const int half = x.P / 2;
    for (int j = blockIdx.x * 256 + threadIdx.x; j < half; j += gridDim.x * 256) {
        const int lo = 2 * j - (j & (stride - 1));
        const bool up = (lo & size) == 0;
        const Key<KW> a = x.g[lo], b = x.g[lo + stride];
        if (key_less(b, a) == up) {
            x.g[lo] = b;
            x.g[lo + stride] = a;
        }
    }
}

// the stages of strides C/2 .. 1 of size `size` per chunk; after the last
// merge (size == P) each chunk's distinct count and end keys
template <int KW>
__global__ __launch_bounds__(kSortThreads) void k_msort_merge(const InstDev* __restrict__ insts,
                                                              const InstCounters* __restrict__ ctr,
                                                              uint64_t* __restrict__ keys,
                                                              uint64_t* __restrict__ tmp,
                                                              uint64_t* __restrict__ side,
                                                              const SortCand* __restrict__ cand,
                                                              int size) {
    constexpr int C = 4096 / KW;
    __shared__ Key<KW> sk[C];
    __shared__ int red[kSortThreads / 64];
    SortCtx<KW> x;
    if (!sort_ctx<KW>(insts, ctr, keys, tmp, side, cand[blockIdx.y], x)) return;
    if (size > x.P) return;
    const bool final_merge = size == x.P;
    for (int ch = blockIdx.x; ch < x.chunks; ch += gridDim.x) {
        const int base = ch * C;
        for (int i = threadIdx.x; i < C; i += kSortThreads) sk[i] = x.g[base + i];
        __syncthreads();
        for (int stride = C >> 1; stride > 0; stride >>= 1) {
            for (int j = threadIdx.x; j < C / 2; j += kSortThreads) {
                const int lo = 2 * j - (j & (stride - 1));
                const bool up = ((base + lo) & size) == 0;
                const Key<KW> a = sk[lo], b = sk[lo + stride];
                if (key_less(b, a) == up) {
                    sk[lo] = b;
                    sk[lo + stride] = a;
                }
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < C; i += kSortThreads) x.g[base + i] = sk[i];
        if (final_merge) {
            // keys at positions < n only; the chunk's first key counts for now
            int c = 0;
            for (int i = threadIdx.x; i < C; i += kSortThreads)
                c += (base + i < x.n && (i == 0 || !key_eq(sk[i], sk[i - 1]))) ? 1 : 0;
            for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
            if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
            __syncthreads();
            if (threadIdx.x == 0) {
                int t = 0;
                for (int w = 0; w < kSortThreads / 64; w++) t += red[w];
                x.co[ch] = (uint64_t)(uint32_t)t;
                x.first[ch] = sk[0];
                const int in_chunk = x.n - base < C ? x.n - base : C;
                x.last[ch] = sk[in_chunk > 0 ? in_chunk - 1 : 0];
            }
        }
        __syncthreads();
    }
}

// per candidate: drop the chunk-initial repeats, exclusive scan of the
// chunk counts into output offsets, the distinct total
template <int KW>
__global__ __launch_bounds__(64) void k_msort_scan(const InstDev* __restrict__ insts,
                                                   InstCounters* __restrict__ ctr,
                                                   uint64_t* __restrict__ keys,
                                                   uint64_t* __restrict__ tmp,
                                                   uint64_t* __restrict__ side,
                                                   const SortCand* __restrict__ cand) {
    SortCtx<KW> x;
    const SortCand c = cand[blockIdx.x];
    if (!sort_ctx<KW>(insts, ctr, keys, tmp, side, c, x)) return;
    const int lane = lane_id();
    unsigned long long run = 0;
    for (int c0 = 0; c0 < x.chunks; c0 += 64) {
        const int ch = c0 + lane;
        int cnt = 0;
        if (ch < x.chunks && ch * (4096 / KW) < x.n) {
            cnt = (int)(uint32_t)x.co[ch];
            if (ch > 0 && key_eq(x.first[ch], x.last[ch - 1])) cnt--;
        }
        const int incl = wave_incl_scan(cnt);
        if (ch < x.chunks)
            x.co[ch] = (uint64_t)(uint32_t)cnt | ((uint64_t)(run + (unsigned long long)(incl - cnt)) << 32);
        run += (unsigned long long)__shfl(incl, 63, 64);
    }
    if (lane == 0) ctr[c.inst].uniq = run;
}

// distinct keys of every chunk into the scratch at the chunk's offset
template <int KW>
__global__ __launch_bounds__(kSortThreads) void k_msort_compact(const InstDev* __restrict__ insts,
                                                                const InstCounters* __restrict__ ctr,
                                                                uint64_t* __restrict__ keys,
                                                                uint64_t* __restrict__ tmp,
                                                                uint64_t* __restrict__ side,
                                                                const SortCand* __restrict__ cand) {
    constexpr int C = 4096 / KW;
    __shared__ int scan[kSortThreads / 64 + 1];
    SortCtx<KW> x;
    if (!sort_ctx<KW>(insts, ctr, keys, tmp, side, cand[blockIdx.y], x)) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int ch = blockIdx.x; ch < x.chunks; ch += gridDim.x) {
        const int base = ch * C;
        int written = (int)(x.co[ch] >> 32);
        for (int c0 = 0; c0 < C; c0 += kSortThreads) {
            const int i = base + c0 + threadIdx.x;
            Key<KW> v;
#pragma unroll
            for (int w = 0; w < KW; w++) v.w[w] = 0ull;
            bool keep = false;
            if (i < x.n) {
                v = x.g[i];
                keep = i == 0 || !key_eq(v, i == base ? x.last[ch - 1] : x.g[i - 1]);
            }
            const unsigned long long bm = ballot(keep);
            if (lane == 0) scan[wid] = __popcll(bm);
            __syncthreads();
            if (threadIdx.x == 0) {
                int acc = 0;
                for (int q = 0; q < kSortThreads / 64; q++) {
                    const int t = scan[q];
                    scan[q] = acc;
                    acc += t;
                }
                scan[kSortThreads / 64] = acc;
            }
            __syncthreads();
            if (keep) x.tmp[written + scan[wid] + rank_below(bm)] = v;
            written += scan[kSortThreads / 64];
            __syncthreads();
        }
    }
}

// the distinct keys back to the instance's key area
template <int KW>
__global__ __launch_bounds__(256) void k_msort_copy(const InstDev* __restrict__ insts,
                                                    const InstCounters* __restrict__ ctr,
                                                    uint64_t* __restrict__ keys,
                                                    uint64_t* __restrict__ tmp,
                                                    uint64_t* __restrict__ side,
                                                    const SortCand* __restrict__ cand) {
    SortCtx<KW> x;
    const SortCand c = cand[blockIdx.y];
    if (!sort_ctx<KW>(insts, ctr, keys, tmp, side, c, x)) return;
    const long long u = (long long)ctr[c.inst].uniq;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < u; i += (long long)gridDim.x * 256)
        x.g[i] = x.tmp[i];
}

// ------------------------------------------------------------- launchers

hipError_t launch_reset(const LaunchPlan& p, const DevBufs& b, unsigned long long item_cap,
                        unsigned long long part_cap, hipStream_t stream) {
    int blocks = (p.n_inst + 255) / 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, stream, b.ctr, p.n_inst, b.q, item_cap,
                       part_cap, p.deep_cap);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_parts, dim3(1024), dim3(256), 0, stream, b.parts, part_cap);
    return hipGetLastError();
}

hipError_t launch_pack(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.max_n_lmers <= 0) return hipSuccess;
    dim3 grid((p.max_n_lmers + 255) / 256, p.n_inst);
    if (p.words == 1)
        hipLaunchKernelGGL(k_pack<1>, grid, dim3(256), 0, stream, b.inst, b.chars, b.lut,
                           (Lm<1>*)b.lmers, b.ctr);
    else if (p.words == 2)
        hipLaunchKernelGGL(k_pack<2>, grid, dim3(256), 0, stream, b.inst, b.chars, b.lut,
                           (Lm<2>*)b.lmers, b.ctr);
    else
        hipLaunchKernelGGL(k_pack<3>, grid, dim3(256), 0, stream, b.inst, b.chars, b.lut,
                           (Lm<3>*)b.lmers, b.ctr);
    return hipGetLastError();
}

hipError_t launch_compat(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.max_n_lmers <= 0) return hipSuccess;
    if (p.compat_kernel == 2) {
        dim3 grid((unsigned)((p.max_n_lmers + 31) / 32), p.n_inst);
        if (p.words == 1)
            hipLaunchKernelGGL(k_compat_mfma<1>, grid, dim3(64), 0, stream, b.inst,
                               (const Lm<1>*)b.lmers, b.compat);
        else if (p.words == 2)
            hipLaunchKernelGGL(k_compat_mfma<2>, grid, dim3(64), 0, stream, b.inst,
                               (const Lm<2>*)b.lmers, b.compat);
        else
            hipLaunchKernelGGL(k_compat_mfma<3>, grid, dim3(64), 0, stream, b.inst,
                               (const Lm<3>*)b.lmers, b.compat);
        return hipGetLastError();
    }
    const int ntile = (p.max_n_lmers + kCompatTile - 1) / kCompatTile;
    const long tasks = (long)ntile * p.max_n;
    dim3 grid((unsigned)((tasks + 3) / 4), p.n_inst);
    if (p.words == 1)
        hipLaunchKernelGGL(k_compat<1>, grid, dim3(256), 0, stream, b.inst, (const Lm<1>*)b.lmers,
                           b.compat);
    else if (p.words == 2)
        hipLaunchKernelGGL(k_compat<2>, grid, dim3(256), 0, stream, b.inst, (const Lm<2>*)b.lmers,
                           b.compat);
    else
        hipLaunchKernelGGL(k_compat<3>, grid, dim3(256), 0, stream, b.inst, (const Lm<3>*)b.lmers,
                           b.compat);
    return hipGetLastError();
}

hipError_t launch_expand(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.max_r <= 0) return hipSuccess;
    dim3 grid((p.max_r + 3) / 4, p.n_inst);
    hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, stream, b.inst, b.compat, b.items, b.q, b.ctr);
    return hipGetLastError();
}

size_t lmer_bytes(int words) {
    return words == 1 ? sizeof(Lm<1>) : words == 2 ? sizeof(Lm<2>) : sizeof(Lm<3>);
}

size_t search_lds_bytes(const LaunchPlan& p) {
    const size_t lm = lmer_bytes(p.words);
    // levels 2 .. max(2, t-1): the last member never gets a level of its own
    // (the tail batch replaces that push)
    const size_t lv = (size_t)(p.tmax > 3 ? p.tmax - 2 : 1) * (size_t)p.level_words * 8u;
    const size_t tail = (size_t)p.s2cap * lm + (size_t)kTailSlots * lm + (size_t)kLeafCap * lm;
    const size_t kids = p.words == 3 ? (size_t)32 * 64 * 4 : 0;  // child masks per depth and lane
    return lv + tail + kids;
}

template <int W, int TMAX>
static hipError_t search_t(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    const size_t lds = search_lds_bytes(p);
    const int lv_words = (p.tmax > 3 ? p.tmax - 2 : 1) * p.level_words;
    const int last = 1 + p.deep_phases;
    for (int phase = 0; phase <= last; phase++) {
        if (phase >= 3) {
            // the deep queue phase - 1 consumed is appended to by this phase
            hipLaunchKernelGGL(k_reset_queue, dim3(1), dim3(64), 0, stream, b.q, 2 + ((phase - 1) & 1));
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((k_search<W, TMAX>), dim3(p.search_blocks), dim3(64), lds, stream, b.inst,
                           (const Lm<W>*)b.lmers, b.compat, b.items, b.parts, b.deep[0], b.deep[1],
                           b.q, b.keys, b.ctr, p.level_words, lv_words, p.s2cap, phase, last,
                           p.split);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int W>
static hipError_t search_w(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.tmax <= 2) return search_t<W, 2>(p, b, stream);
    if (p.tmax <= 3) return search_t<W, 3>(p, b, stream);
    if (p.tmax <= 4) return search_t<W, 4>(p, b, stream);
    if (p.tmax <= 5) return search_t<W, 5>(p, b, stream);
    if (p.tmax <= 6) return search_t<W, 6>(p, b, stream);
    return search_t<W, 8>(p, b, stream);
}

hipError_t launch_search(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.max_r <= 0 || p.search_blocks <= 0) return hipSuccess;
    return p.words == 1 ? search_w<1>(p, b, stream)
         : p.words == 2 ? search_w<2>(p, b, stream)
                        : search_w<3>(p, b, stream);
}

template <int KW>
static hipError_t sort_kw(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    constexpr int C = 4096 / KW;
    const int multi = p.sort_cands > 0 ? 1 : 0;
    hipLaunchKernelGGL(k_sort<KW>, dim3(p.n_inst), dim3(kSortThreads), 0, stream, b.inst, b.keys,
                       b.ctr, multi);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !multi) return e;
    const SortCand* cand = reinterpret_cast<const SortCand*>(b.sort_cand);
    for (int c0 = 0; c0 < p.sort_cands; c0 += 65535) {
        const int nc = p.sort_cands - c0 < 65535 ? p.sort_cands - c0 : 65535;
        const SortCand* cc = cand + c0;
        const long long maxP = (long long)p.sort_pmax;
        const unsigned chunk_blocks = (unsigned)std::min<long long>(maxP / C, 256);
        const unsigned pair_blocks = (unsigned)std::min<long long>(maxP / 2 / 256, 1024);
        hipLaunchKernelGGL(k_msort_local<KW>, dim3(chunk_blocks, nc), dim3(kSortThreads), 0, stream,
                           b.inst, b.ctr, b.keys, b.sort_tmp, b.sort_side, cc);
        e = hipGetLastError();
        for (long long size = 2 * C; e == hipSuccess && size <= maxP; size <<= 1) {
            for (long long stride = size / 2; e == hipSuccess && stride >= C; stride >>= 1) {
                hipLaunchKernelGGL(k_msort_global<KW>, dim3(pair_blocks, nc), dim3(256), 0, stream,
                                   b.inst, b.ctr, b.keys, b.sort_tmp, b.sort_side, cc, (int)size,
                                   (int)stride);
                e = hipGetLastError();
            }
            if (e == hipSuccess) {
                hipLaunchKernelGGL(k_msort_merge<KW>, dim3(chunk_blocks, nc), dim3(kSortThreads), 0,
                                   stream, b.inst, b.ctr, b.keys, b.sort_tmp, b.sort_side, cc,
                                   (int)size);
                e = hipGetLastError();
            }
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_msort_scan<KW>, dim3(nc), dim3(64), 0, stream, b.inst, b.ctr,
                               b.keys, b.sort_tmp, b.sort_side, cc);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_msort_compact<KW>, dim3(chunk_blocks, nc), dim3(kSortThreads), 0,
                               stream, b.inst, b.ctr, b.keys, b.sort_tmp, b.sort_side, cc);
            e = hipGetLastError();
        }
        if (e == hipSuccess) {
            hipLaunchKernelGGL(k_msort_copy<KW>, dim3(pair_blocks, nc), dim3(256), 0, stream, b.inst,
                               b.ctr, b.keys, b.sort_tmp, b.sort_side, cc);
            e = hipGetLastError();
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_sort(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    return p.kwords == 1 ? sort_kw<1>(p, b, stream) : sort_kw<2>(p, b, stream);
}

size_t sort_cand_bytes() { return sizeof(SortCand); }

void sort_cand_fill(void* dst, int i, int inst, long long tmp_off, long long side_off) {
    SortCand c{};
    c.inst = inst;
    c.tmp_off = tmp_off;
    c.side_off = side_off;
    reinterpret_cast<SortCand*>(dst)[i] = c;
}

}  // namespace pms
