// gfx950 kernels for exact (l,d) planted motif search (PMS8).
//
// Data layout (per instance, all in HBM):
//   chars   n*m bytes, row-major (string i at i*m)
//   lmers   N = n*r packed l-mers, id g = row*r + window.  Planar 2-bit
//           packing: bit p of plane h / lo is the high / low bit of the code
//           of character p, so Hd(u,v) = popcount((u.h^v.h) | (u.lo^v.lo)).
//           W = 1: two 32-bit planes (l <= 32); W = 2: two 64-bit planes.
//   compat  [N][n][bw] u64 bitsets: bit x of word (u, j, x/64) is set iff
//           Hd(u, window x of string j) <= 2d and u is not in string j
//           (the pair condition of Section 2.4, precomputed as Section 2.1
//           describes).
//   keys    motif keys, 2 bits per character, first character in the most
//           significant bits; W words per key.
//
// Pipeline: pack -> compat -> expand (level 1, one wave per S_1 window;
// pushes level-2 work items to a device queue) -> search (persistent waves
// pop items and run the rest of Algorithm 2 depth-first with per-level row
// bitsets in LDS, the Theorem 1 survivor filter, Algorithm 1's pruned tree
// and the candidate check) -> sort/unique.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pms_internal.h"

namespace pms {

template <int W> struct Lm;
template <> struct Lm<1> { uint32_t h, lo; };
template <> struct Lm<2> { uint64_t h, lo; };
template <int W> struct MaskOf { typedef uint64_t type; };
template <> struct MaskOf<1> { typedef uint32_t type; };

__device__ __forceinline__ uint32_t dmask(const Lm<1>& a, const Lm<1>& b) {
    return (a.h ^ b.h) | (a.lo ^ b.lo);
}
__device__ __forceinline__ uint64_t dmask(const Lm<2>& a, const Lm<2>& b) {
    return (a.h ^ b.h) | (a.lo ^ b.lo);
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
                        unsigned long long part_cap) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_inst) {
        ctr[i].out_count = 0;
        ctr[i].uniq = 0;
        ctr[i].flags = 0;
        ctr[i].pad = 0;
        ctr[i].items = 0;
    }
    if (i < 2) {
        q[i].item_count = 0;
        q[i].item_next = 0;
        q[i].item_cap = i == 0 ? item_cap : part_cap;
        q[i].pad = 0;
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
    M h = 0, lo = 0;
    bool bad = false;
    for (int i = 0; i < I.l; i++) {
        uint32_t c = tab[p[i]];
        bad |= c == 0xFFu;
        h |= (M)((c >> 1) & 1u) << i;
        lo |= (M)(c & 1u) << i;
    }
    if (bad) atomicOr(&ctr[blockIdx.y].flags, kFlagBadChar);
    Lm<W> v;
    v.h = h;
    v.lo = lo;
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
    const int ntile = (N + kCompatTile - 1) / kCompatTile;
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
        if (g < N) {
            u[k] = L[g];
            urow[k] = g / I.r;
        } else {
            u[k].h = 0;
            u[k].lo = 0;
            urow[k] = -1;
        }
    }
    const int thr = 2 * I.d;
    uint64_t* out = compat + I.compat_off;
    for (int w = 0; w < I.bw; w++) {
        const int x = w * 64 + lane;
        const bool valid = x < I.r;
        Lm<W> v;
        if (valid) v = L[j * I.r + x];
        else {
            v.h = 0;
            v.lo = 0;
        }
#pragma unroll
        for (int k = 0; k < kCompatTile; k++) {
            if (urow[k] < 0) continue;
            bool pred = valid && urow[k] != j && pc(dmask(u[k], v)) <= thr;
            unsigned long long b = ballot(pred);
            if (lane == 0) out[((int64_t)(u0 + k) * I.n + j) * I.bw + w] = b;
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
                items[at] = ((uint64_t)inst << 43) | ((uint64_t)u1 << 16);
            else
                atomicOr(&ctr[inst].flags, kFlagItemOverflow);
            atomicAdd(&ctr[inst].items, 1ull);
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
            items[base + o++] =
                ((uint64_t)inst << 43) | ((uint64_t)u1 << 16) | ((uint64_t)p2 << 11) | x2;
        }
        done += __shfl(incl, 63, 64);
    }
}

// --------------------------------------------------------------- search

template <int W, int TMAX>
struct SearchLds {
    uint32_t rows[TMAX + 1];         // strings not on the stack at each level
    int prow[TMAX + 1];              // string whose survivors are pushed next
    int cursor[TMAX + 1];            // next window to try in that string
    Lm<W> st[TMAX];                  // the stack
    typename MaskOf<W>::type E[TMAX][TMAX];  // e(s_a, s_b) differing-position masks
    int HD[TMAX][TMAX];              // Hd(s_a, s_b)
    typename MaskOf<W>::type rh[kRing], rl[kRing];  // generator node ring: prefix planes
    uint8_t rd[kRing];                               // and depth
    Lm<W> cand[kCandCap];            // complete common neighbours awaiting the check
    Lm<W> vset[kVCap];               // staged survivors (verification)
    uint16_t voff[kMaxN + 1];        // segment g of vset: [voff[g], voff[g+1])
    uint16_t rowbase[kMaxN];         // first vset slot of string j's segment
    int nseg;                        // staged segments (remaining strings)
    int item;
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

template <int W, int TMAX>
struct Searcher {
    typedef typename MaskOf<W>::type M;
    SearchLds<W, TMAX>& S;
    uint64_t* lv;  // LDS level bitsets: level k at lv + (k - 2) * level_words
    int level_words;
    const InstDev& I;
    int inst;
    const Lm<W>* L;       // this instance's l-mers
    const uint64_t* C;    // this instance's compat matrix
    uint64_t u1g;         // global id of the level-1 l-mer (string 0)
    Node* nodes;          // this wave's generator stack
    uint64_t* keys;
    InstCounters* ctr;
    int lane;

    __device__ uint64_t* level(int k) { return lv + (k - 2) * level_words; }

    // Push the window px of string prow as stack member k (stack size becomes
    // k + 1) and filter every remaining string's survivors into level k + 1:
    // keep v iff Hd(top, v) <= 2d (compat bit) and, for every earlier member
    // s_a, Cd(s_a, top, v) <= 3d (Theorem 1 with d1 = d2 = d3 = d; its pair
    // conditions already hold).  Returns whether every remaining string still
    // has a survivor (Algorithm 2's R'.size > 0).
    __device__ bool push_filter(int k, int prow, int px) {
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
        const uint64_t* Cu = C + (int64_t)ug * n * bw;
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

    // string index of flattened row word i (i < n * bw <= 1024): an exact
    // reciprocal multiply instead of a division
    __device__ __forceinline__ int row_of(int i) const {
        return (int)(((unsigned)i * (unsigned)inv_bw) >> 16);
    }

    // Lanes over the row words of the remaining strings: child = parent AND
    // compat(top).  With the Theorem 1 filter, the set bits of each block of
    // 64 words are listed in LDS (the staging buffer, kVCap entries per
    // pass: l-mer index and word/bit) by a wave prefix sum, lanes then test
    // one listed survivor each (independent l-mer loads) and clear the
    // failures with an LDS atomic AND.  Counts are taken afterwards.
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
        for (int i0 = 0; i0 < total; i0 += 64) {
            const int i = i0 + lane;
            const int j = row_of(i);
            const bool act = i < total && ((rows >> j) & 1u);
            const uint64_t nb = act ? (parent[i] & Cu[i]) : 0ull;
            if (act) child[i] = nb;
            if (!I.triple) continue;
            const int c = pc(nb);
            const int incl = wave_incl_scan(c);
            const int T = __shfl(incl, 63, 64);
            const int w = i - j * bw;
            for (int lo = 0; lo < T; lo += kVCap) {
                // list the bits of rank [lo, lo + kVCap) of this block
                int rank = incl - c;
                uint64_t bits = nb;
                while (bits && rank < lo + kVCap) {
                    const int bb = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    if (rank >= lo) {
                        S.vset[rank - lo].h = (M)(j * r + w * 64 + bb);
                        S.vset[rank - lo].lo = (M)((i << 6) | bb);
                    }
                    rank++;
                }
                __syncthreads();
                const int cnt = T - lo < kVCap ? T - lo : kVCap;
                for (int q0 = 0; q0 < cnt; q0 += 64) {
                    const int q = q0 + lane;
                    if (q < cnt) {
                        const int g = (int)S.vset[q].h;
                        const int e = (int)S.vset[q].lo;
                        const Lm<W> v = L[g];
                        const int hv = pc(dmask(top, v));
                        bool ok = true;
#pragma unroll
                        for (int a = 0; a < TMAX; a++) {
                            if (a < k) {
                                const M da = dmask(sa[a], v);
                                ok &= ha[a] + pc(da) + hv - pc((M)(ea[a] | da)) <= thr3;
                            }
                        }
                        if (!ok)
                            atomicAnd((unsigned long long*)&child[e >> 6], ~(1ull << (e & 63)));
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

    // counts live in 32-bit LDS words for atomics; cnt16 reads them back
    __device__ unsigned& cnt_word(int k, int j) { return cntw[k * kMaxN + j]; }
    __device__ unsigned cnt16(int k, int j) { return cntw[k * kMaxN + j]; }
    unsigned* cntw;
    int inv_bw;  // ceil(65536 / bw)

    __device__ int choose_row(int k) {
        const uint32_t rows = S.rows[k];
        int v = 0x7FFFFFFF;
        if (lane < I.n && ((rows >> lane) & 1u)) v = (int)(cnt16(k, lane) << 5) | lane;
        v = wave_min(v);
        return v & 31;
    }

    // window of the survivor of rank nth (0-based) of string p at level k,
    // or -1 if the string has no more survivors; lanes hold one word each
    // (bw <= 32)
    __device__ int nth_bit(int k, int p, int nth) {
        const uint64_t* row = level(k) + p * I.bw;
        const uint64_t w = lane < I.bw ? row[lane] : 0ull;
        const int c = pc(w);
        const int incl = wave_incl_scan(c);
        const unsigned long long m = ballot(incl - c <= nth && nth < incl);
        if (m == 0ull) return -1;
        const int src = __builtin_ctzll(m);
        int res = -1;
        if (lane == src) {
            uint64_t x = w;
            for (int i = incl - c; i < nth; i++) x &= x - 1;
            res = lane * 64 + __builtin_ctzll(x);
        }
        return __shfl(res, src, 64);
    }

    // next survivor of string p at level k with window >= from, or -1
    __device__ int next_bit(int k, int p, int from) {
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

    __device__ void emit(const Lm<W>& mv) {
        const uint64_t h = (uint64_t)mv.h, lo = (uint64_t)mv.lo;
        const unsigned long long at = atomicAdd(&ctr[inst].out_count, 1ull);
        if (at < (unsigned long long)I.out_cap) {
            uint64_t* dst = keys + (I.out_off + (int64_t)at) * W;
            dst[0] = key_word<W>(h, lo, 0, I.l < 32 ? I.l : 32);
            if (W == 2) dst[1] = I.l > 32 ? key_word<W>(h, lo, 32, I.l) : 0ull;
        } else {
            atomicOr(&ctr[inst].flags, kFlagOutOverflow);
        }
    }

    // Check candidates cand[0..nc) against every remaining string of level k
    // (Algorithm 2's isMotif on the filtered rows).
    //
    // Staged survivors: one string segment at a time, fewest survivors first,
    // over the candidates still alive.  With A alive candidates padded to a
    // power of two Ap, lane (sub, c) tests candidate c against survivors
    // sub, sub + 64/Ap, ... of the segment; a wave ballot folded over the
    // replicas gives which candidates have a survivor within d.  Those are
    // compacted to the front of cand and the rest are dropped, so a segment
    // costs ceil(size * Ap / 64) steps.  Unstaged (too many survivors for
    // LDS): lane c checks candidate c against the level bitsets.
    __device__ void verify(int k, int nc, bool staged) {
        const int d = I.d;
        if (staged) {
            int A = nc;
            const int R = S.nseg;
            for (int g = 0; g < R && A > 0; g++) {
                const int a = S.voff[g], e = S.voff[g + 1];
                const int lg = A > 32 ? 6 : A > 16 ? 5 : A > 8 ? 4 : A > 4 ? 3 : A > 2 ? 2 : A > 1 ? 1 : 0;
                const int Ap = 1 << lg, P = 64 >> lg;
                const int ci = lane & (Ap - 1), sub = lane >> lg;
                const bool vc = ci < A;
                const Lm<W> mv = S.cand[vc ? ci : 0];
                bool hit = false;
                if (vc)
                    for (int q = a + sub; q < e; q += P) hit |= pc(dmask(mv, S.vset[q])) <= d;
                uint64_t m = ballot(hit);
                for (int sh = 32; sh >= Ap; sh >>= 1) m |= m >> sh;
                const uint64_t found = m & (A >= 64 ? ~0ull : ((1ull << A) - 1ull));
                const bool keep = lane < A && ((found >> lane) & 1ull);
                const Lm<W> mk = S.cand[lane < A ? lane : 0];
                __syncthreads();
                if (keep) S.cand[rank_below(found)] = mk;
                __syncthreads();
                A = __popcll(found);
            }
            if (lane < A) emit(S.cand[lane]);
            __syncthreads();
            return;
        }
        const Lm<W> mv = S.cand[lane < nc ? lane : 0];
        bool ok = lane < nc;
        const uint32_t rows = S.rows[k];
        for (int j = 0; j < I.n; j++) {
            if (!((rows >> j) & 1u)) continue;
            if (ballot(ok) == 0ull) break;
            bool found = false;
            const uint64_t* row = level(k) + j * I.bw;
            for (int w = 0; w < I.bw; w++) {
                uint64_t bits = row[w];
                while (bits) {
                    const int b = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    found |= pc(dmask(mv, L[j * I.r + w * 64 + b])) <= d;
                }
                if (ballot(ok && !found) == 0ull) break;
            }
            ok &= found;
        }
        if (ok) emit(mv);
    }

    // Stage the survivors of level k into LDS if they fit: one segment per
    // remaining string, segments ordered by survivor count (ties: lower
    // string first), so the check meets the most selective strings first.
    __device__ bool stage(int k) {
        const int n = I.n;
        const uint32_t rows = S.rows[k];
        const bool mine = lane < n && ((rows >> lane) & 1u);
        const int c = mine ? (int)cnt16(k, lane) : 0;
        const int incl = wave_incl_scan(c);
        const int tot = __shfl(incl, 63, 64);
        if (tot > kVCap) return false;
        // rank of this string among the remaining ones by (count, index)
        int rank = 0;
        for (int j = 0; j < n; j++) {
            const int cj = __shfl(c, j, 64);
            const bool in = (rows >> j) & 1u;
            rank += (in && (cj < c || (cj == c && j < lane))) ? 1 : 0;
        }
        // segment starts: prefix sum of the counts in rank order
        const unsigned long long inm = ballot(mine);
        const int R = __popcll(inm);
        if (mine) S.voff[rank] = (uint16_t)c;  // count, turned into a start below
        __syncthreads();
        const int cr = lane < R ? (int)S.voff[lane] : 0;
        const int ir = wave_incl_scan(cr);
        __syncthreads();
        if (lane < R) S.voff[lane] = (uint16_t)(ir - cr);
        if (lane == 0) {
            S.voff[R] = (uint16_t)tot;
            S.nseg = R;
        }
        __syncthreads();
        if (mine) S.rowbase[lane] = S.voff[rank];
        const int natural = incl - c;  // start of this string in index order
        __syncthreads();
        // slot -> l-mer index first (ALU only), then one independent load per
        // slot
        const uint64_t* lvk = level(k);
        const int total = n * I.bw;
        int done = 0;
        for (int i0 = 0; i0 < total; i0 += 64) {
            const int i = i0 + lane;
            const int j = row_of(i);
            uint64_t bits = (i < total && ((rows >> j) & 1u)) ? lvk[i] : 0ull;
            const int cb = pc(bits);
            const int inc = wave_incl_scan(cb);
            const int nat_j = __shfl(natural, j < 64 ? j : 0, 64);
            int o = (int)S.rowbase[j < kMaxN ? j : 0] + (done + inc - cb - nat_j);
            const int w = i - j * I.bw;
            while (bits) {
                const int b = __builtin_ctzll(bits);
                bits &= bits - 1;
                S.vset[o++].h = (M)(j * I.r + w * 64 + b);
            }
            done += __shfl(inc, 63, 64);
        }
        __syncthreads();
        for (int q = lane; q < tot; q += 64) S.vset[q] = L[(int)S.vset[q].h];
        __syncthreads();
        return true;
    }

    // Algorithm 1 on the stack st[0..k) with budgets d, pruned by negative
    // budgets, by the pair condition on suffixes (Hd > r_i + r_j) and by
    // Theorem 1 on suffixes of every triple (Cd > r_i + r_j + r_q); a leaf is
    // reported only with every budget >= 0.  Wave-parallel: each step pops up
    // to 16 nodes from the top of the node stack and lanes evaluate their 4
    // children; surviving internal children are pushed (ballot + prefix
    // sum), complete l-mers go to the candidate buffer.  A node is its prefix
    // (bit-planes of positions < depth) and its depth; the budgets are
    // recomputed from the prefix.  The stack's top kRing entries live in an
    // LDS ring; older entries move to this wave's global node area in blocks
    // of 64 when the ring fills and come back when pops reach them.
    __device__ void generate(int k) {
        const bool staged = stage(k);
        switch (k) {
            case 1: gen_tree<1>(staged); break;
            case 2: gen_tree<2>(staged); break;
            case 3: if constexpr (TMAX >= 3) gen_tree<3>(staged); break;
            case 4: if constexpr (TMAX >= 4) gen_tree<4>(staged); break;
            case 5: if constexpr (TMAX >= 5) gen_tree<5>(staged); break;
            case 6: if constexpr (TMAX >= 6) gen_tree<6>(staged); break;
            case 7: if constexpr (TMAX >= 7) gen_tree<7>(staged); break;
            case 8: if constexpr (TMAX >= 8) gen_tree<8>(staged); break;
            default: break;
        }
    }

    // The tree for a stack of exactly K members (K known at compile time,
    // so every per-member test is unrolled and evaluated without branches).
    template <int K>
    __device__ void gen_tree(bool staged) {
        const int k = K;
        Lm<W> s[K];
        M e[K][K];
#pragma unroll
        for (int a = 0; a < K; a++) {
            s[a] = S.st[a];
#pragma unroll
            for (int b = 0; b < K; b++) e[a][b] = (a < b) ? S.E[a][b] : (M)0;
        }
        const int l = I.l, d = I.d;
        if (lane == 0) {
            S.rh[0] = 0;
            S.rl[0] = 0;
            S.rd[0] = 0;
        }
        __syncthreads();
        int size = 1;  // stack entries
        int g = 0;     // entries [0, g) are in the global node area, [g, size) in the ring
        int nc = 0;    // candidates waiting in S.cand
        while (size > 0) {
            if (size > kNodeCap - 4 * kNodeBatch) {
                // cannot happen (each depth holds at most one batch of 4*16
                // children); kept as a guard so the stack never overruns
                if (lane == 0) atomicOr(&ctr[inst].flags, kFlagNodeOverflow);
                break;
            }
            const int B = size < kNodeBatch ? size : kNodeBatch;
            const int base = size - B;
            if (base < g) {
                // bring back the block of 64 below the ring (the ring then
                // holds fewer than 16 + 64 entries, so no slot is live twice)
                g -= 64;
                const Node x = nodes[g + lane];
                const int sl = (g + lane) & (kRing - 1);
                S.rh[sl] = (M)x.h;
                S.rl[sl] = (M)x.lo;
                S.rd[sl] = (uint8_t)x.depth;
                __syncthreads();
            }
            const int ni = lane >> 2;
            const int alpha = lane & 3;
            const bool active = ni < B;
            const int rs = (base + (active ? ni : 0)) & (kRing - 1);
            const M nh = S.rh[rs];
            const M nl = S.rl[rs];
            const int p = (int)S.rd[rs];
            __syncthreads();  // every lane has read its node before pushes overwrite
            size = base;
            const M below = p >= 8 * (int)sizeof(M) ? ~(M)0 : (((M)1 << p) - (M)1);
            const int sfx = p + 1;
            bool valid = active;
            int rb[K];
#pragma unroll
            for (int a = 0; a < K; a++) {
                const M da = ((nh ^ s[a].h) | (nl ^ s[a].lo)) & below;
                const int ca = (int)((((uint64_t)s[a].h >> p) & 1ull) << 1 | (((uint64_t)s[a].lo >> p) & 1ull));
                rb[a] = d - pc(da) - (ca != alpha ? 1 : 0);
                valid &= rb[a] >= 0;
            }
#pragma unroll
            for (int a = 0; a < K; a++)
#pragma unroll
                for (int b = a + 1; b < K; b++) valid &= pc(suf(e[a][b], sfx)) <= rb[a] + rb[b];
#pragma unroll
            for (int a = 0; a < K; a++)
#pragma unroll
                for (int b = a + 1; b < K; b++)
#pragma unroll
                    for (int c = b + 1; c < K; c++) {
                        const M u = suf((M)(e[a][b] | e[a][c]), sfx);
                        const M x = suf((M)(e[a][b] & e[a][c] & e[b][c]), sfx);
                        valid &= pc(u) + pc(x) <= rb[a] + rb[b] + rb[c];
                    }
            const M ch = nh | ((M)(alpha >> 1) << p);
            const M cl = nl | ((M)(alpha & 1) << p);
            const bool leaf = valid && sfx == l;
            const bool push = valid && sfx < l;
            const unsigned long long pm = ballot(push);
            const int npush = __popcll(pm);
            if (size + npush - g > kRing) {
                // move the oldest 64 ring entries to the global node area
                // (the ring holds more than kRing - 64 >= 64 of them)
                const int sl = (g + lane) & (kRing - 1);
                Node x;
                x.h = (uint64_t)S.rh[sl];
                x.lo = (uint64_t)S.rl[sl];
                x.bud = 0;
                x.depth = (uint32_t)S.rd[sl];
                x.pad = 0;
                nodes[g + lane] = x;
                g += 64;
                __syncthreads();  // spilled slots read before the pushes reuse them
            }
            if (push) {
                const int sl = (size + rank_below(pm)) & (kRing - 1);
                S.rh[sl] = ch;
                S.rl[sl] = cl;
                S.rd[sl] = (uint8_t)sfx;
            }
            size += npush;
            const unsigned long long lm = ballot(leaf);
            if (leaf) {
                Lm<W> mv;
                mv.h = ch;
                mv.lo = cl;
                S.cand[nc + rank_below(lm)] = mv;
            }
            nc += __popcll(lm);
            __syncthreads();
            if (nc >= 64) {
                verify(k, 64, staged);
                __syncthreads();
                const int rest = nc - 64;
                Lm<W> mv = S.cand[64 + (lane < rest ? lane : 0)];
                __syncthreads();
                if (lane < rest) S.cand[lane] = mv;
                nc = rest;
                __syncthreads();
            }
        }
        if (nc > 0) verify(k, nc, staged);
        __syncthreads();
    }
};

// Persistent search over one queue.  phase 0 takes the expansion's items;
// when the string chosen at stack size 2 has more than `split` survivors,
// the wave keeps ranks [0, split) and appends part items
// for the rest to the part queue, which phase 0 never reads.  phase 1 (a
// second launch after phase 0 has finished) takes the part items.  Every
// wave leaves when its queue is empty; nothing waits on another wave.
template <int W, int TMAX>
__global__ __launch_bounds__(64) void k_search(const InstDev* __restrict__ insts,
                                               const Lm<W>* __restrict__ lmers,
                                               const uint64_t* __restrict__ compat,
                                               const uint64_t* __restrict__ items,
                                               uint64_t* __restrict__ parts,
                                               QueueCounters* __restrict__ qs,
                                               Node* __restrict__ node_scratch,
                                               uint64_t* __restrict__ keys,
                                               InstCounters* __restrict__ ctr,
                                               int level_words, int phase, int split) {
    extern __shared__ uint64_t dyn[];
    __shared__ SearchLds<W, TMAX> S;
    __shared__ unsigned cntw[(TMAX + 1) * kMaxN];
    const int lane = lane_id();
    Node* nodes = node_scratch + (int64_t)blockIdx.x * kNodeCap;
    QueueCounters* q = qs + phase;
    QueueCounters* qp = qs + 1;
    const uint64_t* src = phase == 0 ? items : parts;
    for (;;) {
        if (lane == 0) {
            unsigned long long it = atomicAdd(&q->item_next, 1ull);
            S.item = it < q->item_count && it < q->item_cap ? (int)it : -1;
        }
        __syncthreads();
        const int it = uni(S.item);
        __syncthreads();
        if (it < 0) break;
        const uint64_t item = src[it];
        if (item == kNoItem) continue;
        const int inst = uni((int)(item >> 43));
        const int lo = uni((int)((item >> 32) & 0x7FF));
        const int u1 = uni((int)((item >> 16) & 0xFFFF));
        const int p2 = uni((int)((item >> 11) & 31));
        const int x2 = uni((int)(item & 0x7FF));
        const InstDev I = insts[inst];
        Searcher<W, TMAX> sr{S, dyn, level_words, I, inst, lmers + I.lmer_off,
                             compat + I.compat_off, (uint64_t)u1, nodes, keys, ctr, lane};
        sr.cntw = cntw;
        sr.inv_bw = (65536 + I.bw - 1) / (I.bw > 0 ? I.bw : 1);
        if (lane == 0) {
            S.st[0] = sr.L[u1];
            S.rows[1] = (I.n >= 32 ? 0xFFFFFFFFu : ((1u << I.n) - 1u)) & ~1u;
        }
        __syncthreads();
        const int t = I.t < TMAX ? I.t : TMAX;
        if (p2 == 0) {  // n == 1: the stack {u1} is complete, nothing to check
            if (lane == 0) S.rows[1] = 0;
            __syncthreads();
            sr.generate(1);
            continue;
        }
        if (!sr.push_filter(1, p2, x2)) continue;
        int k = 2;
        bool descend = true;
        int rank2 = 0, rank2_end = 0x7FFFFFFF;  // survivor ranks this item covers at k == 2
        for (;;) {
            if (descend) {
                if (k >= t || S.rows[k] == 0u) {
                    sr.generate(k);
                    k--;
                    if (k < 2) break;
                    descend = false;
                    continue;
                }
                const int p = uni(sr.choose_row(k));
                int cur = 0;
                if (k == 2) {
                    const int c = uni((int)sr.cnt16(2, p));
                    if (phase == 0) {
                        if (c > split) {
                            const int extra = (c - 1) / split;
                            unsigned long long base = 0;
                            if (lane == 0) base = atomicAdd(&qp->item_count, (unsigned long long)extra);
                            base = __shfl(base, 0, 64);
                            if (base + (unsigned long long)extra <= qp->item_cap) {
                                for (int e = lane; e < extra; e += 64)
                                    parts[base + e] = item | ((uint64_t)((e + 1) * split) << 32);
                                rank2_end = split;
                            }
                        }
                    } else {
                        rank2 = lo;
                        rank2_end = lo + split;
                        cur = uni(sr.nth_bit(2, p, lo));
                        if (cur < 0) cur = 64 * I.bw;
                    }
                }
                if (lane == 0) {
                    S.prow[k] = p;
                    S.cursor[k] = cur;
                }
                __syncthreads();
            }
            const int p = uni(S.prow[k]);
            int x = uni(sr.next_bit(k, p, S.cursor[k]));
            if (k == 2 && x >= 0) {
                if (rank2 >= rank2_end) x = -1;
                else rank2++;
            }
            __syncthreads();
            if (x < 0) {
                k--;
                if (k < 2) break;
                descend = false;
                continue;
            }
            if (lane == 0) S.cursor[k] = x + 1;
            __syncthreads();
            if (sr.push_filter(k, p, x)) {
                k++;
                descend = true;
            } else {
                descend = false;
            }
        }
    }
}

// ---------------------------------------------------------- sort / unique (a8)
// One block per instance: bitonic sort of the emitted keys (LDS when they fit,
// else in place in HBM), then drop repeats with a block prefix sum.

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
    __device__ void put(int i, const Key<KW>& v) const { p[i] = v; }
};
template <int KW> struct HbmKeys {
    Key<KW>* p;
    __device__ Key<KW> get(int i) const { return p[i]; }
    __device__ void put(int i, const Key<KW>& v) const { p[i] = v; }
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
                                                       InstCounters* __restrict__ ctr) {
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

// ------------------------------------------------------------- launchers

hipError_t launch_reset(const LaunchPlan& p, const DevBufs& b, unsigned long long item_cap,
                        unsigned long long part_cap, hipStream_t stream) {
    int blocks = (p.n_inst + 255) / 256;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, stream, b.ctr, p.n_inst, b.q, item_cap,
                       part_cap);
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
    else
        hipLaunchKernelGGL(k_pack<2>, grid, dim3(256), 0, stream, b.inst, b.chars, b.lut,
                           (Lm<2>*)b.lmers, b.ctr);
    return hipGetLastError();
}

hipError_t launch_compat(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.max_n_lmers <= 0) return hipSuccess;
    const int ntile = (p.max_n_lmers + kCompatTile - 1) / kCompatTile;
    const long tasks = (long)ntile * p.max_n;
    dim3 grid((unsigned)((tasks + 3) / 4), p.n_inst);
    if (p.words == 1)
        hipLaunchKernelGGL(k_compat<1>, grid, dim3(256), 0, stream, b.inst, (const Lm<1>*)b.lmers,
                           b.compat);
    else
        hipLaunchKernelGGL(k_compat<2>, grid, dim3(256), 0, stream, b.inst, (const Lm<2>*)b.lmers,
                           b.compat);
    return hipGetLastError();
}

hipError_t launch_expand(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.max_r <= 0) return hipSuccess;
    dim3 grid((p.max_r + 3) / 4, p.n_inst);
    hipLaunchKernelGGL(k_expand, grid, dim3(256), 0, stream, b.inst, b.compat, b.items, b.q, b.ctr);
    return hipGetLastError();
}

size_t search_lds_bytes(const LaunchPlan& p) {
    int tm = p.tmax;
    return (size_t)(tm > 1 ? tm - 1 : 1) * (size_t)p.level_words * 8u;
}

template <int W, int TMAX>
static hipError_t search_t(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    const size_t lds = search_lds_bytes(p);
    for (int phase = 0; phase < 2; phase++) {
        hipLaunchKernelGGL((k_search<W, TMAX>), dim3(p.search_blocks), dim3(64), lds, stream, b.inst,
                           (const Lm<W>*)b.lmers, b.compat, b.items, b.parts, b.q, b.nodes, b.keys,
                           b.ctr, p.level_words, phase, p.split);
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
    return p.words == 1 ? search_w<1>(p, b, stream) : search_w<2>(p, b, stream);
}

hipError_t launch_sort(const LaunchPlan& p, const DevBufs& b, hipStream_t stream) {
    if (p.words == 1)
        hipLaunchKernelGGL(k_sort<1>, dim3(p.n_inst), dim3(kSortThreads), 0, stream, b.inst, b.keys,
                           b.ctr);
    else
        hipLaunchKernelGGL(k_sort<2>, dim3(p.n_inst), dim3(kSortThreads), 0, stream, b.inst, b.keys,
                           b.ctr);
    return hipGetLastError();
}

}  // namespace pms
