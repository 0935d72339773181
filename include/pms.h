/*
 * pms.h -- exact (l,d) planted motif search (PMS8) on one MI355X (gfx950).
 *
 * The problem (Section 1 of Nicolae & Rajasekaran, "Efficient Sequential and
 * Parallel Algorithms for Planted Motif Search"): given n strings S_1..S_n of
 * length m over an alphabet and integers l, d, report every l-mer M such that
 * every S_i has a window S_i[j..j+l-1] with Hamming distance Hd(M, window) <= d.
 * The result is a set; this library returns it sorted byte-lexicographically
 * with no repeats.
 *
 * Every call below runs the whole method on the GPU: planar l-mer packing,
 * the all-pairs Hd <= 2d compatibility bit-matrix (Section 2.1), the
 * sample-driven search over one l-mer per string with per-string survivor
 * filtering by the pair condition and Theorem 1 (Section 2, Section 2.4,
 * Algorithm 2), the pruned common d-neighbourhood generation (Algorithm 1),
 * the candidate check against every remaining string, and sort/unique.
 *
 * Conventions
 *  - Every function returns PMS_OK (0) or a negative pms_status.
 *  - Strings are NUL-terminated and must have exactly m characters.
 *  - The alphabet has 2 to 32 distinct characters (DNA "ACGT", the 20 amino
 *    acids, ...); characters are case-sensitive.  Codes are assigned in
 *    ascending ASCII order, so the result order is byte order of the motifs.
 *  - Limits of the GPU path: 0 <= d < l, 1 <= n <= 32, m - l + 1 <= 8192;
 *    l <= 64 over alphabets of up to 4 letters, l <= 32 over 5 to 16
 *    letters and l <= 24 over 17 to 32 (two key words of B-bit codes, see
 *    pms_result).  One batch holds either instances with l > 32 or
 *    instances over more than 4 letters, not both.  m < l is valid and
 *    yields the empty set.
 *  - Inputs are caller-owned and read only during the call (create/submit
 *    copy them).  Results are library-allocated host memory released with
 *    pms_result_free().  A hip_stream argument is borrowed (NULL = the
 *    library's own stream).
 *  - Thread safety: pms_solve and pms_solve_batch are reentrant; a pms_batch
 *    is used by one thread at a time; a pms_stream accepts submissions from
 *    any number of threads.
 */
#ifndef PMS_H
#define PMS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMS_OK = 0,
    PMS_E_INVAL = -1,       /* bad n, m, l, d, count, NULL pointer or string length */
    PMS_E_ALPHABET = -2,    /* character outside the alphabet, or repeated alphabet character */
    PMS_E_UNSUPPORTED = -3, /* outside the GPU path's limits (|alphabet| > 32, l > 64, n > 32, ...) */
    PMS_E_NOMEM = -4,       /* host or device allocation failed, or above the admission cap */
    PMS_E_DEVICE = -5,      /* a HIP runtime error */
    PMS_E_AGAIN = -6,       /* stream ticket not finished yet */
    PMS_E_ABORTED = -7,     /* request cancelled (stream destroyed or watchdog) */
    PMS_E_TIMEOUT = -8      /* pms_stream_wait timed out */
} pms_status;

/* One problem instance (Section 1): n strings of length m, motif length l,
 * distance d.  seqs[i] points at S_{i+1}. */
typedef struct pms_instance {
    const char* const* seqs;
    int32_t n;
    int32_t m;
    const char* alphabet;
    int32_t l;
    int32_t d;
} pms_instance;

/* Sorted motif set of one instance. */
typedef struct {
    int64_t count;     /* number of motifs */
    int32_t l;         /* motif length */
    int32_t words;     /* 64-bit words per packed key: ceil(l / floor(64 / B)) */
    char* motifs;      /* count*l characters, no separators, sorted, unique */
    uint64_t* packed;  /* count*words keys: B-bit codes (B = 2 for alphabets
                          of up to 4 letters, else ceil(log2 letters)),
                          floor(64 / B) characters per word, first character
                          in the most significant bits (left-aligned), same
                          order */
} pms_result;

/* Search parameters.  Zero / negative fields mean "choose automatically".
 * None of them except s1_begin / s1_end changes the result set (the method
 * is exact for every setting); they change only speed and memory. */
typedef struct pms_tune {
    int32_t threshold;      /* stack size t at which the search switches to
                               neighbourhood generation (Section 2.2,
                               Appendix D); 2..8, 0 = cost model */
    int32_t lmer_words;     /* alphabets of up to 4 letters: 1: l-mers in
                               2 x 32-bit planes (l <= 32); 2: 2 x 64-bit
                               planes ("128-bit"); 0 = 1 if l<=32.  A batch
                               with a larger alphabet always uses 5 x 32-bit
                               planes */
    int32_t triple_filter;  /* >= 0: filter survivors with Theorem 1 (default),
                               < 0: pairwise 2d filter only */
    int32_t waves_per_cu;   /* resident search waves per CU (persistent grid); 0 = auto */
    int32_t compat_kernel;  /* builder of the compat bit-matrix: 1 VALU
                               xor/popcount; 2 int8 MFMA on one-hot codes
                               (Hd <= 2d as matches >= l - 2d); 0 = 2 for
                               alphabets of up to 4 letters, 1 for larger
                               ones.  Values above 2 are PMS_E_INVAL */
    int32_t split;          /* survivors of the next member's string one wave
                               keeps (1..2047; 0 = 32, or 64 when an instance
                               has more than 12000 l-mers); the rest are queued in
                               ranges of this size for other waves: at stack
                               size 2 as part items (a second launch), at 3
                               and up as deep items (further launches) */
    int32_t s1_begin;       /* search only the S_1 windows [s1_begin, s1_end) */
    int32_t s1_end;         /* (Section 2.3's independent sub-problems).  The
                               result is then the motifs that are within d of
                               one of those windows.  0, 0 = every window;
                               end beyond the last window is clamped;
                               begin > end (end > 0) is PMS_E_INVAL */
    int32_t stage_cap;      /* survivors of the remaining strings staged in LDS
                               for one tail batch (256..4096, rounded up to a
                               multiple of 64; 0 = by the batch's sizes);
                               larger sets are checked from the level bitsets */
    int32_t compat_mode;    /* 1: the whole compat bit-matrix; 2: only the rows
                               of S_1's l-mers (n times less memory; every push
                               tests Hd <= 2d on the survivors directly, the
                               long-sequence mode); 0 = 2 for an instance
                               whose whole matrix exceeds 1 GiB, else 1 */
    int64_t out_capacity;   /* motif slots per instance (before removal of
                               repeats); 0 = 4 x the Appendix C expected
                               number of motifs (pms_expected_motifs) + 64,
                               rounded up to a power of two, at most 2^23; an
                               instance that emits more is solved again alone
                               with room for all it emitted.  At most 2^30
                               (PMS_E_INVAL beyond) */
} pms_tune;

/* Autotuner.  Times the device pipeline on an evenly spread sample of at
 * most `sample` of the instances (0 = 32) for candidate settings -- staged
 * survivors per tail batch, part size, waves per CU, the threshold t (which
 * Section 2.2 and Appendix D leave to measurement), the Theorem 1 filter,
 * the l-mer width -- one parameter at a time from
 * `base` (NULL = the defaults), at most max_runs pipeline runs (0 = 16),
 * keeping a change only when it is at least 2% faster on the sample, and
 * writes the best setting to out (a sample can mislead: time the proposal
 * on the whole batch before relying on it).  No setting changes the motif
 * sets; a candidate whose counts differ from the base's is rejected.  The
 * result is cached for batches of the same shape (the distinct (l, d, n/8,
 * m/256, alphabet size) of the instances and log2 of their number), in the
 * process and in the file PMS_TUNE_CACHE names if set;
 * pms_solve_batch / pms_batch_create / pms_batch_workspace_size with
 * tune == NULL use it.  Blocks; uses the device. */
int pms_autotune(const pms_instance* inst, int32_t count, const pms_tune* base, int32_t max_runs,
                 int32_t sample, pms_tune* out);

/* Solve one instance (Section 1 problem statement).  Blocks until done. */
int pms_solve(const char* const* seqs, int32_t n, int32_t m, const char* alphabet,
              int32_t l, int32_t d, pms_result* out);

/* Solve `count` instances of any mix of (l, d, n, m) in one device pass: one
 * pack launch, one compat launch, a persistent search fed by a device work
 * queue (two launches: the level-2 work items, then the parts of items too
 * large for one wave; plus one per deeper stack level of split work when a
 * threshold exceeds 3), one sort/unique launch, all enqueued back to back on
 * hip_stream (NULL = a stream of the library's own).  outs[i] receives
 * instance i's set.  tune may be NULL (the autotuner's cached setting for
 * this shape of batch, else the defaults).  At most 2^20 - 1 instances per call
 * (PMS_E_UNSUPPORTED beyond). */
int pms_solve_batch(const pms_instance* inst, int32_t count, pms_result* outs,
                    const pms_tune* tune, void* hip_stream);

/* ---- device-resident batches: inputs uploaded once, solved many times ---- */
typedef struct pms_batch pms_batch;

/* Validate, encode and upload the instances; plan and allocate device memory.
 * If workspace is non-NULL it must be device memory of at least
 * pms_batch_workspace_size() bytes, borrowed for the batch's lifetime
 * (PMS_E_NOMEM if smaller); otherwise the library allocates.  The uploads
 * are enqueued on a stream of the batch's own; every later run waits for
 * them on its own stream. */
int pms_batch_create(const pms_instance* inst, int32_t count, const pms_tune* tune,
                     void* workspace, size_t workspace_bytes, pms_batch** out);
/* Device bytes a batch of these instances needs (for a caller workspace). */
int pms_batch_workspace_size(const pms_instance* inst, int32_t count, const pms_tune* tune,
                             size_t* bytes);
/* Enqueue the whole device pipeline on hip_stream (NULL = the batch's own
 * stream; inputs already in HBM) and return without waiting.  The phases
 * are launched back to back; stream order sequences them.  use_graph != 0
 * captures the same launches into a hipGraph on the first call (per
 * stream) and replays it on later calls; no memset node is recorded (the
 * counters are cleared by a kernel).  A launch error makes the batch
 * unusable: later calls return the same status. */
int pms_batch_run(pms_batch* b, void* hip_stream, int32_t use_graph);
/* Wait for the last run (its stream only), copy the sets back.  outs has
 * one slot per instance.  An instance whose motifs outnumbered its output
 * slots is solved again alone, in library-allocated device memory with
 * slots for all of them; the other results come from the run itself. */
int pms_batch_results(pms_batch* b, pms_result* outs);
/* Per-phase device times of the last run in milliseconds (pack, compat,
 * expand, search, sort), measured with HIP events on the run's stream. */
int pms_batch_timings(pms_batch* b, float* ms5);
int pms_batch_destroy(pms_batch* b);

/* Work one instance of the last run performed, in the method's own units.
 * compat_pairs is the number of unordered pairs of l-mers from different
 * strings (each one Hamming test of the compatibility matrix, Section 2.1);
 * items are the level-2 work items the expansion queued; motifs_emitted
 * counts motifs before removal of repeats; done_ticks is the device clock
 * (100 MHz) at which the instance's last search work item finished (0 if
 * it had none), so differences between instances of one run give their
 * completion order and spread.  The search-side counters (pushes ...
 * verify_tests) are -1: they are not counted on the device. */
typedef struct {
    int64_t compat_pairs;
    int64_t items;
    int64_t pushes;
    int64_t filter_words;
    int64_t triple_tests;
    int64_t tuples;
    int64_t gen_evals;
    int64_t candidates;
    int64_t verify_tests;
    int64_t motifs_emitted;  /* before removal of repeats */
    int64_t done_ticks;
} pms_work;
int pms_batch_work(pms_batch* b, int32_t instance, pms_work* out);

/* ---- serving: continuous batching with admission by device memory ----
 * The stream owns one device pool of device_mem_cap bytes (allocated on the
 * first pass).  `workers` threads each form a device pass from the queued
 * requests whenever they are free and run it on their own non-blocking
 * stream in a block of the pool, so passes overlap on the device; a request
 * is admitted when its memory bound fits in the pool beside the passes
 * already running. */
typedef struct {
    int64_t device_mem_cap;  /* device pool bytes; 0 = 32 GiB */
    int32_t max_inflight;    /* instances resident at once; 0 = 256 */
    int32_t max_wave;        /* instances admitted per device pass; 0 = 64 */
    pms_tune tune;
    int32_t workers;         /* passes on the device at once; 0 = 3 (at most 16) */
} pms_stream_config;

typedef struct pms_stream pms_stream;

int pms_stream_create(const pms_stream_config* cfg, pms_stream** s);
/* Copy the instance and queue it; returns a ticket.  PMS_E_NOMEM if the
 * instance alone exceeds device_mem_cap. */
int pms_stream_submit(pms_stream* s, const pms_instance* inst, uint64_t* ticket);
/* PMS_E_AGAIN while not finished; otherwise the ticket's status and set. */
int pms_stream_poll(pms_stream* s, uint64_t ticket, pms_result* out);
/* Block until finished or timeout_us elapses (<0: forever). */
int pms_stream_wait(pms_stream* s, uint64_t ticket, pms_result* out, int64_t timeout_us);
/* Finishes in-flight work, fails queued tickets with PMS_E_ABORTED, frees. */
int pms_stream_destroy(pms_stream* s);

/* ---- allocation-free variant of pms_solve ----
 * For callers that cannot allocate device memory: code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Solves
 * one instance with every intermediate buffer in a fixed device array of
 * the library (pms_noalloc_scratch_bytes() = 256 MiB per GPU, held from the
 * first call on that GPU until the process ends); calls no hipMalloc,
 * hipFree or other allocating routine and enqueues only kernels (no memset
 * or copy) on hip_stream (NULL = the legacy default stream), then returns
 * without waiting.
 *   chars     device, n*m characters, string i at chars + i*m (no
 *             terminators); caller-owned, read until the stream reaches the
 *             end of this call's work.
 *   alphabet  host string of exactly 4 distinct characters (DNA "ACGT");
 *             codes by ascending byte value, as for pms_solve.
 *   keys_out  device, keys_cap * words uint64 (words = 1 if l <= 32, else 2):
 *             receives the sorted motif set as pms_result.packed lays it out.
 *   count_out device int64: the number of motifs, or a negative pms_status:
 *             PMS_E_ALPHABET (a window holds a character outside the
 *             alphabet), PMS_E_NOMEM (more motifs than keys_cap, or more
 *             emitted motifs than the scratch's key slots).
 * An instance whose whole compat bit-matrix would take over a quarter of the
 * array keeps only the rows of S_1's l-mers (pms_tune.compat_mode 2); its
 * work items take (m-l+1)^2 * 8 bytes, so m-l+1 stays below about 5000.
 * Returns PMS_E_INVAL / PMS_E_ALPHABET / PMS_E_UNSUPPORTED as pms_solve does
 * for bad arguments, PMS_E_NOMEM when the instance's buffers do not fit in
 * the scratch array (nothing is enqueued then), PMS_E_DEVICE on a launch
 * error.  Every call on one GPU uses the same scratch and leaves its
 * contents there; calls that overlap on one GPU (other streams, threads)
 * race and must be serialised by the caller. */
int pms_solve_device_noalloc(const uint8_t* chars, int32_t n, int32_t m, const char* alphabet,
                             int32_t l, int32_t d, uint64_t* keys_out, int64_t keys_cap,
                             int64_t* count_out, void* hip_stream);
/* Size of that scratch array in bytes (host-only). */
size_t pms_noalloc_scratch_bytes(void);

/* Appendix D cost-model threshold the library uses when tune.threshold is 0
 * (a stack size in [2, 8]) for an alphabet of sigma letters (sigma < 2 is
 * taken as 4); host-only. */
int pms_default_threshold(int n, int m, int l, int d, int sigma);
/* Appendix C expected number of motifs of a random instance (n strings of
 * length m, i.i.d. uniform letters of an alphabet of sigma, sigma < 2 taken
 * as 4): sigma^l (1 - (1 - N_d / sigma^l)^(m-l+1))^n with
 * N_d = sum_{i<=d} C(l,i) (sigma-1)^i; host-only.  Sizes the output slots
 * when tune.out_capacity is 0. */
double pms_expected_motifs(int n, int m, int l, int d, int sigma);

/* Number of visible GPUs (0 when none; never an error for "no device"). */
int pms_device_count(int32_t* count);
/* Wait for all work the process enqueued on the current device. */
int pms_device_synchronize(void);

void pms_result_free(pms_result* r);
const char* pms_strerror(int status);
/* Library version string. */
const char* pms_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PMS_H */
