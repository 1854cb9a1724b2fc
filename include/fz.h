/*
 * fz.h -- libfz: bounded lexicographic enumeration of factorization sets on
 * AMD Instinct MI355X (gfx950).
 *
 * The factorization set of an element n with respect to generators g_1..g_d
 * (paper Sec. 1) is
 *
 *     Z(n, g) = { (a_1, ..., a_d) in N^d : a_1 g_1 + ... + a_d g_d = n }.
 *
 * Generators may come in any order and may repeat (footnote to Sec. 1).  The
 * caller's order fixes the lexicographic order of every output, and two equal
 * generators are two distinct coordinates.
 *
 * Every call enumerates Z on the GPU.  The lex-ordered set is cut into
 * disjoint bounded slices (Sec. 4); wavefronts walk their slices with the
 * successor of Alg. 3.1 and its modulo skip (Sec. 3.2.4) and feed one
 * consumer (Sec. 2): a counter, a length histogram, a predicate or a store.
 * Slice bounds come from ranks: the set is counted by a dynamic-programming
 * table on the device and each bound is the element of a chosen rank.
 *
 * Conventions shared by every entry point
 *   n, g, d   the element, a HOST pointer to d generators (read during the
 *             call only, never retained), and the dimension.
 *   limits    1 <= d <= FZ_MAX_D; every g_i >= 1; n < 2^31 and
 *             n + 2 max_i g_i < 2^31 (for d = 1 also n + 2 (n + 1) < 2^31);
 *             n < 2^30 when d <= 2;
 *             g_d <= FZ_MAX_LAST_GEN.  Breaking one
 *             returns FZ_EINVAL (d, g, NULL pointers) or FZ_EOVERFLOW (sizes)
 *             or FZ_E2BIG (g_d), and no output is written.
 *   counts    exact unsigned 64-bit; a set with 2^64 - 1 or more elements
 *             is FZ_EOVERFLOW.
 *   errors    a negative status; no output argument is written unless the
 *             entry point says otherwise.  FZ_EDEVICE: a HIP call failed (no
 *             GPU, launch failure).  FZ_EINTERNAL: the per-slice element
 *             counts disagreed with the ranks of the slice bounds (a
 *             self-check that never fires on a correct build).
 *   device    the current HIP device of the calling thread.  Calls are
 *             synchronous and thread-safe: they are serialized per process.
 *   memory    device scratch (count tables, slice bounds, per-workgroup
 *             partial results) belongs to the library, which keeps it cached
 *             between calls and frees it at process exit.
 *   empty Z   is not an error: count 0, no rows, found 0.
 *   n = 0     Z holds exactly one element, (0, ..., 0), of length 0.
 */
#ifndef FZ_H
#define FZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FZ_MAX_D 16
#define FZ_MAX_LAST_GEN (1u << 24)

typedef enum {
    FZ_OK = 0,
    FZ_TRUNCATED = 1,   /* fz_enumerate*: fewer rows than |Z| were asked for */
    FZ_EINVAL = -1,
    FZ_EOVERFLOW = -2,
    FZ_ENOMEM = -3,
    FZ_EDEVICE = -4,
    FZ_E2BIG = -5,
    FZ_EINTERNAL = -6
} fz_status;

/* |Z(n, g)| into *count.  Each element is visited by the successor and
 * counted (Sec. 2, the counting consumer). */
int fz_count(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count);

/* Number of bins a length histogram of Z(n, g) needs: n / min_i g_i + 1
 * (every element has length sum_i a_i <= n / min g).  0 for invalid input. */
uint64_t fz_length_bins(uint64_t n, const uint32_t *g, uint32_t d);

/* Length histogram: bins[l] = #{a in Z : a_1 + ... + a_d = l} for
 * l < nbins (host array of nbins words, nbins >= fz_length_bins(...), else
 * FZ_EINVAL).  *min_len / *max_len: the shortest and longest length that
 * occurs (UINT64_MAX and 0 when Z is empty).  The set of lengths of an
 * element is the classic "length set" of numerical semigroups; this consumer
 * is not in the paper, whose Sec. 2 names counters, predicates and stores. */
int fz_length_hist(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *bins,
                   uint64_t nbins, uint64_t *min_len, uint64_t *max_len);

/* Predicate consumer (Sec. 2): *found = 1 if some a in Z has length
 * a_1 + ... + a_d == target_len, else 0.  Workers stop early once one
 * wavefront has found a witness. */
int fz_exists(uint64_t n, const uint32_t *g, uint32_t d, uint64_t target_len,
              int *found);

/* Store consumer (Sec. 2): the min(|Z|, max_tuples) lex-smallest elements of
 * Z in ascending lexicographic order (the reverse of the paper's descending
 * walk, Sec. 3.2), row-major into the HOST buffer out[max_tuples][d] (uint32
 * coordinates).  *total = |Z|, *written = rows written.  Returns FZ_OK, or
 * FZ_TRUNCATED when max_tuples < |Z| (a success: the rows are valid). */
int fz_enumerate(uint64_t n, const uint32_t *g, uint32_t d, uint32_t *out,
                 uint64_t max_tuples, uint64_t *total, uint64_t *written);

/* As fz_enumerate, but d_out is a DEVICE pointer (for instance the data of a
 * torch tensor) on the current device, and the work is queued on `stream`
 * (a hipStream_t; NULL for the library's own stream).  The call waits for
 * that stream before it returns *total and *written. */
int fz_enumerate_device(uint64_t n, const uint32_t *g, uint32_t d,
                        uint32_t *d_out, uint64_t max_tuples, uint64_t *total,
                        uint64_t *written, void *stream);

/* As fz_count, queued on `stream` (a hipStream_t, NULL: the library's own);
 * waits for it before returning. */
int fz_count_stream(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count,
                    void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the count
 * of fz_count_stream, by the same kernels, with no hipMalloc, hipFree or
 * other allocation.  Every device buffer of the query (count and work tables,
 * residue table, slice bounds and records, control block) is a piece of one
 * fixed array of FZ_NOALLOC_SCRATCH_BYTES bytes inside the library, which
 * each GPU holds from the first call on it until the process ends.  A query
 * that needs more (about (2d - 3)(n + 1) 8 bytes of tables plus ~9 MB of
 * slice data on MI355X) is refused with FZ_E2BIG (fz_last_error says how
 * much it needed), before any device work.  The work is queued on `stream`
 * (a hipStream_t; NULL: the device's null stream) and the call waits for it.
 * Calls are serialized per process and each waits for its stream, so two
 * calls never use the array at once; the array keeps the last call's
 * contents, which the next call overwrites before reading.  Other errors as
 * fz_count. */
#define FZ_NOALLOC_SCRATCH_BYTES (64u << 20)
int fz_count_noalloc(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count,
                     void *stream);

/* The slice-bound primitive (Sec. 4, bounds; done here by ranks): for each
 * of the nranks ranks (0-based, host array), the element of that rank in
 * ascending lex order, row-major into the HOST buffer out[nranks][d].  A
 * rank >= |Z| gives FZ_EINVAL and writes nothing. */
int fz_unrank(uint64_t n, const uint32_t *g, uint32_t d, const uint64_t *ranks,
              uint64_t nranks, uint32_t *out);

/* ------------------------------------------------------------------------
 * Batches: many queries (any d, n and consumer) enumerated by one persistent
 * launch.  Large queries are cut into slices of equal work by their count
 * tables; small ones are one slice each; all slices of all queries go to one
 * work queue, so wavefronts that finish one query's slice take the next
 * slice of any query.
 * ------------------------------------------------------------------------ */
typedef enum {
    FZ_MODE_COUNT = 0,  /* |Z|                                  (fz_count) */
    FZ_MODE_HIST = 1,   /* length histogram              (fz_length_hist) */
    FZ_MODE_EXISTS = 2, /* an element of length target_len?   (fz_exists) */
    FZ_MODE_STORE = 3   /* lex-smallest rows to a device buffer
                           (fz_enumerate_device) */
} fz_mode;

typedef struct {
    uint64_t n;
    const uint32_t *g;     /* HOST pointer to d generators */
    uint32_t d;
    uint32_t mode;         /* fz_mode */
    uint64_t target_len;   /* FZ_MODE_EXISTS */
    uint64_t *bins;        /* FZ_MODE_HIST: HOST array of nbins words */
    uint64_t nbins;        /*   >= fz_length_bins(n, g, d) */
    uint32_t *d_out;       /* FZ_MODE_STORE: DEVICE buffer of max_tuples rows */
    uint64_t max_tuples;
} fz_query;

typedef struct {
    int status;            /* FZ_OK, FZ_TRUNCATED (store) or a negative error */
    int found;             /* FZ_MODE_EXISTS */
    uint64_t count;        /* elements visited (|Z| unless exists stopped early) */
    uint64_t total;        /* |Z| from the count table, when the query was cut
                              by it (every store query), else equal to count */
    uint64_t min_len;      /* FZ_MODE_HIST (UINT64_MAX when Z is empty) */
    uint64_t max_len;      /* FZ_MODE_HIST (0 when Z is empty) */
    uint64_t written;      /* FZ_MODE_STORE rows written */
} fz_result;

/* Runs nq queries as one batch on `stream` (a hipStream_t, NULL: the
 * library's own) and waits for it.  Returns FZ_OK when the batch ran; each
 * query's own outcome (including validation errors, which do not stop the
 * others) is r[i].status.  q and r are HOST arrays of nq entries; FZ_EINVAL
 * for NULL arrays. */
int fz_batch(const fz_query *q, fz_result *r, uint32_t nq, void *stream);

/* ------------------------------------------------------------------------
 * Serving.  A server takes queries one at a time from any thread
 * (fz_submit) and hands each result to fz_wait.  Its own thread keeps up to
 * max_inflight batches on the device, each on its own stream: whatever has
 * arrived is launched as one batch as soon as a launch slot is free, so
 * queries that arrive while others run start without waiting for them, and
 * the batches overlap on the GPU.  A query's result is ready as soon as its
 * own last slice is done, whatever the rest of its batch is doing.
 * Admission: a query whose count/work tables, residue table and bins would
 * exceed mem_budget, or a store query whose count table says |Z| >
 * max_store_tuples, finishes with FZ_E2BIG (a refused store query reports
 * |Z| in total).  Results are the same as alone (fz_batch, or the
 * single-query entry points).
 * The server uses the device current at fz_server_create.  fz_submit copies
 * q and its generators; q->bins (host) and q->d_out (device) must stay valid
 * until fz_wait has returned that ticket's result.  Every ticket must be
 * collected with fz_wait exactly once; FZ_EINVAL for an unknown ticket.
 * fz_server_destroy finishes the queries already submitted, then frees the
 * server (results not yet collected are dropped).
 * ------------------------------------------------------------------------ */
typedef struct {
    uint32_t max_inflight;     /* launch slots (streams), 1..8; 0: 2 */
    uint32_t max_batch;        /* queries per launch, 1..65536; 0: 4096 */
    uint64_t mem_budget;       /* device bytes of tables per launch; 0: 8 GiB */
    uint64_t max_store_tuples; /* admission cap of a store query; 0: 10^7 */
} fz_server_cfg;

typedef struct fz_server fz_server;

typedef struct {
    uint64_t submitted, completed, launches;
    double mean_batch;         /* queries per launch */
    double p50_us, p99_us, max_us, mean_us; /* fz_submit to result ready */
    double mean_phase1_us;     /* per launch: admission to the walk's launch
                                  (tables, their totals read back, the cut) */
    double mean_phase2_us;     /* per launch: the walk's launch to its last result */
} fz_server_stats;

int fz_server_create(const fz_server_cfg *cfg, fz_server **out); /* cfg may be NULL */
int fz_submit(fz_server *s, const fz_query *q, uint64_t *ticket);
int fz_wait(fz_server *s, uint64_t ticket, fz_result *r); /* blocks */
int fz_server_stats_read(fz_server *s, fz_server_stats *out, int reset);
int fz_server_destroy(fz_server *s);

/* Work statistics of the last successful enumeration on this device:
 * slices used, rows walked (one row = one prefix a_1..a_{d-3}), prefixes
 * (a_1..a_{d-2}) visited by lanes, candidate steps taken (one per element
 * visited plus one failing test per prefix), and elements.  After fz_batch
 * the slices are the batch's work items, and the other figures are summed
 * over them only while profiling is on (fz_profile_enable), else 0. */
typedef struct {
    uint64_t slices;
    uint64_t rows;
    uint64_t prefixes;
    uint64_t candidates;
    uint64_t elements;
} fz_stats;
int fz_last_stats(fz_stats *out);

/* Per-slice record of the last successful enumeration on this device: the
 * elements, rows and lane prefixes a_1..a_{d-2} of each slice and the device
 * wall clock (100 MHz ticks)
 * when a wavefront took it and finished it; for judging the balance of the
 * slice cut.  After fz_batch, the records are the batch's work items, in
 * the order of its work queue.  Copies min(cap, slices)
 * records, *n_slices = slices. */
typedef struct {
    uint64_t elements;
    uint64_t rows;
    uint64_t prefixes;
    uint64_t t_begin;
    uint64_t t_end;
    uint32_t query;     /* fz_batch: index of the query the slice belongs to */
    uint32_t slice;     /* fz_batch: slice index within that query */
} fz_slice_info;
int fz_last_slices(fz_slice_info *out, uint32_t cap, uint32_t *n_slices);

/* Tuning knobs (0 restores the default): "slices_per_wave" (slices cut per
 * resident wavefront; default 16 for a single query, 8 for a batch),
 * "workgroups_per_cu" (persistent workgroups per compute unit; default 8, 4
 * for a batch), "work_row", "work_chunk", "work_element" (weights, in 1/64 of a
 * wavefront instruction, of a row a_1..a_{d-3}, of a 64-lane chunk of a row
 * and of an element, when slices are cut to equal work), "skip_empty_rows"
 * (0: for sets with few elements per row, skip rows and subtrees that the
 * count table shows empty; 1: always; 2: never), "walk_order" (0: count,
 * histogram and predicate walk the set with the generators in descending
 * order, which visits the fewest rows; 1: in the caller's order; stores
 * always use the caller's order, their output order), "batch_graph" (1:
 * fz_batch and the server queue a batch's slice bounds and walker as one
 * HIP graph, updated in place from batch to batch; 0: plain launches; with
 * profiling on, batches use plain launches), "pair_table" (single queries
 * with d >= 4: 0: when the last pair represents few remainders, about
 * n D / (2 A B) < 1/4, rows walk only the remainders it represents, listed
 * per residue chain from the count table, and skip empty rows too; 1:
 * always; 2: never; batches never use it), "min_slice_work" (single
 * queries: a query whose whole modelled work is small is cut into fewer
 * slices, each carrying at least this much work, so that it occupies a few
 * wavefronts briefly; default 65536, about a thousand wavefront
 * instructions; 1: always the full slice count), "variant" (0: the plain
 * walk; 1: count, histogram and predicate of a query with d >= 4 that is
 * walked without row skipping or pair table also skip, by the common divisor
 * of the last two and of the last three generators (Sec. 3.2.4), the lane
 * prefixes and rows that cannot hold an element, and count a lane's run of
 * elements in closed form), "tables" (count, histogram and predicate of a
 * single query: 0: build the count and work tables unless they would take
 * more than 64 GiB; 1: always; 2: never.  Without tables the slices are cut
 * by splitWork (Sec. 4) from the set's lexicographic range, halving each
 * range where its estimated number of elements is split in two),
 * "host_threads" (hybrid pool, Sec. 6.3: count, histogram and predicate of
 * a single query with tables: that many host threads, 0..64, walk the last
 * slices of the work while the device walks the others; 0: off) and
 * "host_share_ppm" (their share of the modelled work in millionths, up to
 * 500000; 0: 3 per thread, about a host thread's rate against the device's),
 * "trailing" (Sec. 6.1, dynamic behavior: 1: count and store of a single
 * query with d >= 4 walked without row skipping or pair table take each full
 * row's elements Z(R, (g_{d-2}, g_{d-1}, g_d)) at once -- the count from the
 * count table, the store by copying them from a table of every Z(x) up to
 * the largest x whose elements fit in 2 GiB; 0: off), "packed" (count,
 * histogram and predicate: the lane prefixes of up to 64 consecutive rows
 * of the deepest row level are walked end to end, 64 at a time; 0: for
 * sparse sets that skip empty rows, 1: always, 2: never; the batch walker
 * walks every order-free consumer packed), "empty_row_test" (single queries
 * with d >= 4 and tables, walked without row skipping, pair table or
 * packing: 0 or 1, the default: the rows of each block of up to 64 rows of
 * the deepest row level are tested against the count table, and a row with
 * no completion is not walked; 2: never), "batch_min_item_work" (the least
 * modelled work of a batch's work item, so that a small batch is not cut
 * into a chip's worth of tiny items; up to 2^30; 0: 2^20 units),
 * "wave_bins32" (single-query histograms of up to ~680 bins: 1, the default:
 * each wave adds its runs to 32-bit bins of its own in LDS, folded into the
 * workgroup's 64-bit bins before they could overflow; 0: all waves add to the
 * workgroup's 64-bit bins), "wave_bins32_limit" (the elements a wave's
 * 32-bit bins may hold before they are folded, at most 2^20 here; 0: 2^31;
 * small values exercise the folding), "wave_bins32_copies" (interleaved
 * copies of each wave's 32-bit bins, lane l adding to copy l mod copies, so
 * that lanes whose runs start in the same bin are served by different LDS
 * banks: 0, the default: 4, else 2, else 1, while 8 workgroups per CU (or
 * the "workgroups_per_cu" value) still fit the CU's 160 KiB of LDS; 1, 2 or
 * 4: that many, as far as a workgroup's 64 KiB allow), "short_last_slices"
 * (count, histogram and predicate of a single query cut into 64 or more
 * slices without host threads: 0 or 1, the default: the last quarter of the
 * slices carries a quarter of the modelled work of each of the others, so
 * that the slices still walked after the last one was taken are short; 2:
 * equal slices).
 * FZ_EINVAL for an
 * unknown key or a value outside its range (0..2^20 for the sizes and
 * weights).  Results never depend on the knobs. */
int fz_config_set(const char *key, int64_t value);

/* Autotuner.  Runs the given queries (one fz_batch call when nq > 1, else the
 * single-query entry point of the query's mode) under every candidate pair of
 * slices per wave {4, 8, 16, 32, 64} x workgroups per CU {2, 4, 8}, reps
 * timed runs each after one warm-up, and keeps the pair with the smallest
 * median wall time as this process's configuration (as fz_config_set would).
 * The queries' own buffers (bins, store destinations) are overwritten; their
 * results are not reported.  FZ_EINVAL: NULL q or out, nq == 0, reps outside
 * 1..100; a failing run returns its status and restores the previous knobs. */
typedef struct {
    uint32_t slices_per_wave;
    uint32_t workgroups_per_cu;
    double ms;          /* median wall time of the chosen pair */
    double default_ms;  /* median wall time with the defaults */
    uint32_t candidates; /* pairs timed */
} fz_tune_result;
int fz_autotune(const fz_query *q, uint32_t nq, uint32_t reps, fz_tune_result *out);

/* Kernel timing with HIP events on the launch stream.  fz_profile_enable(1)
 * starts recording (it adds no synchronization of its own); fz_profile_read
 * gives the summed milliseconds and launch count of one kernel ("dp",
 * "restab", "slices", "enum.count", "enum.hist", "enum.exists", "enum.store",
 * "finalize", "unrank"; for fz_batch "batch.tables" (count and work tables,
 * residue tables), "batch.slices" (slice bounds), "batch.walk") since the
 * last reset. */
int fz_profile_enable(int on);
int fz_profile_reset(void);
int fz_profile_read(const char *kernel, double *total_ms, uint64_t *launches);

/* The HIP call that produced this thread's last FZ_EDEVICE / FZ_ENOMEM, with
 * the HIP error text ("" if none).  The string is owned by the library and
 * stays valid until the thread's next failing call. */
const char *fz_last_error(void);

/* Diagnostic: the current device's sustained int32 vector-ALU rate, in lane
 * operations per second (*lane_ops_per_s), from a kernel in which every lane
 * runs eight independent chains of 32-bit adds; *ms (may be NULL) is the
 * kernel's best time of three.  The ceiling that the count walker's
 * integer-op rate is compared with.  Takes ~0.1 s; FZ_EINVAL for a NULL
 * rate, FZ_EDEVICE / FZ_ENOMEM on HIP errors. */
int fz_probe_int_valu(double *lane_ops_per_s, double *ms);

/* Diagnostic: the current device's sustained HBM write rate in bytes per
 * second (*bytes_per_s): a kernel writes a fresh device buffer of `bytes`
 * (at least 1 MiB; rounded down to 16 B) with 16-byte stores in a
 * grid-stride loop, reading nothing; *ms (may be NULL) is its best time of
 * three.  The ceiling that the store walker's write rate is compared with.
 * The buffer is allocated and freed by the call.  FZ_EINVAL for a NULL rate
 * or fewer bytes, FZ_ENOMEM / FZ_EDEVICE on HIP errors. */
int fz_probe_hbm_write(uint64_t bytes, double *bytes_per_s, double *ms);

/* Static description of a status code. */
const char *fz_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* FZ_H */
