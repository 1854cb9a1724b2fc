// fz_internal.h -- plan and buffer layout shared by the libfz host engine and
// its HIP kernels.  Not part of the public ABI (include/fz.h is).
//
// Coordinates are 0-based here: the paper's a_1..a_d are a[0..d-1].  Calls
// with d < 3 are padded in front with "virtual" coordinates whose generator
// n+1 exceeds n, so they are always 0; every kernel therefore sees d >= 3 and
// splits a tuple into
//   a[0..M-1]      the row prefix (M = d-3), walked by a wave-uniform
//                  odometer held in scalar registers,
//   a[M]  = x      the lane coordinate: 64 consecutive values per chunk, one
//                  per lane of the wavefront,
//   a[d-2], a[d-1] the last pair, solved per lane: the valid a[d-2] for a
//                  given remainder form an arithmetic progression with step
//                  ord = g[d-1] / gcd(g[d-2], g[d-1]) (the modulo skip of
//                  Sec. 3.2.4), so a lane steps through exactly the elements.
#pragma once
#include <stdint.h>

#define FZK_MAX_D 16            // effective (padded) dimension bound
#define FZK_SENTINEL 0xFFFFFFFFu
#define FZK_NONE_E (1 << 30)    // residue-table mark: no solution in class
#define FZK_WAVE 64
#define FZK_WG 256              // threads per workgroup of the walker
#define FZK_DP_UNITS 65536      // threads per level of a single query's table scans

enum FzMode { FZM_COUNT = 0, FZM_HIST = 1, FZM_EXISTS = 2, FZM_STORE = 3 };

// Division by an invariant 32-bit divisor (Granlund and Montgomery, "Division
// by invariant integers using multiplication", PLDI 1994, Fig. 4.1):
// t = mulhi(m, x); q = (t + ((x - t) >> s1)) >> s2.  Exact for every x < 2^32.
struct FzFastDiv {
    uint32_t m, s1, s2, d;
};

struct FzPlan {
    uint32_t n;
    uint32_t d;          // effective dimension, >= 3
    uint32_t d_user;     // the caller's d
    uint32_t pad;        // d - d_user virtual leading coordinates
    uint32_t g[FZK_MAX_D];
    uint32_t G2;         // g[d-3], generator of the lane coordinate
    uint32_t A, B;       // g[d-2], g[d-1]
    uint32_t D;          // gcd(A, B)
    uint32_t ord;        // B / D: step of a[d-2] between elements
    uint32_t delta;      // A / D: matching decrease of a[d-1]
    uint32_t inv;        // (A/D)^{-1} mod ord
    uint32_t mode;
    FzFastDiv div_B, div_delta, div_G2;
    uint32_t w_row;      // slice-cut weight of one row (prefix a[0..M-1])
    uint32_t w_chunk;    // ... of one 64-lane chunk of a row
    uint32_t w_el;       // ... of one element
    uint32_t restab_in_lds;
    uint32_t nbins;      // histogram bins (n / min g + 1)
    uint32_t hist_in_lds; // histogram bins: 0 global; a batch: 1 per-wave LDS 64-bit, 2 per-wave
                          // LDS 32-bit; a single query: 1 the workgroup's LDS 64-bit set, 2 that
                          // set and a 32-bit set per wave
    uint32_t prune;      // skip rows whose subtree is empty (sparse sets; needs S)
    uint32_t pair;       // walk only the pair remainders the last pair represents (pair table)
    uint32_t w_skip;     // slice-cut weight of a skipped (empty) row
    uint32_t n_slices;   // W
    uint32_t stride;     // n + 1: row length of the count table
    uint64_t target_len; // predicate target
    uint64_t max_tuples; // store limit; UINT64_MAX for the other consumers
    uint64_t min_slice_work; // single query: least modelled work of a slice (0: always W)
    // The variant walk (cdv = 1): the common-divisor skip of the last two and
    // three generators (Sec. 3.2.4) and closed-form run lengths.  A lane
    // coordinate x can have an element only when x G2 = R (mod D), D =
    // gcd(A, B): e2 = gcd(G2, D) must divide R, and then x = ((R mod D) / e2)
    // inv2 (mod sx), sx = D / e2.  Likewise the rows of the deepest row level
    // with D3 = gcd(G2, A, B) = e2: e3 = gcd(g[d-4], D3), sy = D3 / e3.
    uint32_t cdv;
    uint32_t cd_sx, cd_e2, cd_inv2;
    uint32_t cd_D3, cd_sy, cd_e3, cd_inv3;
    // divisions by D, e2 and sx (the packed walk's lane stride too), D3, e3
    // and sy; sx, sy < 2^16, so the residue products fit 32 bits
    FzFastDiv div_D, div_e2, div_sx, div_D3, div_e3, div_sy;
    // Table-free walk (notab = 1; count, histogram and predicate only): no
    // count or work table; the W slices are cut by repeated splitWork
    // (Sec. 4, Alg. 4.1) from the whole set, and no slice is checked
    // against ranks.
    uint32_t notab;
    // Hybrid pool (host_slices = T > 0; count, histogram and predicate of a
    // single query with tables): slices W..W+T-1 cover the last host_ppm
    // millionths of the modelled work and are walked by T host threads while
    // the device walks slices 0..W-1 (n_slices = W).
    uint32_t host_slices;
    uint32_t host_ppm;
    // Trailing-index tables (Sec. 6.1, knob "trailing"): a full row whose
    // remainder R is below ctl->trail_m takes its elements from Z(R, (G2,
    // A, B)) at once -- the count table's row M for the count, a table of
    // the triples (a_{d-2}, a_{d-1}, a_d) of every Z(x), x <= trail_m, for
    // the store (at most trail_cap triples).
    uint32_t trail;
    uint64_t trail_cap;
    // Packed walk of short rows (pack = 1; count, histogram and predicate,
    // d >= 4): the lane prefixes of up to 64 consecutive rows of the deepest
    // row level fill the chunks end to end.
    uint32_t pack;
    // Block walk with tables (rowtest = 1): the rows of a block whose
    // remainder has no completion in the count table (S[M][R] = 0) are
    // dropped before the block is walked.
    uint32_t rowtest;
    // Single-query histograms with a 32-bit set of bins per wave: a wave
    // folds its set into the workgroup's before it holds this many elements
    // (at most 2^31), and walks a slice of at least this many elements into
    // the workgroup's set directly.
    uint64_t hist32_limit;
    // ... and 2^hist32_copies interleaved copies of each wave's 32-bit set:
    // lane l adds to copy l mod 2^hist32_copies, word bin * 2^hist32_copies
    // + copy, so lanes whose runs start in the same bin use different banks.
    uint32_t hist32_copies;
    // Single-query slice cut: the last quarter of the slices is cut a
    // quarter of the size of the others (guided = 1).
    uint32_t guided;
};

// Control block in device memory.  The slice cursor and the early-exit flag
// sit on their own 128-byte lines.
struct FzCtl {
    uint32_t cursor;
    uint32_t pad0[31];
    uint32_t found;
    uint32_t pad1[31];
    uint32_t status;     // FZS_* bits
    uint32_t slices;     // slices cut: W, or fewer for a small query
    uint64_t trail_m;    // trailing tables: rows with remainder < trail_m take them
    uint64_t total;      // |Z| from the count table
    uint64_t count;      // elements the walkers visited
    uint64_t rows, prefixes;
    uint64_t min_len, max_len;
    uint64_t written;
};

enum { FZS_OVERFLOW = 1u, FZS_MISMATCH = 2u, FZS_TOOBIG = 4u };

// Per-slice record written by the walker (one wave per slice).
struct FzSliceRec {
    uint64_t elements;
    uint64_t rows;
    uint64_t prefixes;   // lane prefixes a[0..M] visited
    uint64_t t_begin;    // device wall clock (100 MHz) when the wave took it
    uint64_t t_end;
};

struct FzBufs {
    uint64_t *S;          // count table: rows k = 0..d-2, each n+1 words
    uint64_t *C;          // work table: rows k = 0..M, each n+1 words
    int2 *restab;         // 2B entries {t0, E2}, indexed by rho' = rho + B - lr
    uint32_t *bounds;     // (W+1) x (d-2) slice start prefixes a[0..M]
    uint64_t *base;       // (W+1) rank of the first element of each slice
    FzSliceRec *recs;     // W
    FzCtl *ctl;
    uint64_t *hist_rows;  // nwg x nbins partial histograms
    uint64_t *hist;       // nbins final histogram
    uint32_t *out;        // store destination (row-major [.][d_user])
    uint64_t *PC;         // pair table (P.pair): n+1 chain prefix counts
    uint32_t *PE;         //   up to n+1 representable remainders
    uint32_t *PO;         //   min(G2, n+1) + 1 chain starts
    uint64_t *dpart;      // FZK_DP_UNITS block sums of the table scans
    uint64_t *TO;         // trailing tables: TO[x] = first triple of Z(x) in TT, x <= n + 1
    uint32_t *TT;         //   the triples, 3 words each
};

// ---------------------------------------------------------------------------
// Batches: many queries walked by one persistent launch.  Each query has a
// plan and the offsets of its device data; its work is cut into W_q slices
// (W_q = 1 for queries too small to be worth a count table: their one slice
// runs from the prefix (0,...,0) to the end of the set).
// ---------------------------------------------------------------------------
struct FzBatchQuery {
    FzPlan plan;
    uint64_t s_off;       // count table (rows 0..d-2), when sliced
    uint64_t c_off;       // work table (rows 0..M), when sliced
    uint64_t tab_off;     // residue table (2B int2)
    uint64_t bins_off;    // histogram bins (nbins u64), hist queries
    uint32_t *out;        // store destination (device), store queries
    uint64_t max_total;   // a store query with |Z| above this is refused (FZS_TOOBIG)
    uint32_t sliced;      // 1: count/work tables and W_q rank-cut slices
    uint32_t n_slices;    // W_q
    uint32_t bound_off;   // first boundary of this query in the bounds array
    uint32_t item_off;    // first walker item of this query
};

// Per-query result in device memory.  The walkers add their items' counts;
// the wave that completes a query's last item (items_done) finishes it.
struct FzBatchResult {
    uint64_t count;       // elements the walkers visited
    uint64_t total;       // |Z| from the count table (sliced queries)
    uint64_t min_len, max_len;
    uint64_t written;
    uint32_t found;
    uint32_t status;      // FZS_* bits
    uint32_t items_done;
    uint32_t pad;
};

// A boundary job of the batch slice kernel / a walker work item.
struct FzBatchJob {
    uint32_t q;           // query index
    uint32_t j;           // slice index within the query (boundary j for jobs)
};

struct FzBatchBufs {
    const FzBatchQuery *queries;
    const FzBatchJob *bjobs;   // boundary jobs: sum over queries of (W_q + 1)
    const FzBatchJob *items;   // walker items: sum over queries of W_q
    uint64_t *tables;          // count and work tables of sliced queries
    int2 *restabs;             // residue tables
    uint32_t *bounds;          // boundaries, stride bstride words
    uint64_t *base;            // element rank of each boundary
    FzSliceRec *recs;          // per item
    uint64_t *bins;            // histogram bins of hist queries
    FzBatchResult *res;        // per query
    uint64_t *totals;          // C[0][n], S[0][n] of each query with tables (ids order)
    uint32_t *cursor;          // walker item cursor (own 128-byte line)
    // optional host-visible copies (pinned, coherent): a finished query's
    // result and bins are written there and host_done[q] is set to 1 with a
    // system-scope release, so the host can collect it while the launch runs
    FzBatchResult *host_res;
    uint64_t *host_bins;
    uint32_t *host_done;
    uint32_t nq, n_bjobs, n_items, bstride;
    uint64_t n_bins;           // words of the histogram buffer
};

// Launchers (fz_kernels.hip).
#include <hip/hip_runtime.h>
hipError_t fzk_launch_dp(const FzPlan &p, const FzBufs &b, hipStream_t s);
hipError_t fzk_launch_restab(const FzPlan &p, const FzBufs &b, hipStream_t s);
hipError_t fzk_launch_slices(const FzPlan &p, const FzBufs &b, hipStream_t s);
hipError_t fzk_launch_split(const FzPlan &p, const FzBufs &b, hipStream_t s);
hipError_t fzk_launch_trail(const FzPlan &p, const FzBufs &b, hipStream_t s);
hipError_t fzk_launch_enum(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s);
hipError_t fzk_launch_finalize(const FzPlan &p, const FzBufs &b, uint32_t nwg, hipStream_t s);
hipError_t fzk_launch_unrank(const FzPlan &p, const FzBufs &b, const uint64_t *ranks,
                             uint64_t nranks, uint32_t *out, hipStream_t s);
size_t fzk_enum_lds_bytes(const FzPlan &p);
// batch: zeroing, count / work tables (and their totals) and residue tables;
// then, once the host has cut the queries, slice bounds; then the persistent
// walker, which also finishes each query
// Tables of a batch: one workgroup builds all rows of each of the n_small
// queries small_ids (device array); then pass p = 0 .. n_pass-1 launches the
// jobs (query, group, groups) pass_jobs[3 pass_off[p] ..) (device array;
// pass_off on the host, n_pass + 1 entries): one row computation of each
// larger query, its rows shared by several workgroups; then the totals of
// all n_tabled queries tabled_ids.
hipError_t fzk_launch_batch_tables(const FzBatchBufs &b, uint32_t n_tabled,
                                   const uint32_t *tabled_ids, uint32_t n_small,
                                   const uint32_t *small_ids, const uint32_t *pass_jobs,
                                   const uint32_t *pass_off, uint32_t n_pass, hipStream_t s);
hipError_t fzk_launch_batch_slices(const FzBatchBufs &b, hipStream_t s);
hipError_t fzk_launch_batch_walk(const FzBatchBufs &b, uint32_t maxm, uint32_t nwg,
                                 uint32_t lds_bins, uint32_t max_du, hipStream_t s);
