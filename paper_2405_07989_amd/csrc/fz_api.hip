// fz_api.hip -- libfz host engine: validation and normalization of a query,
// planning, device scratch, kernel launches and the C ABI of include/fz.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fz.h"
#include "fz_host.h"
#include "fz_internal.h"

namespace fzh {

constexpr int kMaxDevices = 64;
constexpr uint32_t kDefaultSlicesPerWave = 16;
constexpr uint32_t kDefaultWgPerCu = 8;
constexpr uint32_t kBatchSlicesPerWave = 8; // batches and the server
constexpr uint32_t kBatchWgPerCu = 4;
constexpr uint32_t kMaxSlices = 1u << 22;
// Least modelled work of a single query's slice (1/64 wave instructions):
// about a thousand wave instructions, a few microseconds.
constexpr uint64_t kMinSliceWork = 1u << 16;
// Count and work tables of a single order-free query above this size are not
// built: its slices are cut by splitWork instead (the table-free walk).
constexpr uint64_t kTableBudget = 64ull << 30;
// Hybrid pool: a host thread walks about 1e7 elements per second against
// ~3e12 on MI355X, so each thread takes about 3 millionths of the work.
constexpr uint32_t kHostPpmPerThread = 3;
constexpr uint32_t kMaxHostThreads = 64;
// Trailing-index tables of a store: at most 2 GiB of triples.
constexpr uint64_t kTrailBytes = 2ull << 30;
constexpr size_t kLdsHistBudget = 64 * 1024;
// ... and for the workgroup's set with a 32-bit set per wave beside it.
constexpr size_t kLdsHist32Budget = 16 * 1024;
// LDS of a compute unit, shared by its resident workgroups; one workgroup
// may take at most 64 KiB
constexpr size_t kLdsPerCu = 160 * 1024;
constexpr size_t kLdsPerWg = 64 * 1024;
constexpr size_t kLdsRestabBudget = 16 * 1024; // keeps 8 workgroups per CU
// per-wave LDS histogram in batches, 8 KB per wave: 1024 64-bit bins, or
// 2048 32-bit bins for a histogram that needs more
constexpr uint32_t kBatchLdsBins = 2048;
// Work model of the walker for cutting slices, in 1/64 of a wave instruction
// (measured on the compiled walker): a row costs about 50 instructions (the
// odometer step and the row bounds), a 64-lane chunk about 23 plus one trip
// of the element loop (7 instructions, two candidate steps) per two units of
// the spread of progression lengths across its lanes, and an element about
// 3.5/64 (its share of a trip) when counted, more when binned or stored.
constexpr double kWorkRow = 50.0 * 64;
constexpr double kWorkChunk = 23.0 * 64;
constexpr double kWorkTrip = 7.0 * 64;
constexpr double kWorkElem[4] = {4, 8, 5, 40}; // count, hist, exists, store
// A skipped row costs about 1/2 instruction: 64 siblings per ballot scan.
constexpr uint32_t kWorkSkip = 32;
// Rows are skipped when the set has fewer elements than this per row.
constexpr double kPruneElementsPerRow = 0.5;
// The pair table is used when fewer pair remainders than this are representable.
constexpr double kPairMaxFraction = 0.25;
// Short rows are walked packed when a row has fewer lane prefixes than this.
constexpr double kPackPrefixesPerRow = 48.0;

struct Ctx {
    bool ready = false;
    int device = -1;
    int cus = 0;
    hipStream_t stream = nullptr;
    FzCtl *host_ctl = nullptr; // pinned
    DevBuf S, C, restab, bounds, base, recs, ctl, hist_rows, hist, ranks, rows_out, pt, dpart;
    DevBuf trail_o, trail_t; // trailing tables of a store (knob "trailing")
    BatchSlot batch; // fz_batch
    bool last_batch = false; // fz_last_slices reads the batch's items
    fz_stats last{};
    // hybrid pool: the host slices' bounds and base ranks (pinned), the
    // event after their copy, the host part's histogram of the last call
    void *h_hostb = nullptr;
    size_t h_hostb_cap = 0;
    hipEvent_t host_ev = nullptr;
    std::vector<uint64_t> host_hist;
};

std::mutex g_mu;
Ctx g_ctx[kMaxDevices];
uint32_t g_slices_per_wave = 0;
uint32_t g_wg_per_cu = 0;
uint32_t g_work_row = 0;
uint32_t g_work_chunk = 0;
uint32_t g_work_elem = 0;
uint32_t g_prune_mode = 0; // 0: by the set's density, 1: always, 2: never
uint32_t g_walk_order = 0; // 0: descending for order-free consumers, 1: the caller's
uint32_t g_batch_graph = 1; // batch phase 2 as a HIP graph (1) or plain launches (0)
uint32_t g_pair_mode = 0;   // pair table: 0 by sparsity of the last pair, 1 always, 2 never
uint64_t g_min_slice_work = 0; // 0: kMinSliceWork
uint32_t g_variant = 0; // 1: the variant walk (common-divisor skip, closed-form run lengths)
uint32_t g_tables = 0;  // 0: count tables unless above kTableBudget, 1: always, 2: never
uint32_t g_host_threads = 0; // hybrid pool: host worker threads (0: off)
uint32_t g_host_ppm = 0;     // their share of the work in millionths (0: kHostPpmPerThread each)
uint32_t g_trailing = 0;     // 1: trailing-index tables (count and store of the block walk)
uint32_t g_pack_mode = 0;    // packed walk of short rows: 0 by row length, 1 always, 2 never
uint32_t g_row_test = 0;     // block walk drops rows with no completion: 0/1 with tables, 2 never
uint32_t g_hist32_copies = 0; // copies of a wave's 32-bit bins: 0 by LDS room, else 1, 2 or 4
uint32_t g_guided = 0;       // short last slices of a single query: 0/1 on, 2 off
uint64_t g_batch_min_item = 0; // 0: kBatchMinItemWork
uint32_t g_hist32 = 1;         // single-query histograms: 32-bit LDS bins per wave when they fit
uint64_t g_hist32_limit = 0;   // their fold threshold in elements (0: 2^31)

bool worth_pruning(const FzPlan &P);
uint32_t pack_rows(const FzPlan &P);
bool worth_pair(const FzPlan &P);
hipError_t ensure_pinned(void **p, size_t *cap, size_t bytes);
uint64_t pair_words(const FzPlan &P);

struct ProfEntry {
    double ms = 0;
    uint64_t n = 0;
};
bool g_prof = false;
std::map<std::string, ProfEntry> g_prof_stats;
struct PendingEv {
    const char *name;
    hipEvent_t a, b;
};
std::vector<PendingEv> g_pending;

thread_local char g_err_msg[256] = "";

int dev_err_at(hipError_t e, const char *what, int line)
{
    std::snprintf(g_err_msg, sizeof g_err_msg, "%s (line %d): %s (%d)", what, line,
                  hipGetErrorString(e), (int)e);
    if (e == hipErrorOutOfMemory) return FZ_ENOMEM;
    return FZ_EDEVICE;
}

hipError_t ensure(DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (bytes <= b.cap) return hipSuccess;
    if (b.p) {
        hipError_t e = hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (e != hipSuccess) return e;
    }
    size_t want = std::max(bytes, (size_t)4096);
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        b.p = nullptr;
        return e;
    }
    b.cap = want;
    return hipSuccess;
}

#define FZ_TRY(expr)                                                                                \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) {                                                                    \
            (void)hipGetLastError();                                                               \
            return dev_err_at(e_, #expr, __LINE__);                                                \
        }                                                                                          \
    } while (0)

#define FZ_LAUNCH(name, stream, call)                                                              \
    do {                                                                                           \
        hipEvent_t ev_;                                                                            \
        prof_begin(stream, &ev_);                                                                  \
        hipError_t e_ = (call);                                                                    \
        prof_end(stream, name, ev_);                                                               \
        if (e_ != hipSuccess) {                                                                    \
            (void)hipGetLastError();                                                               \
            return dev_err_at(e_, name, __LINE__);                                                 \
        }                                                                                          \
    } while (0)

int get_ctx(Ctx **out)
{
    // Drop an error another library may have left in this thread's HIP
    // state, so that the launch checks below see only this call's errors.
    (void)hipGetLastError();
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return dev_err_at(e == hipSuccess ? hipErrorInvalidDevice : e, "hipGetDevice", __LINE__);
    }
    Ctx &c = g_ctx[dev];
    if (!c.ready) {
        int cus = 0;
        FZ_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        FZ_TRY(hipStreamCreateWithFlags(&c.stream, hipStreamNonBlocking));
        FZ_TRY(hipHostMalloc((void **)&c.host_ctl, sizeof(FzCtl), hipHostMallocDefault));
        c.device = dev;
        c.cus = cus;
        c.ready = true;
    }
    *out = &c;
    return FZ_OK;
}

uint64_t gcd64(uint64_t a, uint64_t b)
{
    while (b) {
        uint64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

// inverse of a modulo m (gcd(a, m) = 1), extended Euclid; 0 when m == 1
uint32_t modinv(uint64_t a, uint64_t m)
{
    if (m == 1) return 0;
    int64_t t = 0, nt = 1;
    int64_t r = (int64_t)m, nr = (int64_t)(a % m);
    while (nr) {
        int64_t q = r / nr;
        int64_t tmp = t - q * nt;
        t = nt;
        nt = tmp;
        tmp = r - q * nr;
        r = nr;
        nr = tmp;
    }
    if (t < 0) t += (int64_t)m;
    return (uint32_t)t;
}

// Granlund-Montgomery (1994) Fig. 4.1 constants for divisor d >= 1.
FzFastDiv make_fastdiv(uint32_t d)
{
    uint32_t l = 0;
    while (l < 32 && (1ull << l) < d) ++l;
    FzFastDiv f;
    f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - d)) / d + 1);
    f.s1 = l < 1 ? l : 1;
    f.s2 = l > 0 ? l - 1 : 0;
    f.d = d;
    return f;
}

// Validation and normalization (all limits of include/fz.h).
int make_plan(uint64_t n, const uint32_t *g, uint32_t d, uint32_t mode, FzPlan *P)
{
    if (g == nullptr || d == 0 || d > FZ_MAX_D) return FZ_EINVAL;
    uint64_t maxg = 0, ming = UINT64_MAX;
    for (uint32_t i = 0; i < d; ++i) {
        if (g[i] == 0) return FZ_EINVAL;
        maxg = std::max<uint64_t>(maxg, g[i]);
        ming = std::min<uint64_t>(ming, g[i]);
    }
    // every coordinate, remainder and walker counter stays a non-negative
    // int32; the virtual generator of d = 1 is n + 1
    // (each term is bounded before the sum, which then cannot wrap)
    if (n >= (1ull << 31)) return FZ_EOVERFLOW;
    const uint64_t maxa = d == 1 ? std::max<uint64_t>(maxg, n + 1) : maxg;
    if (n + 2 * maxa >= (1ull << 31)) return FZ_EOVERFLOW;
    if (d <= 2 && n >= (1ull << 30)) return FZ_EOVERFLOW;
    if (g[d - 1] > FZ_MAX_LAST_GEN) return FZ_E2BIG;
    std::memset(P, 0, sizeof *P);
    P->n = (uint32_t)n;
    P->d_user = d;
    P->pad = d < 3 ? 3 - d : 0;
    P->d = d + P->pad;
    for (uint32_t i = 0; i < P->pad; ++i) P->g[i] = (uint32_t)n + 1; // virtual: always 0
    for (uint32_t i = 0; i < d; ++i) P->g[P->pad + i] = g[i];
    const uint32_t D3 = P->d;
    P->G2 = P->g[D3 - 3];
    P->A = P->g[D3 - 2];
    P->B = P->g[D3 - 1];
    P->D = (uint32_t)gcd64(P->A, P->B);
    P->ord = P->B / P->D;
    P->delta = P->A / P->D;
    P->inv = modinv(P->delta % P->ord, P->ord);
    P->mode = mode;
    P->div_B = make_fastdiv(P->B);
    P->div_delta = make_fastdiv(P->delta);
    P->div_G2 = make_fastdiv(P->G2);
    P->div_D = make_fastdiv(P->D);
    // lanes of a chunk differ by up to 63 G2 in remainder, i.e. by about
    // 63 G2 D / (A B) elements in progression length
    const double spread = 63.0 * P->G2 * P->D / ((double)P->A * P->B);
    const double wchunk = kWorkChunk + kWorkTrip * (std::min(spread, 1e4) / 2 + 1);
    P->w_row = g_work_row ? g_work_row : (uint32_t)kWorkRow;
    P->w_chunk = g_work_chunk ? g_work_chunk : (uint32_t)(wchunk + 0.5);
    P->w_el = g_work_elem ? g_work_elem : (uint32_t)kWorkElem[mode & 3];
    P->restab_in_lds = (size_t)2 * P->B * sizeof(int2) <= kLdsRestabBudget;
    P->prune = 0;
    P->pair = 0;
    P->w_skip = kWorkSkip;
    P->nbins = (uint32_t)(n / ming + 1);
    P->stride = (uint32_t)n + 1;
    P->target_len = 0;
    P->max_tuples = UINT64_MAX;
    return FZ_OK;
}

// Plan of a walk whose result does not depend on the coordinate order
// (count, histogram of lengths, predicate on the length): the same set is
// walked with its generators in descending order, which leaves the fewest
// rows (prefixes of the largest generators) and lane prefixes, and the
// longest progressions (the two smallest generators last).  Validation and
// its errors are those of the caller's order.  Stores keep the caller's
// order: it is their output order.
int make_walk_plan(uint64_t n, const uint32_t *g, uint32_t d, uint32_t mode, FzPlan *P)
{
    int rc = make_plan(n, g, d, mode, P);
    if (rc || mode == FZM_STORE || g_walk_order == 1 || d < 2) return rc;
    uint32_t s[FZ_MAX_D];
    std::memcpy(s, g, d * sizeof(uint32_t));
    for (uint32_t i = 1; i < d; ++i) // descending insertion sort (d <= 16)
        for (uint32_t j = i; j > 0 && s[j - 1] < s[j]; --j) std::swap(s[j - 1], s[j]);
    if (std::equal(s, s + d, g)) return FZ_OK;
    FzPlan Q;
    if (make_plan(n, s, d, mode, &Q)) return FZ_OK; // keep the caller's order
    *P = Q;
    return FZ_OK;
}

void prof_begin(hipStream_t s, hipEvent_t *ev)
{
    *ev = nullptr;
    if (!g_prof) return;
    if (hipEventCreate(ev) != hipSuccess) {
        *ev = nullptr;
        return;
    }
    hipEventRecord(*ev, s);
}

void prof_end(hipStream_t s, const char *name, hipEvent_t a)
{
    if (!g_prof || !a) return;
    hipEvent_t b;
    if (hipEventCreate(&b) != hipSuccess) return;
    hipEventRecord(b, s);
    g_pending.push_back({name, a, b});
}

void prof_collect()
{
    for (auto &p : g_pending) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            auto &e = g_prof_stats[p.name];
            e.ms += ms;
            e.n += 1;
        }
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    g_pending.clear();
}

struct Launch {
    uint32_t nwg;
};

// The variant walk (knob "variant"): order-free consumers of a query walked
// by the block walker (d >= 4, no row skipping, no pair table) skip, besides
// the rows and lane prefixes of the plain walk, every lane coordinate x whose
// remainder the last pair's common divisor D does not divide, and every row
// of the deepest row level whose remainder D3 = gcd(G2, A, B) does not
// divide (Sec. 3.2.4: a common divisor of the last generators), and count a
// lane's run of elements in closed form.  Strides that would leave the
// 31-bit remainders are not taken (the walk is then the same, only slower).
void set_variant(FzPlan &P)
{
    P.cdv = 0;
    if (g_variant != 1 || P.mode == FZM_STORE || P.prune || P.pair || P.d < 4) return;
    const uint64_t D = P.D;
    const uint64_t e2 = gcd64(P.G2, D);
    uint64_t sx = D / e2;
    if (sx >= (1u << 16) || (uint64_t)P.G2 * sx >= (1ull << 31)) sx = 1;
    const uint64_t gy = P.g[P.d - 4];
    const uint64_t D3 = e2;
    const uint64_t e3 = gcd64(gy, D3);
    uint64_t sy = D3 / e3;
    if (sy >= (1u << 16) || gy * sy >= (1ull << 31)) sy = 1;
    P.cd_sx = (uint32_t)sx;
    P.cd_e2 = (uint32_t)e2;
    P.cd_inv2 = sx > 1 ? modinv((P.G2 / e2) % sx, sx) : 0;
    P.cd_D3 = (uint32_t)D3;
    P.cd_sy = (uint32_t)sy;
    P.cd_e3 = (uint32_t)e3;
    P.cd_inv3 = sy > 1 ? modinv((gy / e3) % sy, sy) : 0;
    P.div_e2 = make_fastdiv(P.cd_e2);
    P.div_sx = make_fastdiv(P.cd_sx);
    P.div_D3 = make_fastdiv(P.cd_D3);
    P.div_e3 = make_fastdiv(P.cd_e3);
    P.div_sy = make_fastdiv(P.cd_sy);
    P.cdv = 1;
}

// The packed walk's lanes step x by sx = D / gcd(g_{d-2}, D): only the x with
// x g_{d-2} = R (mod D), D = gcd(A, B), can have an element (the
// common-divisor skip of Sec. 3.2.4).  Counts, histograms and predicates of
// the packed walk visit the same elements with fewer idle lanes.
void set_lane_stride(FzPlan &P)
{
    const uint64_t D = P.D;
    const uint64_t e2 = gcd64(P.G2, D);
    uint64_t sx = D / e2;
    if (sx >= (1u << 16)) sx = 1;
    P.cd_sx = (uint32_t)sx;
    P.cd_e2 = (uint32_t)e2;
    P.cd_inv2 = sx > 1 ? modinv((P.G2 / e2) % sx, sx) : 0;
    P.div_e2 = make_fastdiv(P.cd_e2);
    P.div_sx = make_fastdiv(P.cd_sx);
}

// Slice count, walker grid and walker variant of plan P on a device with
// `cus` compute units (no allocation).
void plan_launch(int cus, FzPlan &P, Launch &L)
{
    const uint32_t wgcu = g_wg_per_cu ? g_wg_per_cu : kDefaultWgPerCu;
    const uint32_t spw = g_slices_per_wave ? g_slices_per_wave : kDefaultSlicesPerWave;
    const uint64_t waves = (uint64_t)cus * wgcu * (FZK_WG / FZK_WAVE);
    P.n_slices = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(waves * spw, 1), kMaxSlices);
    P.min_slice_work = g_min_slice_work ? g_min_slice_work : kMinSliceWork;
    L.nwg = (uint32_t)std::min<uint64_t>((uint64_t)cus * wgcu,
                                         (P.n_slices + (FZK_WG / FZK_WAVE) - 1) / (FZK_WG / FZK_WAVE));
    P.hist_in_lds = (P.mode == FZM_HIST) &&
                    (((size_t)P.nbins + 1) * 8 <= kLdsHistBudget); // one set per workgroup
    P.prune = (g_prune_mode == 1 || (g_prune_mode == 0 && worth_pruning(P))) ? 1 : 0;
    P.pair = worth_pair(P) ? 1 : 0;
    if (P.pair && g_prune_mode != 2) P.prune = 1; // the pair walker skips empty rows too
    if (P.d < 4) P.prune = P.pair = 0;
    // table-free walk: order-free consumers whose tables would pass the
    // budget (or every one, knob "tables" = 2); stores place rows by rank
    // and always have tables
    const uint64_t table_bytes = (uint64_t)(2 * P.d - 3) * P.stride * 8;
    P.notab = (P.mode != FZM_STORE &&
               (g_tables == 2 || (g_tables == 0 && table_bytes > kTableBudget))) ? 1 : 0;
    if (P.notab) {
        P.prune = P.pair = 0;
        P.min_slice_work = 0; // no work table: always the full slice count
    }
    // a 32-bit set of bins per wave beside the workgroup's 64-bit set, when
    // both fit in kLdsHist32Budget (the waves' flushes are sized by slice
    // ranks, so not without tables)
    if (P.hist_in_lds && !P.notab && g_hist32 &&
        (size_t)((P.nbins + 2) & ~1u) * (8 + 4 * (FZK_WG / FZK_WAVE)) <= kLdsHist32Budget)
        P.hist_in_lds = 2;
    P.hist32_limit = g_hist32_limit ? g_hist32_limit : (1ull << 31);
    // interleaved copies of each wave's 32-bit set: 4, else 2, while the
    // workgroup's LDS leaves room for wgcu workgroups per CU (or the
    // requested count, within a workgroup's limit)
    P.hist32_copies = 0;
    if (P.hist_in_lds == 2) {
        const uint32_t want = g_hist32_copies ? (uint32_t)__builtin_ctz(g_hist32_copies) : 2u;
        const size_t room = g_hist32_copies ? kLdsPerWg : std::min(kLdsPerWg, kLdsPerCu / wgcu);
        for (uint32_t k = want; k > 0; --k) {
            P.hist32_copies = k;
            if (fzk_enum_lds_bytes(P) <= room) break;
            P.hist32_copies = 0;
        }
    }
    // hybrid pool (order-free consumers with tables): host threads take the
    // last slices of the work
    P.host_slices = 0;
    P.host_ppm = 0;
    if (g_host_threads && !P.notab && P.mode != FZM_STORE) {
        P.host_slices = g_host_threads;
        P.host_ppm = g_host_ppm ? g_host_ppm : kHostPpmPerThread * g_host_threads;
    }
    set_variant(P);
    P.pack = pack_rows(P);
    if (P.pack) set_lane_stride(P);
    // trailing-index tables: rows of the block walk (d >= 4, no row skipping
    // or pair table), count and store
    P.trail = (g_trailing && !P.notab && !P.prune && !P.pair && !P.cdv && !P.pack && P.d >= 4 &&
               (P.mode == FZM_COUNT || P.mode == FZM_STORE)) ? 1 : 0;
    P.trail_cap = P.trail && P.mode == FZM_STORE ? kTrailBytes / 12 : 0;
    // the block walk (d >= 4, no row skipping, pair table or packing) drops
    // the rows of a block that the count table shows empty
    P.rowtest = (g_row_test != 2 && !P.notab && !P.prune && !P.pair && !P.pack && P.d >= 4) ? 1 : 0;
    // short last slices for the order-free consumers (a store's slices
    // each stage and write their own rows: more of them cost more)
    P.guided = (g_guided != 2 && P.mode != FZM_STORE) ? 1 : 0;
}

// Bytes of each device buffer a single query of plan P needs.
struct ScratchSizes {
    size_t S, C, restab, bounds, base, recs, ctl, dpart, pt, hist, hist_rows;
};

ScratchSizes scratch_sizes(const FzPlan &P, const Launch &L)
{
    ScratchSizes z;
    z.S = P.notab ? 8 : (size_t)(P.d - 1) * P.stride * 8;
    z.C = P.notab ? 8 : (size_t)(P.d - 2) * P.stride * 8;
    z.restab = (size_t)2 * P.B * sizeof(int2);
    z.bounds = (size_t)(P.n_slices + P.host_slices + 1) * (P.d - 2) * 4;
    z.base = (size_t)(P.n_slices + P.host_slices + 1) * 8;
    z.recs = (size_t)P.n_slices * sizeof(FzSliceRec);
    z.ctl = sizeof(FzCtl);
    z.dpart = (size_t)FZK_DP_UNITS * 8;
    z.pt = P.pair ? (size_t)pair_words(P) * 8 : 0;
    z.hist = P.mode == FZM_HIST ? ((size_t)P.nbins + 1) * 8 : 0; // and a spare bin
    z.hist_rows = (P.mode == FZM_HIST && P.hist_in_lds) ? (size_t)L.nwg * P.nbins * 8 : 0;
    return z;
}

void bind_pair(const FzPlan &P, uint64_t *pt, FzBufs &B)
{
    if (P.pair) {
        B.PC = pt;
        B.PE = (uint32_t *)(B.PC + P.stride);
        B.PO = B.PE + 2 * ((P.stride + 1) / 2);
    } else {
        B.PC = nullptr;
        B.PE = nullptr;
        B.PO = nullptr;
    }
}

// Sizes the scratch for plan P and fills the buffer table.
int prepare(Ctx &c, FzPlan &P, FzBufs &B, Launch &L)
{
    plan_launch(c.cus, P, L);
    const ScratchSizes z = scratch_sizes(P, L);
    FZ_TRY(ensure(c.S, z.S));
    FZ_TRY(ensure(c.C, z.C));
    FZ_TRY(ensure(c.restab, z.restab));
    FZ_TRY(ensure(c.bounds, z.bounds));
    FZ_TRY(ensure(c.base, z.base));
    FZ_TRY(ensure(c.recs, z.recs));
    FZ_TRY(ensure(c.ctl, z.ctl));
    FZ_TRY(ensure(c.dpart, z.dpart));
    if (P.pair) FZ_TRY(ensure(c.pt, z.pt));
    bind_pair(P, (uint64_t *)c.pt.p, B);
    if (P.mode == FZM_HIST) {
        FZ_TRY(ensure(c.hist, z.hist));
        if (P.hist_in_lds) FZ_TRY(ensure(c.hist_rows, z.hist_rows));
    }
    B.S = (uint64_t *)c.S.p;
    B.C = (uint64_t *)c.C.p;
    B.restab = (int2 *)c.restab.p;
    B.bounds = (uint32_t *)c.bounds.p;
    B.base = (uint64_t *)c.base.p;
    B.recs = (FzSliceRec *)c.recs.p;
    B.ctl = (FzCtl *)c.ctl.p;
    B.hist_rows = (uint64_t *)c.hist_rows.p;
    B.dpart = (uint64_t *)c.dpart.p;
    B.hist = (uint64_t *)c.hist.p;
    B.out = nullptr;
    B.TO = nullptr;
    B.TT = nullptr;
    if (P.trail && P.mode == FZM_STORE) {
        FZ_TRY(ensure(c.trail_o, ((size_t)P.stride + 1) * 8));
        FZ_TRY(ensure(c.trail_t, (size_t)P.trail_cap * 12));
        B.TO = (uint64_t *)c.trail_o.p;
        B.TT = (uint32_t *)c.trail_t.p;
    }
    return FZ_OK;
}


// ---------------------------------------------------------------------------
// Hybrid pool (Sec. 6.3): host threads walk the last few slices of a query
// while the device walks the others.  A host worker walks its slice [b0, b1)
// of prefixes (a_1 .. a_{d-2}) in ascending lexicographic order and, for each
// prefix with remainder R, the elements of the last pair: the first a_{d-1}
// with A a_{d-1} = R (mod B), then steps of (ord, -delta) while a_d >= 0
// (the modulo skip of Sec. 3.2.4).  Counts, a plain length histogram, or the
// length predicate.
// ---------------------------------------------------------------------------
struct HostPart {
    uint64_t elements = 0;
    bool found = false;
    std::vector<uint64_t> hist;
};

void host_walk(const FzPlan &P, const uint32_t *b0, const uint32_t *b1, HostPart &o)
{
    const uint32_t K = P.d - 2;
    if (P.mode == FZM_HIST) o.hist.assign(P.nbins, 0);
    if (b0[0] == FZK_SENTINEL) return; // an empty slice
    const bool open = b1[0] == FZK_SENTINEL;
    uint32_t a[FZK_MAX_D];
    uint64_t rr[FZK_MAX_D + 1];
    rr[0] = P.n;
    uint64_t plen = 0;
    for (uint32_t k = 0; k < K; ++k) {
        a[k] = b0[k];
        rr[k + 1] = rr[k] - (uint64_t)a[k] * P.g[k];
        plen += a[k];
    }
    const uint64_t A = P.A, Bg = P.B, D = P.D, ord = P.ord, dl = P.delta, inv = P.inv;
    for (;;) {
        if (!open) { // stop at the end bound
            uint32_t k = 0;
            while (k < K && a[k] == b1[k]) ++k;
            if (k == K || a[k] > b1[k]) break;
        }
        const uint64_t R = rr[K];
        if (R % D == 0) {
            const uint64_t t0 = ((R / D) % ord) * inv % ord;
            if (A * t0 <= R) {
                uint64_t e = (R - A * t0) / Bg, t = t0;
                for (;;) { // one element per step
                    ++o.elements;
                    const uint64_t len = plen + t + e;
                    if (P.mode == FZM_HIST) ++o.hist[len];
                    else if (P.mode == FZM_EXISTS && len == P.target_len) o.found = true;
                    if (e < dl) break;
                    e -= dl;
                    t += ord;
                }
            }
        }
        // the next prefix: the deepest coordinate that can grow
        int kk = (int)K - 1;
        while (kk >= 0 && rr[kk + 1] < P.g[kk]) --kk;
        if (kk < 0) break;
        ++a[kk];
        rr[kk + 1] -= P.g[kk];
        for (uint32_t j = kk + 1; j < K; ++j) {
            plen -= a[j];
            a[j] = 0;
            rr[j + 1] = rr[j];
        }
        plen += 1;
    }
}

// Queues the whole path for one query and waits: count table, residue table,
// slice bounds, walker, finalize, control-block readback.
int run_query(Ctx &c, FzPlan &P, FzBufs &B, const Launch &L, hipStream_t s)
{
    if (!P.notab) FZ_LAUNCH("dp", s, fzk_launch_dp(P, B, s));
    if (P.trail && P.mode == FZM_STORE) FZ_LAUNCH("trail", s, fzk_launch_trail(P, B, s));
    FZ_LAUNCH("restab", s, fzk_launch_restab(P, B, s));
    if (P.notab) FZ_LAUNCH("slices", s, fzk_launch_split(P, B, s));
    else FZ_LAUNCH("slices", s, fzk_launch_slices(P, B, s));
    // hybrid pool: the host slices' bounds and base ranks come back while
    // the device walks its own
    const uint32_t T = P.host_slices, W = P.n_slices, KP = P.d - 2;
    uint32_t *hb = nullptr;
    uint64_t *hbase = nullptr;
    if (T) {
        const size_t bb = (size_t)(T + 1) * KP * 4, bo = (bb + 7) & ~(size_t)7;
        FZ_TRY(ensure_pinned(&c.h_hostb, &c.h_hostb_cap, bo + (size_t)(T + 1) * 8));
        hb = (uint32_t *)c.h_hostb;
        hbase = (uint64_t *)((char *)c.h_hostb + bo);
        FZ_TRY(hipMemcpyAsync(hb, B.bounds + (uint64_t)W * KP, bb, hipMemcpyDeviceToHost, s));
        FZ_TRY(hipMemcpyAsync(hbase, B.base + W, (size_t)(T + 1) * 8, hipMemcpyDeviceToHost, s));
        if (!c.host_ev) FZ_TRY(hipEventCreateWithFlags(&c.host_ev, hipEventDisableTiming));
        FZ_TRY(hipEventRecord(c.host_ev, s));
    }
    static const char *const kEnumNames[] = {"enum.count", "enum.hist", "enum.exists",
                                             "enum.store"};
    FZ_LAUNCH(kEnumNames[P.mode & 3], s, fzk_launch_enum(P, B, L.nwg, s));
    FZ_LAUNCH("finalize", s, fzk_launch_finalize(P, B, L.nwg, s));
    FZ_TRY(hipMemcpyAsync(c.host_ctl, B.ctl, sizeof(FzCtl), hipMemcpyDeviceToHost, s));
    std::vector<HostPart> parts(T);
    if (T) {
        FZ_TRY(hipEventSynchronize(c.host_ev));
        std::vector<std::thread> th;
        for (uint32_t t = 0; t < T; ++t)
            th.emplace_back(host_walk, std::cref(P), hb + (size_t)t * KP, hb + (size_t)(t + 1) * KP,
                            std::ref(parts[t]));
        for (auto &x : th) x.join();
    }
    FZ_TRY(hipStreamSynchronize(s));
    prof_collect();
    FzCtl &h = *c.host_ctl;
    if (h.status & FZS_OVERFLOW) return FZ_EOVERFLOW;
    if (h.status & FZS_MISMATCH) return FZ_EINTERNAL;
    c.host_hist.clear();
    if (T) { // fold the host part into the device's results
        for (uint32_t t = 0; t < T; ++t) {
            const HostPart &o = parts[t];
            if (P.mode != FZM_EXISTS && o.elements != hbase[t + 1] - hbase[t]) return FZ_EINTERNAL;
            h.count += o.elements;
            h.found = h.found || o.found;
            if (P.mode == FZM_HIST && o.hist.size() == P.nbins) {
                if (c.host_hist.empty()) c.host_hist.assign(P.nbins, 0);
                for (uint32_t l = 0; l < P.nbins; ++l) c.host_hist[l] += o.hist[l];
            }
        }
    }
    c.last.slices = h.slices;
    c.last_batch = false;
    c.last.rows = h.rows;
    c.last.prefixes = h.prefixes;
    c.last.elements = h.count;
    c.last.candidates = h.count + h.prefixes;
    return FZ_OK;
}

int do_count(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count, void *stream)
{
    if (count == nullptr) return FZ_EINVAL;
    FzPlan P;
    int rc = make_walk_plan(n, g, d, FZM_COUNT, &P);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *c;
    if ((rc = get_ctx(&c))) return rc;
    FzBufs B;
    Launch L;
    if ((rc = prepare(*c, P, B, L))) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    if ((rc = run_query(*c, P, B, L, s))) return rc;
    if (c->host_ctl->count != c->host_ctl->total) return FZ_EINTERNAL;
    *count = c->host_ctl->count;
    return FZ_OK;
}

int do_enumerate(uint64_t n, const uint32_t *g, uint32_t d, uint32_t *out, bool out_on_device,
                 uint64_t max_tuples, uint64_t *total, uint64_t *written, void *stream)
{
    if (total == nullptr || written == nullptr) return FZ_EINVAL;
    if (out == nullptr && max_tuples > 0) return FZ_EINVAL;
    FzPlan P;
    int rc = make_plan(n, g, d, FZM_STORE, &P);
    if (rc) return rc;
    P.max_tuples = max_tuples;
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *c;
    if ((rc = get_ctx(&c))) return rc;
    FzBufs B;
    Launch L;
    if ((rc = prepare(*c, P, B, L))) return rc;
    hipStream_t s = stream ? (hipStream_t)stream : c->stream;
    uint32_t *dev_out = out;
    if (!out_on_device) {
        // The host buffer needs a device staging copy of min(|Z|, max_tuples)
        // rows: count first (one small readback), then size the staging.
        FZ_LAUNCH("dp", s, fzk_launch_dp(P, B, s));
        uint64_t N = 0;
        FZ_TRY(hipMemcpyAsync(&N, B.S + P.n, 8, hipMemcpyDeviceToHost, s));
        FZ_TRY(hipStreamSynchronize(s));
        if (N == UINT64_MAX) return FZ_EOVERFLOW;
        const uint64_t rows = std::min(N, max_tuples);
        FZ_TRY(ensure(c->rows_out, rows * P.d_user * 4));
        dev_out = (uint32_t *)c->rows_out.p;
    }
    B.out = dev_out;
    if ((rc = run_query(*c, P, B, L, s))) return rc;
    const FzCtl &h = *c->host_ctl;
    const uint64_t N = h.total;
    const uint64_t wr = std::min(N, max_tuples);
    if (h.count != wr) return FZ_EINTERNAL;
    if (!out_on_device && wr) {
        FZ_TRY(hipMemcpyAsync(out, dev_out, wr * P.d_user * 4, hipMemcpyDeviceToHost, s));
        FZ_TRY(hipStreamSynchronize(s));
    }
    *total = N;
    *written = wr;
    return wr < N ? FZ_TRUNCATED : FZ_OK;
}

// Rough counts of a query's rows (a_1..a_{d-3}), lane prefixes
// (a_1..a_{d-2}) and elements, from the leading terms: a set
// {a : sum_{i<k} a_i g_i <= v} has about v^k / (k! prod g_i) points.  Only
// used to decide how finely to cut and whether to skip empty rows.
void estimate_counts(const FzPlan &P, double *rows, double *pref, double *el)
{
    const uint32_t M = P.d - 3;
    const double ln1 = std::log((double)P.n + 1.0);
    double lg_rows = 0, lg_pref = 0, lg_el = 0;
    for (uint32_t k = 0; k < M; ++k) lg_rows -= std::log((double)P.g[k]);
    lg_pref = lg_rows - std::log((double)P.g[M]);
    lg_el = lg_pref - std::log((double)P.g[M + 1]) - std::log((double)P.g[M + 2]);
    lg_rows += M * ln1 - std::lgamma(M + 1.0);
    lg_pref += (M + 1) * ln1 - std::lgamma(M + 2.0);
    lg_el += (M + 2) * ln1 - std::lgamma(M + 3.0);
    *rows = std::max(std::exp(std::min(lg_rows, 200.0)), 1.0);
    *pref = std::exp(std::min(lg_pref, 200.0));
    *el = std::exp(std::min(lg_el, 200.0));
}

// Sparse sets (few elements per row) walk only the rows that have elements:
// most rows then have none, and skipping them costs a fraction of a walk.
bool worth_pruning(const FzPlan &P)
{
    if (P.d < 4) return false;
    double rows, pref, el;
    estimate_counts(P, &rows, &pref, &el);
    return el < kPruneElementsPerRow * rows;
}

// Order-free consumers of sparse sets walk their rows packed: a row has
// about n / ((M + 1) g_{d-2}) lane prefixes, and a row of fewer than a
// chunk's lanes leaves the rest of its chunk idle.  Only walks that skip
// empty rows: without skipping, the block walk (rows prepared in lanes, one
// table offset stepped per chunk) walks short rows faster than the packed
// walk solves each lane's remainder (the d = 11 length set, 27 prefixes per
// row: 355 ms block walk, 382 ms packed).  (Not with the pair table or the
// variant walk, which choose their own prefixes.)
uint32_t pack_rows(const FzPlan &P)
{
    if (P.mode == FZM_STORE || P.d < 4 || P.pair || P.cdv || g_pack_mode == 2) return 0;
    if (g_pack_mode == 1) return 1;
    if (!P.prune) return 0;
    double rows, pref, el;
    estimate_counts(P, &rows, &pref, &el);
    return pref < kPackPrefixesPerRow * rows ? 1 : 0;
}

// A sparse last pair: a remainder v <= n is representable by (A, B) with
// probability about n D / (2 A B) when that is small, so the lanes of a row
// walking every x mostly find nothing.  Then the walker reads the
// representable remainders from the pair table instead (needs M >= 1).
bool worth_pair(const FzPlan &P)
{
    if (P.d < 4 || g_pair_mode == 2) return false;
    if (g_pair_mode == 1) return true;
    const double frac = (double)P.n * P.D / (2.0 * (double)P.A * (double)P.B);
    return frac < kPairMaxFraction;
}

// Words of a query's pair table: counts (n+1), remainders, chain starts.
uint64_t pair_words(const FzPlan &P)
{
    const uint64_t nc = std::min<uint64_t>(P.G2, P.stride);
    return (uint64_t)P.stride + (P.stride + 1) / 2 + (nc + 2) / 2;
}

// Rough work of a query in the walker's units.  With pruning, each element
// is charged a row and a chunk of its own (an upper bound for a sparse set)
// and every row the cost of being skipped.
double estimate_work(const FzPlan &P)
{
    double rows, pref, el;
    estimate_counts(P, &rows, &pref, &el);
    if (P.prune)
        return P.w_skip * rows + (double)(P.w_row + P.w_chunk + P.w_el) * el;
    if (P.pack) return P.w_row * rows + P.w_chunk * (pref / FZK_WAVE) + P.w_el * el;
    return P.w_row * rows + P.w_chunk * (pref / FZK_WAVE + rows) + P.w_el * el;
}

// The knobs of a batch (fz_batch and the server).  Their defaults differ
// from a single query's: the batch walker holds up to 2048 histogram words
// of LDS per wave, so fewer workgroups fit a CU, and fewer, longer items
// per wave cost less set-up (mixed 4096-query batch: 84 ms with 16 slices
// per wave x 8 workgroups per CU, 74 ms with 8 x 4).
void current_knobs(uint32_t *spw, uint32_t *wgcu)
{
    *spw = g_slices_per_wave ? g_slices_per_wave : kBatchSlicesPerWave;
    *wgcu = g_wg_per_cu ? g_wg_per_cu : kBatchWgPerCu;
}

hipError_t ensure_pinned(void **p, size_t *cap, size_t bytes)
{
    if (bytes <= *cap && *p) return hipSuccess;
    if (*p) (void)hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t want = std::max(bytes, (size_t)4096);
    hipError_t e = hipHostMalloc(p, want, hipHostMallocCoherent);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return e;
    }
    *cap = want;
    return hipSuccess;
}

void BatchSlot::release()
{
    for (DevBuf *b :
         {&meta, &tables, &restabs, &bounds, &base, &recs, &bins, &res, &cursor, &totals}) {
        if (b->p) (void)hipFree(b->p);
        b->p = nullptr;
        b->cap = 0;
    }
    for (void **h : {(void **)&h_meta, (void **)&h_res, (void **)&h_done, (void **)&h_bins,
                     (void **)&h_totals}) {
        if (*h) (void)hipHostFree(*h);
        *h = nullptr;
    }
    h_meta_cap = 0;
    h_cap = 0;
    h_bins_cap = 0;
    h_totals_cap = 0;
    if (tables_ev) (void)hipEventDestroy(tables_ev);
    tables_ev = nullptr;
    if (walk_exec) (void)hipGraphExecDestroy(walk_exec);
    walk_exec = nullptr;
    walk_pending = false;
}

// Work weights of the batch walker, in its own units (1/8 of the time of an
// element step of a long run), fitted to per-query wave time over the mixed
// 4096-query workload: a row about 110 element steps, a row visited while
// skipping empty rows about 300 (its emptiness test is a dependent load), a
// 64-lane chunk about 37, a skipped row about 8.
constexpr uint32_t kBatchRow = 880, kBatchRowSkipping = 2370, kBatchChunk = 300,
                   kBatchSkip = 62;
constexpr uint32_t kBatchElem[4] = {35, 40, 40, 48}; // count, hist, exists, store
// A batch table row of more entries than this is shared by several
// workgroups (one per this many entries, at most one per chain).
constexpr uint32_t kDpGroupEntries = 1u << 16;
// ... when at most this many queries of a batch have such rows.
constexpr uint32_t kDpMaxSharedQueries = 128;
// Least modelled work of a batch's work item (a 64-lane chunk is ~300 units).
constexpr uint64_t kBatchMinItemWork = 1u << 20;
// Skipping pays off only on sets with enough rows.
constexpr double kPruneMinRows = 4096.0;

int batch_launch_tables(BatchSlot &S, int cus, uint32_t spw, uint32_t wgcu, const fz_query *qs,
                        uint32_t nq, hipStream_t st, uint64_t store_cap, bool profile)
{
    // plans; a rejected query keeps d = 0 and takes no device work
    std::vector<FzBatchQuery> &Q = S.Q;
    Q.assign(nq, FzBatchQuery{});
    S.qst.assign(nq, FZ_OK);
    S.nq = nq;
    S.n_items = 0;
    S.walk_pending = false;
    std::vector<double> &work = S.work;
    work.assign(nq, 0.0);
    double est_total = 0;
    uint32_t maxm = 0, max_du = 0, bstride = 1;
    bool any_hist = false;
    for (uint32_t i = 0; i < nq; ++i) {
        std::memset(&Q[i], 0, sizeof(FzBatchQuery));
        const fz_query &q = qs[i];
        if (q.mode > FZ_MODE_STORE) { S.qst[i] = FZ_EINVAL; continue; }
        FzPlan &P = Q[i].plan;
        int e = make_walk_plan(q.n, q.g, q.d, q.mode, &P);
        if (!e && q.mode == FZ_MODE_HIST && (q.bins == nullptr || q.nbins < P.nbins)) e = FZ_EINVAL;
        if (!e && q.mode == FZ_MODE_STORE && q.d_out == nullptr && q.max_tuples > 0) e = FZ_EINVAL;
        if (e) {
            S.qst[i] = e;
            std::memset(&P, 0, sizeof P);
            continue;
        }
        P.target_len = q.target_len;
        if (q.mode == FZ_MODE_STORE) P.max_tuples = q.max_tuples;
        Q[i].max_total = store_cap;
        double rows, pref, el;
        estimate_counts(P, &rows, &pref, &el);
        P.prune = (P.d >= 4 && (g_prune_mode == 1 ||
                                (g_prune_mode == 0 && worth_pruning(P) && rows >= kPruneMinRows)))
                      ? 1 : 0;
        P.w_row = g_work_row ? g_work_row : (P.prune ? kBatchRowSkipping : kBatchRow);
        P.w_chunk = g_work_chunk ? g_work_chunk : kBatchChunk;
        P.w_el = g_work_elem ? g_work_elem : kBatchElem[P.mode & 3];
        P.w_skip = kBatchSkip;
        // No pair table in a batch: the batch walker is one kernel for all
        // variants, and the pair variant's registers would halve its occupancy.
        P.pair = 0;
        // the batch walker walks every order-free consumer packed
        P.pack = P.mode != FZM_STORE ? 1 : 0;
        if (P.pack) set_lane_stride(P);
        work[i] = estimate_work(P);
        est_total += work[i];
        maxm = std::max(maxm, P.d - 3);
        bstride = std::max(bstride, P.d - 2);
        if (q.mode == FZ_MODE_STORE) max_du = std::max(max_du, P.d_user);
        if (q.mode == FZ_MODE_HIST) any_hist = true;
    }
    const double slots = (double)cus * wgcu * (FZK_WG / FZK_WAVE) * spw;
    const uint32_t lds_bins = any_hist ? kBatchLdsBins : 0;

    // Phase 1: count and work tables for every query that may be cut --
    // stores (rows placed by rank), sparse queries (they skip empty rows by
    // the count table) and any query estimated above half a slice -- and the
    // exact modelled work of each, read back to size its slice count.
    std::vector<uint32_t> &tabled = S.tabled;
    tabled.clear();
    uint64_t tab_words = 0, res_words = 0, bin_words = 0;
    const double est_target =
        std::max(est_total / slots, (double)(g_batch_min_item ? g_batch_min_item : kBatchMinItemWork));
    for (uint32_t i = 0; i < nq; ++i) {
        FzBatchQuery &B = Q[i];
        FzPlan &P = B.plan;
        if (!P.d) continue;
        // (histograms that may take 32-bit LDS bins get tables too: the
        // count table bounds their bins exactly)
        const bool mid_hist = P.mode == FZM_HIST && P.nbins > kBatchLdsBins / 2 &&
                              P.nbins <= kBatchLdsBins;
        B.sliced = (P.mode == FZM_STORE || P.prune || mid_hist || work[i] > 0.5 * est_target)
                       ? 1 : 0;
        P.hist_in_lds = 0; // decided with the cut (32-bit LDS bins need a bound)
        P.restab_in_lds = 0;
        if (B.sliced) {
            B.s_off = tab_words;
            tab_words += (uint64_t)(P.d - 1) * P.stride;
            B.c_off = tab_words;
            tab_words += (uint64_t)(P.d - 2) * P.stride;
            tabled.push_back(i);
        }
        B.tab_off = res_words;
        res_words += 2 * (uint64_t)P.B;
        if (P.mode == FZM_HIST) {
            B.bins_off = bin_words;
            bin_words += P.nbins;
        }
        B.out = qs[i].d_out;
    }
    const uint32_t n_tab = (uint32_t)tabled.size();
    // Tables: one workgroup builds all rows of a query (one launch for all
    // of them) -- but when few queries have large rows (more than
    // kDpGroupEntries entries), a workgroup each would leave most of the
    // chip idle: those are built pass by pass (their 2d - 3 row computations
    // in order, a launch each), every row shared by up to one workgroup per
    // kDpGroupEntries entries (by chains; C row M by ranges).  With many
    // large queries the chip is full anyway, and one workgroup per query
    // overlaps the queries' rows better than passes, which wait for their
    // slowest row (4096-query batch: 6.4 ms against 20 ms).
    std::vector<uint32_t> &pjobs = S.pass_jobs;
    std::vector<uint32_t> &poff = S.pass_off;
    std::vector<uint32_t> &small = S.small_ids;
    pjobs.clear();
    poff.assign(1, 0);
    small.clear();
    uint32_t n_pass = 0, n_large = 0;
    for (uint32_t i : tabled) n_large += Q[i].plan.stride > kDpGroupEntries ? 1 : 0;
    const bool by_pass = n_large > 0 && n_large <= kDpMaxSharedQueries;
    for (uint32_t i : tabled) {
        if (by_pass && Q[i].plan.stride > kDpGroupEntries)
            n_pass = std::max(n_pass, 2 * Q[i].plan.d - 3);
        else small.push_back(i);
    }
    for (uint32_t p = 0; p < n_pass; ++p) {
        for (uint32_t i : tabled) {
            const FzPlan &P = Q[i].plan;
            if (!by_pass || P.stride <= kDpGroupEntries || p >= 2 * P.d - 3) continue;
            const uint32_t parts = (uint32_t)((P.stride + kDpGroupEntries - 1) / kDpGroupEntries);
            uint32_t G = parts;
            if (p + 1 != P.d) { // a chain scan: row k of S or C, chains g_k
                const uint32_t k = p + 2 <= P.d ? P.d - 2 - p : P.d - 4 - (p - P.d);
                G = std::min(parts, std::min(P.g[k], P.stride));
            }
            G = std::max(G, 1u);
            for (uint32_t w = 0; w < G; ++w) {
                pjobs.push_back(i);
                pjobs.push_back(w);
                pjobs.push_back(G);
            }
        }
        poff.push_back((uint32_t)(pjobs.size() / 3));
    }
    auto up = [](size_t o) { return (o + 63) & ~(size_t)63; };
    const size_t o_q = 0;
    const size_t o_ids = up(o_q + (size_t)nq * sizeof(FzBatchQuery));
    const size_t o_small = up(o_ids + (size_t)n_tab * 4);
    const size_t o_pj = up(o_small + small.size() * 4);
    const size_t meta1 = up(o_pj + pjobs.size() * 4);
    FZ_TRY(ensure_pinned((void **)&S.h_meta, &S.h_meta_cap, meta1));
    std::memcpy(S.h_meta + o_q, Q.data(), (size_t)nq * sizeof(FzBatchQuery));
    if (n_tab) std::memcpy(S.h_meta + o_ids, tabled.data(), (size_t)n_tab * 4);
    if (!small.empty()) std::memcpy(S.h_meta + o_small, small.data(), small.size() * 4);
    if (!pjobs.empty()) std::memcpy(S.h_meta + o_pj, pjobs.data(), pjobs.size() * 4);
    if (S.h_cap < nq) {
        size_t c1 = 0, c2 = 0;
        if (S.h_res) (void)hipHostFree(S.h_res);
        if (S.h_done) (void)hipHostFree(S.h_done);
        S.h_res = nullptr;
        S.h_done = nullptr;
        S.h_cap = 0;
        FZ_TRY(ensure_pinned((void **)&S.h_res, &c1, (size_t)nq * sizeof(FzBatchResult)));
        FZ_TRY(ensure_pinned((void **)&S.h_done, &c2, (size_t)nq * 4));
        S.h_cap = nq;
    }
    {
        size_t cap = S.h_bins_cap * 8;
        FZ_TRY(ensure_pinned((void **)&S.h_bins, &cap, std::max<size_t>(bin_words, 1) * 8));
        S.h_bins_cap = cap / 8;
        cap = S.h_totals_cap * 8;
        FZ_TRY(ensure_pinned((void **)&S.h_totals, &cap, std::max<size_t>(n_tab, 1) * 16));
        S.h_totals_cap = cap / 8;
    }
    std::memset(S.h_done, 0, (size_t)nq * 4);
    std::memset(S.h_res, 0, (size_t)nq * sizeof(FzBatchResult));
    FZ_TRY(ensure(S.meta, meta1));
    FZ_TRY(ensure(S.tables, tab_words * 8));
    FZ_TRY(ensure(S.restabs, res_words * sizeof(int2)));
    FZ_TRY(ensure(S.bins, bin_words * 8));
    FZ_TRY(ensure(S.res, (size_t)nq * sizeof(FzBatchResult)));
    FZ_TRY(ensure(S.totals, (size_t)std::max(n_tab, 1u) * 16));
    FZ_TRY(ensure(S.cursor, 256));
    uint8_t *meta = (uint8_t *)S.meta.p;

    FzBatchBufs B;
    std::memset(&B, 0, sizeof B);
    B.queries = (const FzBatchQuery *)(meta + o_q);
    B.tables = (uint64_t *)S.tables.p;
    B.restabs = (int2 *)S.restabs.p;
    B.bins = (uint64_t *)S.bins.p;
    B.res = (FzBatchResult *)S.res.p;
    B.totals = (uint64_t *)S.totals.p;
    B.cursor = (uint32_t *)S.cursor.p;
    B.host_res = S.h_res;
    B.host_bins = S.h_bins;
    B.host_done = S.h_done;
    B.nq = nq;
    B.n_bins = bin_words;
    bool any_valid = false;
    for (uint32_t i = 0; i < nq; ++i) any_valid = any_valid || Q[i].plan.d != 0;
    if (!any_valid) return FZ_OK; // every query was rejected on the host: nothing to walk
    FZ_TRY(hipMemcpyAsync(meta, S.h_meta, meta1, hipMemcpyHostToDevice, st));
    const uint32_t *ids = (const uint32_t *)(meta + o_ids);
    const uint32_t *sids = (const uint32_t *)(meta + o_small);
    const uint32_t *pj = (const uint32_t *)(meta + o_pj);
    const uint32_t n_small = (uint32_t)small.size();
    if (profile)
        FZ_LAUNCH("batch.tables", st,
                  fzk_launch_batch_tables(B, n_tab, ids, n_small, sids, pj, poff.data(), n_pass,
                                          st));
    else
        FZ_TRY(fzk_launch_batch_tables(B, n_tab, ids, n_small, sids, pj, poff.data(), n_pass, st));
    if (n_tab)
        FZ_TRY(hipMemcpyAsync(S.h_totals, S.totals.p, (size_t)n_tab * 16, hipMemcpyDeviceToHost,
                              st));
    if (!S.tables_ev) FZ_TRY(hipEventCreateWithFlags(&S.tables_ev, hipEventDisableTiming));
    FZ_TRY(hipEventRecord(S.tables_ev, st));
    S.B = B;
    S.stream = st;
    S.slots = slots;
    S.cus = (uint32_t)cus;
    S.wgcu = wgcu;
    S.maxm = maxm;
    S.max_du = max_du;
    S.lds_bins = lds_bins;
    S.bstride = bstride;
    S.profile = profile;
    S.walk_pending = true;
    return FZ_OK;
}

// Phase 2 as a HIP graph: the slice-bound and walker launches are captured
// (their topology is the same for every batch of a slot) and the slot's
// executable graph is updated in place with the new kernel arguments, or
// instantiated again when the update is refused (another walker variant).
int launch_walk_graph(BatchSlot &S, const FzBatchBufs &B, uint32_t maxm, uint32_t nwg,
                      uint32_t lds_bins, uint32_t max_du, hipStream_t st)
{
    hipGraph_t g = nullptr;
    FZ_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const hipError_t e1 = fzk_launch_batch_slices(B, st);
    const hipError_t e2 = fzk_launch_batch_walk(B, maxm, nwg, lds_bins, max_du, st);
    const hipError_t e3 = hipStreamEndCapture(st, &g);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        return dev_err_at(e1 != hipSuccess ? e1 : e2 != hipSuccess ? e2 : e3, "batch graph capture",
                          __LINE__);
    }
    if (S.walk_exec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(S.walk_exec, g, &bad, &res) != hipSuccess ||
            res != hipGraphExecUpdateSuccess) {
            (void)hipGetLastError();
            (void)hipGraphExecDestroy(S.walk_exec);
            S.walk_exec = nullptr;
        }
    }
    hipError_t e = hipSuccess;
    if (!S.walk_exec) e = hipGraphInstantiate(&S.walk_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        S.walk_exec = nullptr;
        return dev_err_at(e, "hipGraphInstantiate", __LINE__);
    }
    FZ_TRY(hipGraphLaunch(S.walk_exec, st));
    return FZ_OK;
}

int batch_launch_walk(BatchSlot &S)
{
    if (!S.walk_pending) return FZ_OK;
    S.walk_pending = false;
    std::vector<FzBatchQuery> &Q = S.Q;
    const std::vector<double> &work0 = S.work;
    std::vector<double> work(work0);
    const std::vector<uint32_t> &tabled = S.tabled;
    const uint32_t nq = S.nq, n_tab = (uint32_t)tabled.size();
    const double slots = S.slots;
    const hipStream_t st = S.stream;
    const uint32_t bstride = S.bstride, maxm = S.maxm, max_du = S.max_du, lds_bins = S.lds_bins;
    const uint32_t cus = S.cus, wgcu = S.wgcu;
    const bool profile = S.profile;
    FzBatchBufs B = S.B;
    auto up = [](size_t o) { return (o + 63) & ~(size_t)63; };
    const size_t o_q = 0;

    // Phase 2: cut.  A query with tables gets ceil(work / target) slices of
    // its exact modelled work; the others are one slice each.  Items of large
    // queries first, then the rest by falling work per slice.
    std::vector<double> exact(nq, 0.0);
    std::vector<uint64_t> elements(nq, ~0ull); // |Z| of the queries with tables
    double total = 0;
    for (uint32_t k = 0; k < n_tab; ++k) {
        const uint64_t c = S.h_totals[2 * k];
        exact[tabled[k]] = c == ~0ull ? 0.0 : (double)c; // overflow: walked not at all
        elements[tabled[k]] = S.h_totals[2 * k + 1];
    }
    for (uint32_t i = 0; i < nq; ++i)
        if (Q[i].plan.d) total += Q[i].sliced ? exact[i] : work[i];
    // (a small batch is not cut into a full chip's worth of tiny items: each
    // item carries at least kBatchMinItemWork units, a few hundred
    // microseconds of a wave -- its set-up, histogram flush and records cost
    // tens of microseconds)
    const double target =
        std::max(total / slots, (double)(g_batch_min_item ? g_batch_min_item : kBatchMinItemWork));
    std::vector<uint32_t> order;
    uint32_t n_items = 0, n_bounds = 0;
    for (uint32_t i = 0; i < nq; ++i) {
        FzBatchQuery &B2 = Q[i];
        if (!B2.plan.d) continue;
        if (B2.sliced) work[i] = exact[i];
        B2.n_slices = B2.sliced
                          ? (uint32_t)std::min(std::max(std::ceil(work[i] / target), 1.0), 65536.0)
                          : 1;
        B2.plan.n_slices = B2.n_slices;
        // 64-bit bins when half the area holds them (measured faster), else
        // 32-bit ones when the query has fewer than 2^30 elements (a bin of
        // the difference array moves by at most the elements of one item;
        // |Z| is exact from the count table, which every histogram of this
        // size has), else global atomics
        B2.plan.hist_in_lds = 0;
        if (B2.plan.mode == FZM_HIST && B2.plan.nbins <= lds_bins / 2) B2.plan.hist_in_lds = 1;
        else if (B2.plan.mode == FZM_HIST && B2.plan.nbins <= lds_bins && B2.sliced &&
                 elements[i] < (1ull << 30))
            B2.plan.hist_in_lds = 2;
        B2.bound_off = n_bounds;
        n_bounds += B2.n_slices + 1;
        order.push_back(i);
    }
    const bool small_first = S.small_first;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        if (Q[a].sliced != Q[b].sliced) return (Q[a].sliced > Q[b].sliced) != small_first;
        if (small_first && !Q[a].sliced) return work[a] < work[b];
        return work[a] / Q[a].n_slices > work[b] / Q[b].n_slices;
    });
    for (uint32_t i : order) {
        Q[i].item_off = n_items;
        n_items += Q[i].n_slices;
    }
    S.n_items = n_items;

    const size_t o_jobs = up(o_q + (size_t)nq * sizeof(FzBatchQuery));
    const size_t o_items = up(o_jobs + (size_t)n_bounds * sizeof(FzBatchJob));
    const size_t meta2 = up(o_items + (size_t)n_items * sizeof(FzBatchJob));
    FZ_TRY(ensure_pinned((void **)&S.h_meta, &S.h_meta_cap, meta2));
    uint8_t *hm = S.h_meta;
    std::memcpy(hm + o_q, Q.data(), (size_t)nq * sizeof(FzBatchQuery));
    FzBatchJob *hj = (FzBatchJob *)(hm + o_jobs);
    FzBatchJob *hi = (FzBatchJob *)(hm + o_items);
    for (uint32_t i : order) {
        for (uint32_t j = 0; j <= Q[i].n_slices; ++j) hj[Q[i].bound_off + j] = {i, j};
        for (uint32_t j = 0; j < Q[i].n_slices; ++j) hi[Q[i].item_off + j] = {i, j};
    }
    FZ_TRY(ensure(S.meta, meta2));
    FZ_TRY(ensure(S.bounds, (size_t)n_bounds * bstride * 4));
    FZ_TRY(ensure(S.base, (size_t)n_bounds * 8));
    FZ_TRY(ensure(S.recs, (size_t)std::max(n_items, 1u) * sizeof(FzSliceRec)));
    uint8_t *meta = (uint8_t *)S.meta.p; // a larger staging area moves the device copy
    FZ_TRY(hipMemcpyAsync(meta, hm, meta2, hipMemcpyHostToDevice, st));
    B.queries = (const FzBatchQuery *)(meta + o_q);
    B.bjobs = (const FzBatchJob *)(meta + o_jobs);
    B.items = (const FzBatchJob *)(meta + o_items);
    B.bounds = (uint32_t *)S.bounds.p;
    B.base = (uint64_t *)S.base.p;
    B.recs = (FzSliceRec *)S.recs.p;
    B.n_bjobs = n_bounds;
    B.n_items = n_items;
    B.bstride = bstride;
    const uint32_t nwg = (uint32_t)std::min<uint64_t>((uint64_t)cus * wgcu,
                                                      std::max<uint32_t>(1, (n_items + 3) / 4));
    if (profile) {
        FZ_LAUNCH("batch.slices", st, fzk_launch_batch_slices(B, st));
        FZ_LAUNCH("batch.walk", st, fzk_launch_batch_walk(B, maxm, nwg, lds_bins, max_du, st));
    } else if (g_batch_graph) {
        return launch_walk_graph(S, B, maxm, nwg, lds_bins, max_du, st);
    } else {
        FZ_TRY(fzk_launch_batch_slices(B, st));
        FZ_TRY(fzk_launch_batch_walk(B, maxm, nwg, lds_bins, max_du, st));
    }
    return FZ_OK;
}

int batch_launch(BatchSlot &S, int cus, uint32_t spw, uint32_t wgcu, const fz_query *qs,
                 uint32_t nq, hipStream_t st, uint64_t store_cap, bool profile)
{
    int rc = batch_launch_tables(S, cus, spw, wgcu, qs, nq, st, store_cap, profile);
    if (rc || !S.walk_pending) return rc;
    FZ_TRY(hipEventSynchronize(S.tables_ev));
    return batch_launch_walk(S);
}

void batch_result(const BatchSlot &S, const fz_query &q, uint32_t i, fz_result *out)
{
    fz_result r;
    std::memset(&r, 0, sizeof r);
    r.min_len = UINT64_MAX;
    if (S.qst[i]) {
        r.status = S.qst[i];
        *out = r;
        return;
    }
    const FzBatchResult h = S.h_res[i];
    const FzBatchQuery &B = S.Q[i];
    const FzPlan &P = B.plan;
    r.total = B.sliced ? h.total : h.count;
    if (h.status & FZS_OVERFLOW) r.status = FZ_EOVERFLOW;
    else if (h.status & FZS_TOOBIG) r.status = FZ_E2BIG;
    else if (h.status & FZS_MISMATCH) r.status = FZ_EINTERNAL;
    if (r.status) {
        *out = r;
        return;
    }
    r.count = h.count;
    r.found = h.found ? 1 : 0;
    r.status = FZ_OK;
    if (P.mode == FZM_HIST) {
        const uint64_t *bins = S.h_bins + B.bins_off;
        uint64_t sum = 0;
        for (uint32_t l = 0; l < P.nbins; ++l) sum += bins[l];
        if (sum != h.count) {
            r.status = FZ_EINTERNAL;
        } else {
            std::memcpy(q.bins, bins, (size_t)P.nbins * 8);
            for (uint64_t l = P.nbins; l < q.nbins; ++l) q.bins[l] = 0;
            r.min_len = h.count ? h.min_len : UINT64_MAX;
            r.max_len = h.count ? h.max_len : 0;
        }
    } else if (P.mode == FZM_STORE) {
        r.written = h.count;
        if (h.count != std::min(h.total, P.max_tuples)) r.status = FZ_EINTERNAL;
        else if (h.total > P.max_tuples) r.status = FZ_TRUNCATED;
    } else if (B.sliced && h.count != h.total && !(P.mode == FZM_EXISTS && h.found)) {
        // without an early exit every slice ran to its end: all of Z
        r.status = FZ_EINTERNAL;
    }
    *out = r;
}

int do_batch(const fz_query *qs, fz_result *rs, uint32_t nq, void *stream)
{
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *cp;
    int rc = get_ctx(&cp);
    if (rc) return rc;
    Ctx &c = *cp;
    hipStream_t st = stream ? (hipStream_t)stream : c.stream;
    uint32_t spw, wgcu;
    current_knobs(&spw, &wgcu);
    rc = batch_launch(c.batch, c.cus, spw, wgcu, qs, nq, st, UINT64_MAX, true);
    if (rc) return rc;
    FZ_TRY(hipStreamSynchronize(st));
    prof_collect();
    for (uint32_t i = 0; i < nq; ++i) batch_result(c.batch, qs[i], i, &rs[i]);
    c.last.slices = c.batch.n_items;
    c.last_batch = true;
    c.last.rows = c.last.prefixes = c.last.elements = c.last.candidates = 0;
    if (g_prof && c.batch.n_items) {
        // walker statistics of the batch (profiling runs only: a readback
        // of every item's record)
        std::vector<FzSliceRec> recs(c.batch.n_items);
        FZ_TRY(hipMemcpy(recs.data(), c.batch.recs.p, recs.size() * sizeof(FzSliceRec),
                         hipMemcpyDeviceToHost));
        for (const FzSliceRec &r : recs) {
            c.last.rows += r.rows;
            c.last.prefixes += r.prefixes;
            c.last.elements += r.elements;
        }
        c.last.candidates = c.last.elements + c.last.prefixes;
    }
    return FZ_OK;
}


// ---------------------------------------------------------------------------
// Allocation-free count (fz_count_noalloc).  The count path of
// fz_count_stream, with every device buffer carved from one fixed array of
// this file instead of the library's grow-only buffers.  In host code the
// array's name only stands for the symbol: its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is ever passed to kernels.  Every call on a device reuses the
// same array and leaves its contents behind; the walk rewrites every word it
// reads (tables, bounds, control block and slice records are written by the
// kernels before use), so nothing needs clearing.  Calls are serialized per
// process and wait for their stream, so two calls never overlap on the array.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[FZ_NOALLOC_SCRATCH_BYTES];

struct NoAllocDev {
    bool ready = false;
    int cus = 0;
    uint8_t *ptr = nullptr; // device address of `scratch` on this device
};
NoAllocDev g_noalloc[kMaxDevices];

int noalloc_device(NoAllocDev **out)
{
    (void)hipGetLastError();
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return dev_err_at(e == hipSuccess ? hipErrorInvalidDevice : e, "hipGetDevice", __LINE__);
    }
    NoAllocDev &a = g_noalloc[dev];
    if (!a.ready) {
        int cus = 0;
        FZ_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        void *ptr = nullptr;
        FZ_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (ptr == nullptr) return dev_err_at(hipErrorInvalidSymbol, "hipGetSymbolAddress", __LINE__);
        a.cus = cus;
        a.ptr = (uint8_t *)ptr;
        a.ready = true;
    }
    *out = &a;
    return FZ_OK;
}

int do_count_noalloc(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count, void *stream)
{
    if (count == nullptr) return FZ_EINVAL;
    FzPlan P;
    int rc = make_walk_plan(n, g, d, FZM_COUNT, &P);
    if (rc) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    NoAllocDev *a;
    if ((rc = noalloc_device(&a))) return rc;
    Launch L;
    plan_launch(a->cus, P, L);
    P.host_slices = P.host_ppm = 0; // the device walks every slice here
    P.trail = 0;
    const ScratchSizes z = scratch_sizes(P, L);
    // 256-byte aligned pieces of the array, in a fixed order
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (std::max<size_t>(bytes, 8) + 255) & ~(size_t)255;
        return a->ptr + o;
    };
    FzBufs B;
    std::memset(&B, 0, sizeof B);
    B.S = (uint64_t *)take(z.S);
    B.C = (uint64_t *)take(z.C);
    B.restab = (int2 *)take(z.restab);
    B.bounds = (uint32_t *)take(z.bounds);
    B.base = (uint64_t *)take(z.base);
    B.recs = (FzSliceRec *)take(z.recs);
    B.ctl = (FzCtl *)take(z.ctl);
    B.dpart = (uint64_t *)take(z.dpart);
    uint64_t *pt = P.pair ? (uint64_t *)take(z.pt) : nullptr;
    if (off > (size_t)FZ_NOALLOC_SCRATCH_BYTES) {
        std::snprintf(g_err_msg, sizeof g_err_msg,
                      "fz_count_noalloc: the query needs %zu bytes of device scratch, the fixed "
                      "array holds %zu (FZ_NOALLOC_SCRATCH_BYTES)",
                      off, (size_t)FZ_NOALLOC_SCRATCH_BYTES);
        return FZ_E2BIG;
    }
    bind_pair(P, pt, B);
    const hipStream_t s = (hipStream_t)stream;
    if (!P.notab) FZ_TRY(fzk_launch_dp(P, B, s));
    FZ_TRY(fzk_launch_restab(P, B, s));
    FZ_TRY(P.notab ? fzk_launch_split(P, B, s) : fzk_launch_slices(P, B, s));
    FZ_TRY(fzk_launch_enum(P, B, L.nwg, s));
    FZ_TRY(fzk_launch_finalize(P, B, L.nwg, s));
    FzCtl h;
    FZ_TRY(hipMemcpyAsync(&h, B.ctl, sizeof(FzCtl), hipMemcpyDeviceToHost, s));
    FZ_TRY(hipStreamSynchronize(s));
    if (h.status & FZS_OVERFLOW) return FZ_EOVERFLOW;
    if ((h.status & FZS_MISMATCH) || h.count != h.total) return FZ_EINTERNAL;
    *count = h.count;
    return FZ_OK;
}

} // namespace fzh

using namespace fzh;

extern "C" {

int fz_batch(const fz_query *q, fz_result *r, uint32_t nq, void *stream)
{
    if ((q == nullptr || r == nullptr) && nq > 0) return FZ_EINVAL;
    if (nq == 0) return FZ_OK;
    return do_batch(q, r, nq, stream);
}


int fz_count(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count)
{
    return do_count(n, g, d, count, nullptr);
}

int fz_count_stream(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count, void *stream)
{
    return do_count(n, g, d, count, stream);
}

int fz_count_noalloc(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *count, void *stream)
{
    return do_count_noalloc(n, g, d, count, stream);
}

uint64_t fz_length_bins(uint64_t n, const uint32_t *g, uint32_t d)
{
    FzPlan P;
    if (make_plan(n, g, d, FZM_HIST, &P)) return 0;
    return P.nbins;
}

int fz_length_hist(uint64_t n, const uint32_t *g, uint32_t d, uint64_t *bins, uint64_t nbins,
                   uint64_t *min_len, uint64_t *max_len)
{
    if (bins == nullptr || min_len == nullptr || max_len == nullptr) return FZ_EINVAL;
    FzPlan P;
    int rc = make_walk_plan(n, g, d, FZM_HIST, &P);
    if (rc) return rc;
    if (nbins < P.nbins) return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *c;
    if ((rc = get_ctx(&c))) return rc;
    FzBufs B;
    Launch L;
    if ((rc = prepare(*c, P, B, L))) return rc;
    if ((rc = run_query(*c, P, B, L, c->stream))) return rc;
    const FzCtl &h = *c->host_ctl;
    if (h.count != h.total) return FZ_EINTERNAL;
    std::vector<uint64_t> tmp(P.nbins);
    FZ_TRY(hipMemcpy(tmp.data(), B.hist, (size_t)P.nbins * 8, hipMemcpyDeviceToHost));
    uint64_t lo = h.min_len, hi = h.max_len;
    if (!c->host_hist.empty()) { // the hybrid pool's host part
        for (uint32_t l = 0; l < P.nbins; ++l) tmp[l] += c->host_hist[l];
        lo = UINT64_MAX;
        hi = 0;
        for (uint32_t l = 0; l < P.nbins; ++l)
            if (tmp[l]) {
                lo = std::min<uint64_t>(lo, l);
                hi = l;
            }
    }
    uint64_t sum = 0;
    for (uint64_t v : tmp) sum += v;
    if (sum != h.count) return FZ_EINTERNAL;
    std::memcpy(bins, tmp.data(), (size_t)P.nbins * 8);
    for (uint64_t l = P.nbins; l < nbins; ++l) bins[l] = 0;
    *min_len = h.count ? lo : UINT64_MAX;
    *max_len = h.count ? hi : 0;
    return FZ_OK;
}

int fz_exists(uint64_t n, const uint32_t *g, uint32_t d, uint64_t target_len, int *found)
{
    if (found == nullptr) return FZ_EINVAL;
    FzPlan P;
    int rc = make_walk_plan(n, g, d, FZM_EXISTS, &P);
    if (rc) return rc;
    P.target_len = target_len;
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *c;
    if ((rc = get_ctx(&c))) return rc;
    FzBufs B;
    Launch L;
    if ((rc = prepare(*c, P, B, L))) return rc;
    if ((rc = run_query(*c, P, B, L, c->stream))) return rc;
    const FzCtl &h = *c->host_ctl;
    // Without a witness every slice ran to its end and must account for |Z|.
    if (!h.found && h.count != h.total) return FZ_EINTERNAL;
    *found = h.found ? 1 : 0;
    return FZ_OK;
}

int fz_enumerate(uint64_t n, const uint32_t *g, uint32_t d, uint32_t *out, uint64_t max_tuples,
                 uint64_t *total, uint64_t *written)
{
    return do_enumerate(n, g, d, out, false, max_tuples, total, written, nullptr);
}

int fz_enumerate_device(uint64_t n, const uint32_t *g, uint32_t d, uint32_t *d_out,
                        uint64_t max_tuples, uint64_t *total, uint64_t *written, void *stream)
{
    return do_enumerate(n, g, d, d_out, true, max_tuples, total, written, stream);
}

int fz_unrank(uint64_t n, const uint32_t *g, uint32_t d, const uint64_t *ranks, uint64_t nranks,
              uint32_t *out)
{
    if ((ranks == nullptr || out == nullptr) && nranks > 0) return FZ_EINVAL;
    FzPlan P;
    int rc = make_plan(n, g, d, FZM_COUNT, &P);
    if (rc) return rc;
    if (nranks == 0) return FZ_OK;
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *c;
    if ((rc = get_ctx(&c))) return rc;
    FzBufs B;
    Launch L;
    if ((rc = prepare(*c, P, B, L))) return rc;
    FZ_TRY(ensure(c->ranks, nranks * 8));
    FZ_TRY(ensure(c->rows_out, nranks * P.d_user * 4));
    hipStream_t s = c->stream;
    FZ_TRY(hipMemcpyAsync(c->ranks.p, ranks, nranks * 8, hipMemcpyHostToDevice, s));
    FZ_LAUNCH("dp", s, fzk_launch_dp(P, B, s));
    FZ_LAUNCH("slices", s, fzk_launch_slices(P, B, s)); // resets the control block
    FZ_LAUNCH("unrank", s,
              fzk_launch_unrank(P, B, (const uint64_t *)c->ranks.p, nranks,
                                (uint32_t *)c->rows_out.p, s));
    FZ_TRY(hipMemcpyAsync(c->host_ctl, B.ctl, sizeof(FzCtl), hipMemcpyDeviceToHost, s));
    FZ_TRY(hipStreamSynchronize(s));
    prof_collect();
    if (c->host_ctl->status & FZS_OVERFLOW) return FZ_EOVERFLOW;
    if (c->host_ctl->status & FZS_MISMATCH) return FZ_EINVAL;
    FZ_TRY(hipMemcpy(out, c->rows_out.p, nranks * P.d_user * 4, hipMemcpyDeviceToHost));
    return FZ_OK;
}

int fz_last_stats(fz_stats *out)
{
    if (out == nullptr) return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *c;
    int rc = get_ctx(&c);
    if (rc) return rc;
    *out = c->last;
    return FZ_OK;
}

int fz_last_slices(fz_slice_info *out, uint32_t cap, uint32_t *n_slices)
{
    if (n_slices == nullptr || (out == nullptr && cap > 0)) return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    Ctx *c;
    int rc = get_ctx(&c);
    if (rc) return rc;
    const uint32_t n = (uint32_t)c->last.slices;
    *n_slices = n;
    const uint32_t k = std::min(n, cap);
    if (k == 0) return FZ_OK;
    std::vector<FzSliceRec> tmp(k);
    const void *src = c->last_batch ? c->batch.recs.p : c->recs.p;
    FZ_TRY(hipMemcpy(tmp.data(), src, k * sizeof(FzSliceRec), hipMemcpyDeviceToHost));
    // a batch's items: (query, slice) from the staged item list
    std::vector<FzBatchJob> items;
    if (c->last_batch) {
        items.assign(k, FzBatchJob{0, 0});
        for (uint32_t q = 0; q < c->batch.nq; ++q) {
            const FzBatchQuery &B = c->batch.Q[q];
            if (!B.plan.d) continue;
            for (uint32_t j = 0; j < B.n_slices; ++j)
                if (B.item_off + j < k) items[B.item_off + j] = {q, j};
        }
    }
    for (uint32_t i = 0; i < k; ++i) {
        out[i].elements = tmp[i].elements;
        out[i].rows = tmp[i].rows;
        out[i].prefixes = tmp[i].prefixes;
        out[i].t_begin = tmp[i].t_begin;
        out[i].t_end = tmp[i].t_end;
        out[i].query = c->last_batch ? items[i].q : 0;
        out[i].slice = c->last_batch ? items[i].j : i;
    }
    return FZ_OK;
}

int fz_config_set(const char *key, int64_t value)
{
    if (key == nullptr || value < 0) return FZ_EINVAL;
    // (every knob is a size or weight up to 2^20 but the batch's least item
    // work, up to 2^30)
    if (value > (std::strcmp(key, "batch_min_item_work") == 0 ? (1 << 30) : (1 << 20)))
        return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    if (std::strcmp(key, "slices_per_wave") == 0) g_slices_per_wave = (uint32_t)value;
    else if (std::strcmp(key, "workgroups_per_cu") == 0) g_wg_per_cu = (uint32_t)value;
    else if (std::strcmp(key, "work_row") == 0) g_work_row = (uint32_t)value;
    else if (std::strcmp(key, "work_chunk") == 0) g_work_chunk = (uint32_t)value;
    else if (std::strcmp(key, "work_element") == 0) g_work_elem = (uint32_t)value;
    else if (std::strcmp(key, "skip_empty_rows") == 0 && value <= 2) g_prune_mode = (uint32_t)value;
    else if (std::strcmp(key, "walk_order") == 0 && value <= 1) g_walk_order = (uint32_t)value;
    else if (std::strcmp(key, "batch_graph") == 0 && value <= 1) g_batch_graph = (uint32_t)value;
    else if (std::strcmp(key, "pair_table") == 0 && value <= 2) g_pair_mode = (uint32_t)value;
    else if (std::strcmp(key, "min_slice_work") == 0) g_min_slice_work = (uint64_t)value;
    else if (std::strcmp(key, "variant") == 0 && value <= 1) g_variant = (uint32_t)value;
    else if (std::strcmp(key, "tables") == 0 && value <= 2) g_tables = (uint32_t)value;
    else if (std::strcmp(key, "host_threads") == 0 && value <= kMaxHostThreads)
        g_host_threads = (uint32_t)value;
    else if (std::strcmp(key, "host_share_ppm") == 0 && value <= 500000) g_host_ppm = (uint32_t)value;
    else if (std::strcmp(key, "trailing") == 0 && value <= 1) g_trailing = (uint32_t)value;
    else if (std::strcmp(key, "packed") == 0 && value <= 2) g_pack_mode = (uint32_t)value;
    else if (std::strcmp(key, "empty_row_test") == 0 && value <= 2) g_row_test = (uint32_t)value;
    else if (std::strcmp(key, "batch_min_item_work") == 0) g_batch_min_item = (uint64_t)value;
    else if (std::strcmp(key, "wave_bins32") == 0 && value <= 1) g_hist32 = (uint32_t)value;
    else if (std::strcmp(key, "wave_bins32_limit") == 0) g_hist32_limit = (uint64_t)value;
    else if (std::strcmp(key, "short_last_slices") == 0 && value <= 2) g_guided = (uint32_t)value;
    else if (std::strcmp(key, "wave_bins32_copies") == 0 &&
             (value == 0 || value == 1 || value == 2 || value == 4))
        g_hist32_copies = (uint32_t)value;
    else return FZ_EINVAL;
    return FZ_OK;
}

namespace {
// One timed run of the autotuner: wall milliseconds of a synchronous call.
int tune_run(const fz_query *q, uint32_t nq, std::vector<fz_result> &r, double *ms)
{
    const auto t0 = std::chrono::steady_clock::now();
    int rc = FZ_OK;
    if (nq > 1) {
        rc = fz_batch(q, r.data(), nq, nullptr);
    } else {
        const fz_query &x = q[0];
        uint64_t a = 0, b = 0;
        int f = 0;
        switch (x.mode) {
        case FZ_MODE_COUNT: rc = fz_count(x.n, x.g, x.d, &a); break;
        case FZ_MODE_HIST: rc = fz_length_hist(x.n, x.g, x.d, x.bins, x.nbins, &a, &b); break;
        case FZ_MODE_EXISTS: rc = fz_exists(x.n, x.g, x.d, x.target_len, &f); break;
        case FZ_MODE_STORE:
            rc = fz_enumerate_device(x.n, x.g, x.d, x.d_out, x.max_tuples, &a, &b, nullptr);
            break;
        default: rc = FZ_EINVAL;
        }
    }
    *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc < 0 ? rc : FZ_OK;
}
} // namespace

int fz_autotune(const fz_query *q, uint32_t nq, uint32_t reps, fz_tune_result *out)
{
    if (q == nullptr || out == nullptr || nq == 0 || reps == 0 || reps > 100) return FZ_EINVAL;
    static const uint32_t kSpw[] = {4, 8, 16, 32, 64};
    static const uint32_t kWg[] = {2, 4, 8};
    uint32_t save_spw, save_wg;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        save_spw = g_slices_per_wave;
        save_wg = g_wg_per_cu;
    }
    auto set = [](uint32_t spw, uint32_t wg) {
        std::lock_guard<std::mutex> lk(g_mu);
        g_slices_per_wave = spw;
        g_wg_per_cu = wg;
    };
    std::vector<fz_result> r(nq);
    auto median = [&](uint32_t spw, uint32_t wg, double *ms) -> int {
        set(spw, wg);
        double t;
        int rc = tune_run(q, nq, r, &t); // warm-up
        std::vector<double> v;
        for (uint32_t i = 0; rc == FZ_OK && i < reps; ++i) {
            rc = tune_run(q, nq, r, &t);
            v.push_back(t);
        }
        if (rc != FZ_OK) return rc;
        std::sort(v.begin(), v.end());
        *ms = v[v.size() / 2];
        return FZ_OK;
    };
    fz_tune_result best{};
    int rc = median(0, 0, &best.default_ms);
    // the defaults timed above: a batch's (nq > 1 runs one fz_batch) or a
    // single query's
    const uint32_t def_spw = nq > 1 ? kBatchSlicesPerWave : kDefaultSlicesPerWave;
    const uint32_t def_wg = nq > 1 ? kBatchWgPerCu : kDefaultWgPerCu;
    best.slices_per_wave = def_spw;
    best.workgroups_per_cu = def_wg;
    best.ms = best.default_ms;
    best.candidates = 1;
    for (uint32_t spw : kSpw)
        for (uint32_t wg : kWg) {
            if (rc != FZ_OK) break;
            if (spw == def_spw && wg == def_wg) continue;
            double ms = 0;
            rc = median(spw, wg, &ms);
            ++best.candidates;
            if (rc == FZ_OK && ms < best.ms) {
                best.ms = ms;
                best.slices_per_wave = spw;
                best.workgroups_per_cu = wg;
            }
        }
    if (rc != FZ_OK) {
        set(save_spw, save_wg);
        return rc;
    }
    set(best.slices_per_wave, best.workgroups_per_cu);
    *out = best;
    return FZ_OK;
}

int fz_profile_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof = on != 0;
    return FZ_OK;
}

int fz_profile_reset(void)
{
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof_stats.clear();
    return FZ_OK;
}

int fz_profile_read(const char *kernel, double *total_ms, uint64_t *launches)
{
    if (kernel == nullptr || total_ms == nullptr || launches == nullptr) return FZ_EINVAL;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_prof_stats.find(kernel);
    *total_ms = it == g_prof_stats.end() ? 0.0 : it->second.ms;
    *launches = it == g_prof_stats.end() ? 0 : it->second.n;
    return FZ_OK;
}

const char *fz_last_error(void)
{
    return g_err_msg;
}

const char *fz_strerror(int status)
{
    switch (status) {
    case FZ_OK: return "ok";
    case FZ_TRUNCATED: return "output truncated to max_tuples rows";
    case FZ_EINVAL: return "invalid argument";
    case FZ_EOVERFLOW: return "value out of range (n, generator or count too large)";
    case FZ_ENOMEM: return "out of device memory";
    case FZ_EDEVICE: return "HIP device error";
    case FZ_E2BIG:
        return "query too large (last generator above FZ_MAX_LAST_GEN, store above the "
               "server's tuple cap, or tables above its memory budget)";
    case FZ_EINTERNAL: return "internal self-check failed";
    default: return "unknown status";
    }
}

} // extern "C"
