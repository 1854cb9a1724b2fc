// fz_host.h -- host-side pieces shared by the libfz entry points (fz_api.hip)
// and the request server (fz_server.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "fz.h"
#include "fz_internal.h"

namespace fzh {

// Grow-only device allocation.
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
};
hipError_t ensure(DevBuf &b, size_t bytes);

// Records a failed HIP call for fz_last_error; FZ_ENOMEM or FZ_EDEVICE.
int dev_err_at(hipError_t e, const char *what, int line);

// Validation and normalization of one query (every limit of include/fz.h).
int make_plan(uint64_t n, const uint32_t *g, uint32_t d, uint32_t mode, FzPlan *P);

// Serializes the library's entry points and guards the tuning knobs.
extern std::mutex g_mu;

// One batch: device buffers, pinned host arrays the walker writes finished
// queries into (coherent, so the host may read them while the launch runs),
// and the plan of the batch last launched from it.  fz_batch uses one per
// device; a server owns one per launch slot.
struct BatchSlot {
    DevBuf meta, tables, restabs, bounds, base, recs, bins, res, cursor, totals;
    uint64_t *h_totals = nullptr; // pinned: C[0][n], S[0][n] of the queries with tables
    size_t h_totals_cap = 0;
    uint8_t *h_meta = nullptr;   // pinned staging of queries, jobs and items
    size_t h_meta_cap = 0;
    FzBatchResult *h_res = nullptr;
    uint32_t *h_done = nullptr;
    uint32_t h_cap = 0;          // queries h_res / h_done hold
    uint64_t *h_bins = nullptr;
    uint64_t h_bins_cap = 0;     // words
    std::vector<FzBatchQuery> Q;
    std::vector<int> qst;        // host validation status of each query
    uint32_t nq = 0, n_items = 0;
    // state kept between the two launch phases
    std::vector<double> work;
    std::vector<uint32_t> tabled;
    std::vector<uint32_t> pass_jobs, pass_off; // table jobs pass by pass (host copies)
    std::vector<uint32_t> small_ids;           // queries whose tables one workgroup builds
    FzBatchBufs B{};
    hipStream_t stream = nullptr;
    hipEvent_t tables_ev = nullptr; // recorded after the tables and their totals
    hipGraphExec_t walk_exec = nullptr; // phase 2 (slice bounds, walker) as a graph
    double slots = 0;
    uint32_t cus = 0, wgcu = 0, maxm = 0, max_du = 0, lds_bins = 0, bstride = 1;
    bool profile = false;
    bool walk_pending = false;      // phase 1 queued, phase 2 not yet
    // item order: false (fz_batch) the largest items first, for the shortest
    // whole batch; true (the server) the uncut queries first, so that small
    // queries finish at the start of the walk instead of after the large
    // ones' items have been taken
    bool small_first = false;
    void release();
};

// A batch is launched in two phases.  batch_launch_tables plans qs[0..nq)
// and queues the count and work tables, residue tables and the readback of
// each tabled query's modelled work on stream st, then records
// S.tables_ev (S.walk_pending).  Once that event has completed,
// batch_launch_walk cuts every query into slices by its work and queues the
// slice bounds and the persistent walker.  batch_launch does both, waiting
// in between.  Store queries with |Z| > store_cap are refused on the device
// (FZ_E2BIG).  Requires g_mu held when profile is true.  The slot's previous
// launch must have completed.
int batch_launch_tables(BatchSlot &S, int cus, uint32_t spw, uint32_t wgcu, const fz_query *qs,
                        uint32_t nq, hipStream_t st, uint64_t store_cap, bool profile);
int batch_launch_walk(BatchSlot &S);
int batch_launch(BatchSlot &S, int cus, uint32_t spw, uint32_t wgcu, const fz_query *qs,
                 uint32_t nq, hipStream_t st, uint64_t store_cap, bool profile);

// Result of query i of the slot's batch, once h_done[i] is set or the stream
// has completed (host-rejected queries have their status at once).  Copies
// histogram bins to q.bins.
void batch_result(const BatchSlot &S, const fz_query &q, uint32_t i, fz_result *r);

// Effective slices-per-wave and workgroups-per-CU knobs (g_mu held).
void current_knobs(uint32_t *spw, uint32_t *wgcu);

} // namespace fzh
