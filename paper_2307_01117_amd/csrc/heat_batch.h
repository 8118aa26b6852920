// heat_batch.h -- host-side work list of a fused batch launch (shared by the
// batching form and the server).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "heat_internal.h"

namespace heat {

// Cells per lane of the round kernel that runs a ring in the batching form:
// long binary64 rings take 64-cell lanes (half the halo overhead),
// everything else 32.  (The server runs all rings with 32-cell lanes.)
int batch_cells_per_lane(int precision, int64_t N);
int validate_ring(const heat_ring &g);
// Geometry of one ring in a batch: the tuned round length for its size,
// raised to the kernel class's minimum (binary64/binary32) and balanced into
// equal rounds like the plain planner; K = 0 picks batch_cells_per_lane.
// G > 1: G waves share each tile and swap edges through LDS (K >= 16).
// T > 0 (binary64/binary32): target round length instead of that rule
// (capped by the window); the compensated form keeps its fixed length.
int describe_ring(const heat_ring &g, BatchRing *out, int K = 0, int G = 1, int T = 0);
// Batching form's shape for a ring: the class the batch autotuner picked for
// the ring's precision and length decade (tune.hip), else 32- or 64-cell
// lanes, and for long rings 4 waves per tile when that costs fewer
// wave-steps.
int describe_ring_batch(const heat_ring &g, BatchRing *out);
// The rule describe_ring_batch falls back to (no tuned class).
int describe_ring_rule(const heat_ring &g, BatchRing *out);
// Whether a batch kernel class (precision, K, G) is built.
bool batch_class_exists(int precision, int K, int G);
// Advance the rings (all of one precision) on st in one forced class (K, G,
// target round length T), or with K = 0 each in the class the rule picks;
// one launch per round and class; blocking.  For the batch autotuner.
int batch_run_class(const heat_ring *rings, int32_t count, hipStream_t st, int K, int G, int T);
// The batch autotuner's pick for (precision, length decade of N), if any.
bool tuned_batch_class(int64_t N, int precision, int *K, int *G, int *T);

// Rounds a ring advances in one scheduling step: its remaining rounds
// (copy-back included), at most `cap` (0 = no cap) or, with tick_steps > 0,
// at most the rounds that cover tick_steps steps (at least one).
int32_t scheduled_rounds(const BatchRing &R, int32_t cap, int32_t tick_steps);

class BatchLaunch {
  public:
    // Sort rings (all of one precision and one K class) by the rounds they
    // are scheduled for (scheduled_rounds), most first, and number the work
    // items round-major; each ring starts at its own round0.
    int build(const std::vector<BatchRing> &rings, int precision, int32_t max_rounds = 0,
              int32_t tick_steps = 0);
    // Rings as scheduled (sorted), and the number of rounds each one advances.
    const std::vector<BatchRing> &rings() const { return rings_; }
    int32_t rounds_scheduled() const { return max_rounds_; }
    // Device bytes for tables, epoch counters, work counter and status word.
    size_t device_bytes() const;
    // Upload tables into dev_mem (device_bytes() bytes) and enqueue the work
    // on st: one launch per round (default; `graph` captures those launches
    // in a hipGraph and replays it), or the flag-synchronised persistent
    // kernel (`persistent`).
    int enqueue(void *dev_mem, hipStream_t st, bool persistent, bool graph);
    // Release a captured graph (call after the stream has been synchronised).
    void release();
    // Bytes of the round tables (rings + tile prefix) for enqueue_rounds.
    size_t table_bytes() const;
    // Copy the round tables through `host_staging` (pinned, table_bytes())
    // into `dev_tables` and launch the scheduled rounds on st.  The staging
    // area must stay untouched until st has passed this point.
    int enqueue_rounds(void *dev_tables, void *host_staging, hipStream_t st);
    // Wait for st and report a timed-out dependency wait, if any.
    int check_status(hipStream_t st);
    int64_t total_items() const { return total_items_; }

  private:
    int precision_ = 0;
    int K_ = 16;
    int G_ = 1;
    std::vector<BatchRing> rings_;
    std::vector<int64_t> tile_prefix_;
    std::vector<int64_t> round_start_;
    std::vector<int32_t> active_;
    int64_t nflags_ = 0;
    int32_t max_rounds_ = 0;
    int64_t total_items_ = 0;
    uint32_t *status_dev_ = nullptr;
    hipGraphExec_t graph_exec_ = nullptr;
};

int batch_dev_enqueue(const heat_ring *rings, int32_t count, hipStream_t st,
                      std::vector<BatchLaunch> &launches, void **dev_mem_out, int32_t flags);

}  // namespace heat
