// batch.hip -- batching form: many independent rings advanced together, one
// launch per round over all running rings (k_batch_round), or one persistent
// launch with per-tile epoch counters (k_batch).  This file builds the work
// lists on the host and owns the host-buffer wrapper heat_solve_batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "heat_batch.h"
#include "heat_internal.h"

namespace heat {

static inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int batch_cells_per_lane(int precision, int64_t N) {
    return precision != HEAT_FP32C && N >= 65536 ? 64 : 32;
}

// Shortest target round length of a batch kernel class.  The tuning table's
// round length belongs to the plain kernel's shape for that ring length
// (often narrower lanes); a batch class runs its own lane width, and rounds
// much shorter than its window's natural depth only multiply launches and
// scheduling steps (measured on MI355X: the long binary64 rings of the
// serving mix at 64-step rounds doubled its latency at 1,000 requests/s).
// Tiles of 4 cooperating waves share the outer halo, so deeper rounds pay
// (as for the plain kernel, whose tuned binary64 shape is 4 waves and
// 250-step rounds).
static int64_t batch_min_steps_per_round(int K, int G) {
    if (G > 1) return 240;
    return K >= 64 ? 160 : 96;
}

bool batch_class_exists(int precision, int K, int G) {
    if (precision == HEAT_FP32C) return K == 32 && (G == 1 || G == 4);
    if (precision != HEAT_FP64 && precision != HEAT_FP32) return false;
    return (K == 32 && G == 1) || (K == 64 && (G == 1 || G == 4));
}

int describe_ring(const heat_ring &g, BatchRing *out, int K, int G, int T) {
    if (K == 0) K = batch_cells_per_lane(g.precision, g.N);
    if (G < 1 || G > 8 || (G > 1 && K < 16)) return fail(HEAT_EINVAL, "bad batch tile shape");
    // the deepest rounds this class's window allows
    const int64_t Tmax = (64 * (int64_t)K / 3) & ~int64_t(3);
    int64_t Ttarget = default_steps_per_round(g.N, g.precision);
    // binary64/binary32 results do not depend on the round length; the
    // compensated form's fixed length is kept (and always fits)
    if (g.precision != HEAT_FP32C)
        Ttarget = std::min(T > 0 ? (int64_t)T : std::max(Ttarget, batch_min_steps_per_round(K, G)),
                           Tmax);
    const int64_t Teff = balanced_steps_per_round(g.nt, Ttarget, g.precision);
    BatchRing R{};
    R.buf[0] = g.d_u;
    R.buf[1] = g.d_work;
    R.N = g.N;
    R.H = (int32_t)halo_cells(Teff, g.precision, K);
    R.T = (int32_t)Teff;
    R.W = window_tile_cells(K, R.H, G, G > 1 ? 4 : 0);
    R.tiles = (g.N + R.W - 1) / R.W;
    R.r = g.r;
    R.nt = g.nt;
    const int64_t rounds = g.nt > 0 ? (g.nt + Teff - 1) / Teff : 0;
    if (rounds > (int64_t)1 << 30) return fail(HEAT_EINVAL, "too many rounds");
    if (R.tiles * 64 * G > MAX_GRID_THREADS) return fail(HEAT_EINVAL, "ring too long for one launch");
    R.rounds = (int32_t)rounds;
    R.copy_round = (int32_t)(rounds & 1);
    R.vec_ok = aligned16(g.d_u) && aligned16(g.d_work);
    R.flag_base = 0;
    R.round0 = 0;
    R.K = K;
    R.G = G;
    *out = R;
    return HEAT_OK;
}

int describe_ring_batch(const heat_ring &g, BatchRing *out) {
    int tK = 0, tG = 0, tT = 0;
    if (tuned_batch_class(g.N, g.precision, &tK, &tG, &tT) &&
        batch_class_exists(g.precision, tK, tG) && describe_ring(g, out, tK, tG, tT) == HEAT_OK)
        return HEAT_OK;
    return describe_ring_rule(g, out);
}

int describe_ring_rule(const heat_ring &g, BatchRing *out) {
    const int K = batch_cells_per_lane(g.precision, g.N);
    int rc = describe_ring(g, out, K, 1);
    // the 4-wave classes: binary64 and binary32 at 64-cell lanes, compensated
    // binary32 at 32
    const bool has_x = (g.precision != HEAT_FP32C && K == 64) || g.precision == HEAT_FP32C;
    if (rc || !has_x || g.nt == 0) return rc;
    // Cost in wave-steps: every tile costs its waves x (steps + a per-round
    // overhead for loading and storing the window, about 4 steps' worth);
    // the exchange's own steps cost about 1 % more.
    BatchRing X;
    if (describe_ring(g, &X, K, 4)) return HEAT_OK;   // keep the lone shape
    const double over = 4.0;
    auto cost = [&](const BatchRing &R) {
        const double rounds = std::ceil((double)g.nt / R.T);
        return (double)R.tiles * R.G * ((double)g.nt + over * rounds) * (R.G > 1 ? 1.01 : 1.0);
    };
    if (cost(X) < cost(*out)) *out = X;
    return HEAT_OK;
}

// Host-side work list over rings of one precision.
static inline int32_t remaining_rounds(const BatchRing &R) {
    return R.rounds + R.copy_round - R.round0;
}

int32_t scheduled_rounds(const BatchRing &R, int32_t cap, int32_t tick_steps) {
    const int32_t n = remaining_rounds(R);
    int32_t c = cap;
    if (tick_steps > 0) c = std::max<int32_t>(1, (tick_steps + R.T - 1) / std::max<int32_t>(R.T, 1));
    return c > 0 ? std::min(n, c) : n;
}

int BatchLaunch::build(const std::vector<BatchRing> &rings_in, int precision, int32_t cap,
                       int32_t tick_steps) {
    precision_ = precision;
    K_ = rings_in.empty() ? 32 : rings_in[0].K;
    G_ = rings_in.empty() ? 1 : rings_in[0].G;
    rings_.clear();
    for (const BatchRing &R : rings_in)
        if (remaining_rounds(R) > 0) rings_.push_back(R);
    // most scheduled rounds first (remaining rounds incl. copy-back, capped),
    // stable for determinism
    auto sched = [&](const BatchRing &R) { return scheduled_rounds(R, cap, tick_steps); };
    std::stable_sort(rings_.begin(), rings_.end(), [&](const BatchRing &a, const BatchRing &b) {
        return sched(a) > sched(b);
    });
    const size_t n = rings_.size();
    tile_prefix_.assign(n + 1, 0);
    int64_t flags = 0;
    for (size_t i = 0; i < n; ++i) {
        rings_[i].flag_base = flags;
        flags += rings_[i].tiles;
        tile_prefix_[i + 1] = tile_prefix_[i] + rings_[i].tiles;
    }
    nflags_ = flags;
    max_rounds_ = n ? sched(rings_[0]) : 0;
    active_.assign(max_rounds_, 0);
    round_start_.assign(max_rounds_ + 1, 0);
    // rings are sorted by scheduled rounds, so the rings alive in round k form a prefix
    size_t alive = n;
    for (int32_t k = 0; k < max_rounds_; ++k) {
        while (alive > 0 && sched(rings_[alive - 1]) <= k) --alive;
        active_[k] = (int32_t)alive;
        round_start_[k + 1] = round_start_[k] + tile_prefix_[alive];
    }
    total_items_ = max_rounds_ ? round_start_[max_rounds_] : 0;
    if (tile_prefix_[n] * 64 * G_ > MAX_GRID_THREADS)
        return fail(HEAT_EINVAL, "batch has more tiles than one launch can hold");
    return HEAT_OK;
}

size_t BatchLaunch::device_bytes() const {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    return al(rings_.size() * sizeof(BatchRing)) + al(tile_prefix_.size() * 8) +
           al(round_start_.size() * 8) + al(active_.size() * 4) + al((size_t)nflags_ * 4) + 256;
}

int BatchLaunch::enqueue(void *dev_mem, hipStream_t st, bool persistent, bool graph) {
    if (total_items_ == 0) return HEAT_OK;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    char *p = (char *)dev_mem;
    BatchPlanDev d{};
    d.rings = (const BatchRing *)p;
    HEAT_HIP(hipMemcpyAsync(p, rings_.data(), rings_.size() * sizeof(BatchRing),
                            hipMemcpyHostToDevice, st));
    p += al(rings_.size() * sizeof(BatchRing));
    d.tile_prefix = (const int64_t *)p;
    HEAT_HIP(hipMemcpyAsync(p, tile_prefix_.data(), tile_prefix_.size() * 8, hipMemcpyHostToDevice,
                            st));
    p += al(tile_prefix_.size() * 8);
    if (!persistent) {
        // one launch per round; the kernel boundary is the round barrier
        const int wpg = 4;
        if (!graph) {
            for (int32_t k = 0; k < max_rounds_; ++k)
                HEAT_HIP(launch_batch_round(precision_, K_, G_, d.rings, d.tile_prefix, k, active_[k],
                                            tile_prefix_[active_[k]], wpg, st));
            return HEAT_OK;
        }
        // Capture the round launches on a private stream (the caller's may be
        // the legacy default stream, which cannot capture), then replay the
        // graph on the caller's stream after the table uploads above.
        hipStream_t cs = nullptr;
        HEAT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        for (int32_t k = 0; k < max_rounds_ && e == hipSuccess; ++k)
            e = launch_batch_round(precision_, K_, G_, d.rings, d.tile_prefix, k, active_[k],
                                   tile_prefix_[active_[k]], wpg, cs);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&graph_exec_, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        (void)hipStreamDestroy(cs);
        if (e == hipSuccess) e = hipGraphLaunch(graph_exec_, st);
        if (e != hipSuccess) return fail_hip(e, "batch graph");
        return HEAT_OK;
    }
    // the persistent kernel always runs every ring from its first round to its last
    for (const BatchRing &R : rings_)
        if (R.round0 != 0 || max_rounds_ != remaining_rounds(rings_[0]))
            return fail(HEAT_EINVAL, "persistent batch needs whole runs");
    d.round_start = (const int64_t *)p;
    HEAT_HIP(hipMemcpyAsync(p, round_start_.data(), round_start_.size() * 8,
                            hipMemcpyHostToDevice, st));
    p += al(round_start_.size() * 8);
    d.active = (const int32_t *)p;
    HEAT_HIP(hipMemcpyAsync(p, active_.data(), active_.size() * 4, hipMemcpyHostToDevice, st));
    p += al(active_.size() * 4);
    d.flags = (uint32_t *)p;
    p += al((size_t)nflags_ * 4);
    d.work = (unsigned long long *)p;           // 8 bytes
    d.status = (uint32_t *)(p + 8);             // 4 bytes
    // epoch counters, work counter and status start at zero (fill kernel, no memset)
    HEAT_HIP(launch_fill_u32(d.flags, nflags_, 0u, st));
    HEAT_HIP(launch_fill_u32((uint32_t *)p, 4, 0u, st));
    d.total_items = total_items_;
    d.max_rounds = max_rounds_;
    d.chunk = 4;
    d.spin_limit = (int64_t)1 << 22;
    status_dev_ = d.status;
    const int wpg = 4;
    int grid = 0;
    int rc = batch_grid_size(precision_, K_, wpg, &grid);
    if (rc) return rc;
    HEAT_HIP(launch_batch(precision_, K_, d, grid, wpg, st));
    return HEAT_OK;
}

size_t BatchLaunch::table_bytes() const {
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    return al(rings_.size() * sizeof(BatchRing)) + al(tile_prefix_.size() * 8);
}

int BatchLaunch::enqueue_rounds(void *dev_tables, void *host_staging, hipStream_t st) {
    if (total_items_ == 0) return HEAT_OK;
    auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
    char *h = (char *)host_staging;
    std::memcpy(h, rings_.data(), rings_.size() * sizeof(BatchRing));
    const size_t off = al(rings_.size() * sizeof(BatchRing));
    std::memcpy(h + off, tile_prefix_.data(), tile_prefix_.size() * 8);
    HEAT_HIP(hipMemcpyAsync(dev_tables, host_staging, table_bytes(), hipMemcpyHostToDevice, st));
    const BatchRing *rings = (const BatchRing *)dev_tables;
    const int64_t *prefix = (const int64_t *)((char *)dev_tables + off);
    for (int32_t k = 0; k < max_rounds_; ++k)
        HEAT_HIP(launch_batch_round(precision_, K_, G_, rings, prefix, k, active_[k],
                                    tile_prefix_[active_[k]], 4, st));
    return HEAT_OK;
}

void BatchLaunch::release() {
    if (graph_exec_) (void)hipGraphExecDestroy(graph_exec_);
    graph_exec_ = nullptr;
}

int BatchLaunch::check_status(hipStream_t st) {
    if (!status_dev_) return HEAT_OK;
    uint32_t s = 0;
    HEAT_HIP(hipMemcpyAsync(&s, status_dev_, 4, hipMemcpyDeviceToHost, st));
    HEAT_HIP(hipStreamSynchronize(st));
    if (s) return fail(HEAT_EDEVICE, "fused batch launch: a dependency wait timed out");
    return HEAT_OK;
}

int validate_ring(const heat_ring &g) {
    if (g.N < 1) return fail(HEAT_EINVAL, "ring N must be >= 1");
    if (g.nt < 0) return fail(HEAT_EINVAL, "ring nt must be >= 0");
    if (!std::isfinite(g.r) || g.r < 0.0 || g.r > 0.5)
        return fail(HEAT_EINVAL, "ring r must be finite and in [0, 1/2] (got %g)", g.r);
    if (g.precision != HEAT_FP64 && g.precision != HEAT_FP32 && g.precision != HEAT_FP32C)
        return fail(HEAT_EINVAL, "unknown precision %d", g.precision);
    if (g.nparts < 1 || (int64_t)g.nparts > g.N) return fail(HEAT_EINVAL, "nparts must be in [1, N]");
    if (!g.d_u || (g.nt > 0 && !g.d_work)) return fail(HEAT_EINVAL, "ring buffer is NULL");
    return HEAT_OK;
}

// Enqueue the launches of every kernel class present (one launch per round
// of each (precision, cells-per-lane, waves-per-tile) class, or one
// persistent launch per class with HEAT_BATCH_PERSISTENT), all on `st`.
int batch_dev_enqueue(const heat_ring *rings, int32_t count, hipStream_t st,
                      std::vector<BatchLaunch> &launches, void **dev_mem_out, int32_t flags) {
    *dev_mem_out = nullptr;
    // one launch sequence per (precision, K class); the persistent kernel
    // exists for 32-cell lanes only
    const bool persistent = (flags & HEAT_BATCH_PERSISTENT) != 0;
    // classes: [precision][32-cell lanes, 64-cell lanes, 64-cell lanes x 4 waves per tile]
    std::vector<BatchRing> groups[3][3];
    for (int32_t i = 0; i < count; ++i) {
        BatchRing R;
        int rc = persistent ? describe_ring(rings[i], &R, 32) : describe_ring_batch(rings[i], &R);
        if (rc) return rc;
        groups[rings[i].precision][R.G > 1 ? 2 : (R.K == 64)].push_back(R);
    }
    launches.clear();
    size_t total = 0;
    for (int prec = 0; prec < 3; ++prec)
        for (int cls = 0; cls < 3; ++cls) {
            if (groups[prec][cls].empty()) continue;
            launches.emplace_back();
            int rc = launches.back().build(groups[prec][cls], prec);
            if (rc) return rc;
            total += launches.back().device_bytes();
        }
    if (total == 0) return HEAT_OK;
    int rc = device_pool_setup();
    if (rc) return rc;
    void *mem = nullptr;
    HEAT_HIP(hipMallocAsync(&mem, total, st));
    *dev_mem_out = mem;
    char *p = (char *)mem;
    for (BatchLaunch &L : launches) {
        rc = L.enqueue(p, st, (flags & HEAT_BATCH_PERSISTENT) != 0, (flags & HEAT_BATCH_GRAPH) != 0);
        if (rc) return rc;
        p += L.device_bytes();
    }
    return HEAT_OK;
}

int batch_run_class(const heat_ring *rings, int32_t count, hipStream_t st, int K, int G, int T) {
    if (count < 1) return HEAT_OK;
    // K = 0: every ring in the class the rule picks for it (classes grouped
    // as heat_solve_batch_dev groups them)
    std::vector<BatchRing> groups[3];
    for (int32_t i = 0; i < count; ++i) {
        if (rings[i].precision != rings[0].precision)
            return fail(HEAT_EINVAL, "rings of one precision only");
        BatchRing R;
        int rc;
        if (K == 0) {
            rc = describe_ring_rule(rings[i], &R);
        } else {
            if (!batch_class_exists(rings[i].precision, K, G))
                return fail(HEAT_EINVAL, "no batch kernel class K %d G %d for precision %d", K, G,
                            rings[i].precision);
            rc = describe_ring(rings[i], &R, K, G, T);
        }
        if (rc) return rc;
        groups[R.G > 1 ? 2 : (R.K == 64)].push_back(R);
    }
    std::vector<BatchLaunch> launches;
    size_t bytes = 0;
    for (auto &g : groups) {
        if (g.empty()) continue;
        launches.emplace_back();
        int rc = launches.back().build(g, rings[0].precision);
        if (rc) return rc;
        bytes += launches.back().device_bytes();
    }
    int rc = device_pool_setup();
    if (rc) return rc;
    void *mem = nullptr;
    HEAT_HIP(hipMallocAsync(&mem, bytes, st));
    char *p = (char *)mem;
    for (BatchLaunch &L : launches) {
        if (!rc) rc = L.enqueue(p, st, false, false);
        p += L.device_bytes();
    }
    const hipError_t e = hipStreamSynchronize(st);
    (void)hipFreeAsync(mem, st);
    if (!rc && e != hipSuccess) rc = fail_hip(e, "hipStreamSynchronize");
    return rc;
}

}  // namespace heat

using namespace heat;

extern "C" {

int heat_solve_batch_dev(const heat_ring *rings, int32_t count, void *hip_stream, int32_t flags) {
    if (count < 0 || (count > 0 && !rings)) return fail(HEAT_EINVAL, "bad ring array");
    if (flags & ~(HEAT_BATCH_WAIT | HEAT_BATCH_PERSISTENT | HEAT_BATCH_GRAPH))
        return fail(HEAT_EINVAL, "unknown batch flags 0x%x", flags);
    if ((flags & HEAT_BATCH_GRAPH) && !(flags & HEAT_BATCH_WAIT))
        return fail(HEAT_EINVAL, "HEAT_BATCH_GRAPH needs HEAT_BATCH_WAIT");
    // the persistent launch reports a timed-out dependency wait through a
    // status word that only a waiting call reads back
    if ((flags & HEAT_BATCH_PERSISTENT) && !(flags & HEAT_BATCH_WAIT))
        return fail(HEAT_EINVAL, "HEAT_BATCH_PERSISTENT needs HEAT_BATCH_WAIT");
    for (int32_t i = 0; i < count; ++i) {
        int rc = validate_ring(rings[i]);
        if (rc) return fail(rc, "ring %d: %s", i, heat_last_error());
    }
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<BatchLaunch> launches;
    void *mem = nullptr;
    int rc = batch_dev_enqueue(rings, count, st, launches, &mem, flags);
    if (flags & HEAT_BATCH_WAIT) {
        for (BatchLaunch &L : launches) {
            int rc2 = L.check_status(st);
            if (!rc) rc = rc2;
        }
        hipError_t e = hipStreamSynchronize(st);
        if (!rc && e != hipSuccess) rc = fail_hip(e, "hipStreamSynchronize");
        for (BatchLaunch &L : launches) L.release();
    }
    if (mem) (void)hipFreeAsync(mem, st);
    return rc;
}

int heat_solve_batch(heat_problem *probs, int32_t count) {
    if (count < 0 || (count > 0 && !probs)) return fail(HEAT_EINVAL, "bad problem array");
    int first = HEAT_OK;
    std::vector<int> ok(count, 0);
    for (int32_t i = 0; i < count; ++i) {
        heat_problem &p = probs[i];
        heat_ring g{p.N, p.nt, p.r, p.precision, p.nparts, (void *)1, (void *)1};
        int rc = validate_ring(g);
        if (!rc && (!p.u0 || !p.u_out)) rc = fail(HEAT_EINVAL, "u0/u_out is NULL");
        if (!rc && !std::isfinite(p.shift)) rc = fail(HEAT_EINVAL, "shift must be finite");
        p.status = rc;
        if (rc && first == HEAT_OK) first = rc;
        ok[i] = rc == HEAT_OK;
    }
    hipStream_t st = nullptr;
    HEAT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    int rc = device_pool_setup();
    std::vector<void *> allocs;
    std::vector<heat_ring> rings;
    std::vector<int> idx;
    double *sums = nullptr;   // device: 2 per problem + partials
    auto cleanup = [&]() {
        for (void *a : allocs) (void)hipFreeAsync(a, st);
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    };
    if (rc) {
        cleanup();
        return rc;
    }
    // stage in: binary64 host values -> device state (rounded for FP32 forms);
    // the copies of all problems go through the staging together
    std::vector<StageSeg> segs;
    for (int32_t i = 0; i < count && !rc; ++i) {
        if (!ok[i]) continue;
        heat_problem &p = probs[i];
        const size_t es = storage_bytes(p.precision);
        void *a = nullptr, *b = nullptr;
        hipError_t e = hipMallocAsync(&a, (size_t)p.N * es, st);
        if (e == hipSuccess) {
            allocs.push_back(a);
            e = hipMallocAsync(&b, (size_t)p.N * std::max<size_t>(es, 8), st);
        }
        if (e == hipSuccess) allocs.push_back(b);
        if (e != hipSuccess) {
            rc = fail_hip(e, "hipMallocAsync(batch state)");
            break;
        }
        segs.push_back(StageSeg{p.precision == HEAT_FP64 ? a : b, (void *)p.u0, (size_t)p.N * 8});
        rings.push_back(heat_ring{p.N, p.nt, p.r, p.precision, p.nparts, a, b});
        idx.push_back(i);
    }
    if (!rc) rc = stage_copies(true, segs.data(), segs.size(), st);
    for (size_t j = 0; j < rings.size() && !rc; ++j) {
        if (rings[j].precision == HEAT_FP64) continue;
        hipError_t e = launch_f64_to_f32((const double *)rings[j].d_work, (float *)rings[j].d_u,
                                         rings[j].N, st, probs[idx[j]].shift);
        if (e != hipSuccess) rc = fail_hip(e, "stage-in");
    }
    if (!rc) {
        hipError_t e = hipMallocAsync((void **)&sums, (2 * rings.size() + SUM_BLOCKS + 1) * 8, st);
        if (e != hipSuccess) rc = fail_hip(e, "hipMallocAsync(sums)");
        else allocs.push_back(sums);
    }
    double *partial = sums ? sums + 2 * rings.size() : nullptr;
    for (size_t j = 0; j < rings.size() && !rc; ++j) {
        hipError_t e = launch_sum(rings[j].precision, rings[j].d_u, rings[j].N, partial, sums + 2 * j, st);
        if (e != hipSuccess) rc = fail_hip(e, "sum0");
    }
    std::vector<BatchLaunch> launches;
    void *mem = nullptr;
    if (!rc) {
        rc = batch_dev_enqueue(rings.data(), (int32_t)rings.size(), st, launches, &mem, 0);
        if (mem) allocs.push_back(mem);
    }
    for (size_t j = 0; j < rings.size() && !rc; ++j) {
        hipError_t e = launch_sum(rings[j].precision, rings[j].d_u, rings[j].N, partial,
                                  sums + 2 * j + 1, st);
        if (e != hipSuccess) rc = fail_hip(e, "sum_nt");
    }
    // stage out (FP32 forms are widened exactly into the scratch buffer first)
    segs.clear();
    for (size_t j = 0; j < rings.size() && !rc; ++j) {
        heat_problem &p = probs[idx[j]];
        if (p.precision != HEAT_FP64) {
            hipError_t e = launch_f32_to_f64((const float *)rings[j].d_u,
                                             (double *)rings[j].d_work, p.N, st, p.shift);
            if (e != hipSuccess) rc = fail_hip(e, "stage-out");
        }
        segs.push_back(StageSeg{p.precision == HEAT_FP64 ? rings[j].d_u : rings[j].d_work,
                                p.u_out, (size_t)p.N * 8});
    }
    if (!rc)
        for (BatchLaunch &L : launches) {
            rc = L.check_status(st);
            if (rc) break;
        }
    if (!rc) rc = stage_copies(false, segs.data(), segs.size(), st);
    std::vector<double> hs(2 * rings.size());
    if (!rc && !rings.empty()) {
        hipError_t e = hipMemcpyAsync(hs.data(), sums, hs.size() * 8, hipMemcpyDeviceToHost, st);
        if (e != hipSuccess) rc = fail_hip(e, "sums D2H");
    }
    if (!rc) {
        hipError_t e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail_hip(e, "hipStreamSynchronize");
    }
    for (size_t j = 0; j < rings.size(); ++j) {
        heat_problem &p = probs[idx[j]];
        p.status = rc;
        if (!rc) {
            // sums of the stored offsets, plus N*shift for the shifted forms
            const double base = p.precision == HEAT_FP64 ? 0.0 : (double)p.N * p.shift;
            p.sum0 = base + hs[2 * j];
            p.sum_nt = base + hs[2 * j + 1];
        }
    }
    cleanup();
    if (rc) return rc;
    return first;
}

}  // extern "C"
