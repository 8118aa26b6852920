// runtime.hip -- C ABI of the heat-stencil library: validation, planning,
// the plain / device / batch forms and the checksum.  Kernels live in
// kernels.hip, the serving loop in server.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <thread>
#include <vector>

#include "heat_internal.h"

namespace heat {

// ================================================================== errors

static thread_local char g_err[512] = "";

int fail(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

int fail_hip(hipError_t e, const char *what) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(HEAT_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(HEAT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ================================================================ planning

// Planner defaults come from the tuning table (tune.hip): K, target T,
// waves per group and register form per (precision, log10 N bucket).
//
// Steps per round.  binary64 and plain binary32 results do not depend on it
// (only speed does), so the planner may rebalance it (see make_plan); for the
// compensated form it sets where u + e is folded to binary32, so it is a
// fixed constant, part of the definition of that form's result.
constexpr int FP32C_STEPS_PER_ROUND = 64;

int default_steps_per_round(int64_t N, int precision) {
    if (precision == HEAT_FP32C) return FP32C_STEPS_PER_ROUND;
    int K, T, wpg, form, xchg;
    tuned_shape(N, precision, &K, &T, &wpg, &form, &xchg);
    return T;
}

int default_cells_per_lane(int64_t N, int precision) {
    int K, T, wpg, form, xchg;
    tuned_shape(N, precision, &K, &T, &wpg, &form, &xchg);
    return K;
}

int default_register_form(int64_t N, int precision) {
    int K, T, wpg, form, xchg;
    tuned_shape(N, precision, &K, &T, &wpg, &form, &xchg);
    return form;
}

static int default_waves_per_group(int64_t N, int precision) {
    int K, T, wpg, form, xchg;
    tuned_shape(N, precision, &K, &T, &wpg, &form, &xchg);
    return wpg;
}

static int default_exchange(int64_t N, int precision) {
    int K, T, wpg, form, xchg;
    tuned_shape(N, precision, &K, &T, &wpg, &form, &xchg);
    return xchg;
}

int64_t balanced_steps_per_round(int64_t nt, int64_t T, int precision) {
    // a run shorter than one round is a single round of nt steps
    int64_t Teff = nt > 0 ? std::min<int64_t>(T, nt) : 1;
    if (precision != HEAT_FP32C && nt >= 2) {
        // Result-neutral rebalancing (binary64 and plain binary32 only): an
        // even number of equal rounds, so the state ends in the caller's
        // buffer (no copy-back) and no round is a short remainder.
        int64_t R = (nt + Teff - 1) / Teff;
        if (R & 1) ++R;
        Teff = (nt + R - 1) / R;
    }
    return Teff;
}

static inline int64_t ceil4(int64_t x) { return (x + 3) & ~int64_t(3); }

int halo_cells(int64_t steps, int precision, int K) {
    // Windows start H cells left of their tile and tiles are W = 64K - 2H
    // long, so an H that is a multiple of one 128-byte line keeps every
    // lane's K-cell run on whole cache lines.  Fall back to a multiple of 4
    // (16-byte groups) if the line-aligned halo would be too deep.
    const int64_t line = 128 / (int64_t)storage_bytes(precision);
    int64_t H = (steps + line - 1) / line * line;
    if (3 * H > 64 * (int64_t)K) H = ceil4(steps);
    return (int)H;
}

static int check_problem(int64_t N, int32_t nparts, double r, int64_t nt, int precision) {
    if (N < 1) return fail(HEAT_EINVAL, "N must be >= 1 (got %lld)", (long long)N);
    if (N > (int64_t(1) << 40)) return fail(HEAT_EINVAL, "N too large (%lld)", (long long)N);
    if (nparts < 1 || (int64_t)nparts > N)
        return fail(HEAT_EINVAL, "nparts must be in [1, N] (got %d for N=%lld)", nparts,
                    (long long)N);
    if (nt < 0) return fail(HEAT_EINVAL, "nt must be >= 0 (got %lld)", (long long)nt);
    if (!std::isfinite(r) || r < 0.0 || r > 0.5)
        return fail(HEAT_EINVAL, "r must be finite and in [0, 1/2] (got %g)", r);
    if (precision != HEAT_FP64 && precision != HEAT_FP32 && precision != HEAT_FP32C)
        return fail(HEAT_EINVAL, "unknown precision %d", precision);
    return HEAT_OK;
}


constexpr int FORM_INPLACE_ID = 1;   // register_form of the in-place sweeps

int make_plan(int64_t N, int64_t nt, int precision, const heat_config *cfg, Plan *p) {
    heat_config c{};
    if (cfg) c = *cfg;
    Plan q;
    q.wpg = c.waves_per_group ? c.waves_per_group : default_waves_per_group(N, precision);
    if (q.wpg < 1 || q.wpg > 8)
        return fail(HEAT_EINVAL, "waves_per_group must be in [1, 8] (got %d)", q.wpg);
    int kernel = c.kernel ? c.kernel : HEAT_KERNEL_TB;
    if (kernel != HEAT_KERNEL_STEP && kernel != HEAT_KERNEL_TB && kernel != HEAT_KERNEL_RESIDENT)
        return fail(HEAT_EINVAL, "unknown kernel choice %d", c.kernel);
    if (kernel == HEAT_KERNEL_STEP && precision == HEAT_FP32C)
        return fail(HEAT_EINVAL, "compensated FP32 needs the temporal-blocked kernel");
    q.kernel = kernel;
    if (c.register_form < 0 || c.register_form > 3)
        return fail(HEAT_EINVAL, "register_form must be 1, 2 or 3 (got %d)", c.register_form);
    q.form = c.register_form ? c.register_form : default_register_form(N, precision);
    if (kernel == HEAT_KERNEL_STEP) {
        q.K = 0;
        q.T = 1;
        q.H = 0;
        q.W = step_chunk_cells(precision);
        q.tiles = (N + q.W - 1) / q.W;
        q.rounds = nt;
        if (q.tiles * 64 > MAX_GRID_THREADS)
            return fail(HEAT_EINVAL, "ring of %lld cells is too long for one launch", (long long)N);
        *p = q;
        return HEAT_OK;
    }
    q.K = c.cells_per_lane ? c.cells_per_lane : default_cells_per_lane(N, precision);
    if (q.K != 8 && q.K != 16 && q.K != 32 && q.K != 64)
        return fail(HEAT_EINVAL, "cells_per_lane must be 8, 16, 32 or 64 (got %d)", q.K);
    if (q.K == 64 && q.form == 2 && precision != HEAT_FP32)
        return fail(HEAT_EINVAL, "the ping-pong form holds at most 32 cells per lane here");
    if (c.exchange < 0 || c.exchange > HEAT_EXCHANGE_LDS_DEEP)
        return fail(HEAT_EINVAL, "exchange must be 0, 1, 2 or 3 (got %d)", c.exchange);
    int xchg = c.exchange ? c.exchange : default_exchange(N, precision);
    // exchange depth K/4 (LDS) or K/2 (LDS_DEEP), at least 4 cells, between
    // at least 2 waves; a tuned exchange that the overridden shape cannot use
    // falls back to lone waves, an explicit request is checked
    const int xd = xchg == HEAT_EXCHANGE_LDS ? 4 : xchg == HEAT_EXCHANGE_LDS_DEEP ? 2 : 0;
    if (xd && (q.wpg < 2 || q.K / xd < 4)) {
        if (c.exchange == xchg)
            return fail(HEAT_EINVAL, "the LDS exchange needs waves_per_group >= 2 and an "
                        "exchange depth of at least 4 cells (cells_per_lane >= %d)", 4 * xd);
        xchg = HEAT_EXCHANGE_NONE;
    }
    q.xd = xchg == HEAT_EXCHANGE_NONE ? 0 : xd;
    if (kernel == HEAT_KERNEL_RESIDENT && precision != HEAT_FP64 && q.form != FORM_INPLACE_ID) {
        // the binary32 forms' resident kernels are built in place only
        if (c.register_form)
            return fail(HEAT_EINVAL, "the resident kernel runs the binary32 forms in place "
                        "(register_form 1; got %d)", q.form);
        q.form = FORM_INPLACE_ID;
    }
    if (kernel == HEAT_KERNEL_RESIDENT && !q.xd && q.wpg != 1) {
        // one tile per workgroup: lone waves run one wave per group
        if (c.waves_per_group)
            return fail(HEAT_EINVAL, "the resident kernel with lone waves needs "
                        "waves_per_group 1 (got %d)", q.wpg);
        q.wpg = 1;
    }
    int T = c.steps_per_round ? c.steps_per_round : default_steps_per_round(N, precision);
    if (T < 1) return fail(HEAT_EINVAL, "steps_per_round must be >= 1 (got %d)", T);
    if (c.steps_per_round && (T % 4) != 0)
        return fail(HEAT_EINVAL, "steps_per_round must be a multiple of 4 (got %d)", T);
    if (!c.steps_per_round && 3 * ceil4(T) > 64 * (int64_t)q.K) {
        // the tuned rounds are too deep for an overridden K: the deepest that
        // fits (the compensated form's 64 fits every K)
        T = (64 * q.K / 3) & ~3;
    }
    // the window must keep W >= H so a tile only reads its two neighbours
    if (3 * ceil4(T) > 64 * (int64_t)q.K)
        return fail(HEAT_EINVAL, "steps_per_round %d too deep for %d cells per lane", T, q.K);
    // RESIDENT: the steps between edge exchanges need no balancing (there is
    // no copy-back), but the compensated form's fold interval is its T
    const int64_t Teff =
        c.steps_per_round || kernel == HEAT_KERNEL_RESIDENT
            ? (nt > 0 ? std::min<int64_t>(T, nt) : 1)
            : balanced_steps_per_round(nt, T, precision);
    q.T = (int)Teff;
    q.H = halo_cells(Teff, precision, q.K);
    q.W = window_tile_cells(q.K, q.H, q.wpg, q.xd);
    q.tiles = (N + q.W - 1) / q.W;
    q.parts = q.xd ? q.tiles * q.wpg : q.tiles;
    q.rounds = nt > 0 ? (nt + Teff - 1) / Teff : 0;
    if (kernel == HEAT_KERNEL_RESIDENT) {
        // the halo reads wrap the ring at most once
        if (N < q.H)
            return fail(HEAT_EINVAL, "the resident kernel needs a ring of at least H = %d cells",
                        q.H);
        q.rounds = nt > 0 ? 1 : 0;
    }
    const int64_t threads = q.xd ? q.tiles * q.wpg * 64 : q.tiles * 64;
    if (threads > MAX_GRID_THREADS)
        return fail(HEAT_EINVAL, "ring of %lld cells needs more than one launch's tiles at %d cells "
                    "per lane", (long long)N, q.K);
    *p = q;
    return HEAT_OK;
}

// ================================================================ helpers

static std::once_flag g_pool_once[64];

int device_pool_setup() {
    int dev = 0;
    HEAT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return HEAT_OK;
    int rc = HEAT_OK;
    std::call_once(g_pool_once[dev], [&]() {
        hipMemPool_t pool;
        if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
            uint64_t thr = UINT64_MAX;
            (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
        }
    });
    return rc;
}

// Run the rounds of a plan: state in `a`, scratch `b`; result back in `a`.
// With `sums` (SUM area: partial buffers + 2 results), the binary64 sums of
// the state before and after land in sums->d_out[0] and [1]: fused into the
// first and last window rounds when the plan uses them, otherwise by the
// standalone reduction.
struct SumArea {
    double *partial = nullptr;   // max(SUM_BLOCKS, 2 * parts) doubles
    double *d_out = nullptr;     // 2 doubles
};

// Exchange area, epoch counters and status word of the resident kernel, per
// thread and device, with a pinned host word for the status: grown on demand
// and kept (a resident call waits for its stream before it returns, so the
// next call from the same thread finds them idle).  Tags and counters are
// never cleared between calls: each call counts on from `base`, the highest
// value the previous one left; they are cleared when a buffer is new, after
// a call that failed, and before `base` could wrap.
struct ResidentCache {
    uint32_t *d = nullptr;   // device: [1, 1 + tiles) epochs
    size_t cap = 0;          // words held by d
    uint64_t *x = nullptr;   // device: exchange area
    size_t xcap = 0;         // words held by x
    uint32_t *h = nullptr;   // pinned host: the status word, written by the kernel
    uint32_t base = 0;       // every counter is <= base
    int cus = 0;             // compute units of the device
    std::unordered_map<uint64_t, int> per_cu;   // workgroups per CU by shape
};
static thread_local ResidentCache g_resident_cache[64];

// Waits of a resident launch give up after this many polls (each a load
// and a short sleep, about a microsecond): seconds, far beyond any wait of a
// co-resident grid.
constexpr int64_t RESIDENT_SPIN_LIMIT = int64_t(1) << 22;

// HEAT_RESIDENT_SPIN_LIMIT (polls, >= 0) lowers it, read at every call: a
// test of the failure path sets 0, so a tile gives up at its first poll that
// finds a neighbour not yet there and the call fails with every wave exiting.
static int64_t resident_spin_limit() {
    const char *s = std::getenv("HEAT_RESIDENT_SPIN_LIMIT");
    if (!s || !*s) return RESIDENT_SPIN_LIMIT;
    char *end = nullptr;
    const long long v = std::strtoll(s, &end, 10);
    return (end && *end == '\0' && v >= 0 && v < RESIDENT_SPIN_LIMIT) ? (int64_t)v
                                                                     : RESIDENT_SPIN_LIMIT;
}

// Tiles of a resident plan's shape the current device holds at once (the
// LDS a group takes depends on its tile's W and H, so the occupancy is
// asked for each shape and LDS layout, once per thread), and whether the
// plan's grid needs the LDS copy of the edge regions only to fit.
static int resident_capacity(const Plan &pl, int precision, int64_t *capacity,
                             bool *edges_only = nullptr) {
    int dev = 0;
    HEAT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(HEAT_EDEVICE, "device %d out of range", dev);
    ResidentCache &c = g_resident_cache[dev];
    if (c.cus == 0) {
        hipDeviceProp_t prop;
        HEAT_HIP(hipGetDeviceProperties(&prop, dev));
        c.cus = prop.multiProcessorCount;
    }
    int64_t cap[2] = {0, 0};
    for (int edges = 0; edges < 2; ++edges) {
        const uint64_t key = (uint64_t)precision | (uint64_t)pl.K << 4 | (uint64_t)pl.form << 12 |
                             (uint64_t)pl.wpg << 16 | (uint64_t)pl.xd << 20 |
                             (uint64_t)(pl.W + 2 * pl.H) << 24 | (uint64_t)pl.H << 44 |
                             (uint64_t)edges << 60;
        auto it = c.per_cu.find(key);
        if (it == c.per_cu.end()) {
            ResidentArgs probe{};
            probe.W = pl.W;
            probe.H = pl.H;
            probe.lds_edges = edges;
            int n = 0;
            HEAT_HIP(launch_resident(precision, probe, pl.K, pl.form, pl.wpg, pl.xd, nullptr, &n));
            it = c.per_cu.emplace(key, n).first;
        }
        cap[edges] = it->second > 0 ? (int64_t)it->second * c.cus : 0;
    }
    // the whole tile copy where the grid fits with it (its indexing is the
    // cheaper), else the edge regions only
    const bool edges = pl.tiles > cap[0];
    *capacity = edges ? cap[1] : cap[0];
    if (edges_only) *edges_only = edges;
    return HEAT_OK;
}

// A resident launch whose status is still to be read: the caller waits for
// the stream once (for this and for whatever else it copies back) and then
// settles it.
struct ResidentPending {
    ResidentCache *c = nullptr;
    int64_t tiles = 0;
    int64_t epochs = 0;
};

// After the stream is idle: count the epochs on, and report a wait that
// timed out (then the counters and tags are in any state: they are cleared
// on the next call).
static int resident_settle(const ResidentPending &p) {
    ResidentCache &c = *p.c;
    c.base += (uint32_t)p.epochs;
    if (*c.h != 0) {
        // a fresh status word next time (the launch is done)
        (void)hipHostFree(c.h);
        c.h = nullptr;
        c.cap = 0;
        (void)hipFree(c.d);
        c.d = nullptr;
        c.xcap = 0;
        (void)hipFree(c.x);
        c.x = nullptr;
        return fail(HEAT_EDEVICE, "resident kernel: a tile waited too long for its neighbours "
                    "(were all %lld tiles resident? another launch may hold the CUs); the "
                    "state is undefined", (long long)p.tiles);
    }
    return HEAT_OK;
}

// With `defer` set the status copy is queued and the wait left to the caller
// (who must settle *defer after it); otherwise waits and settles here.
static int run_resident(const Plan &pl, int precision, void *a, void *b, int64_t N, double r,
                        int64_t nt, hipStream_t st, const SumArea *sums,
                        ResidentPending *defer = nullptr) {
    int dev = 0;
    HEAT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(HEAT_EDEVICE, "device %d out of range", dev);
    ResidentCache &c = g_resident_cache[dev];
    int64_t capacity = 0;
    bool edges_only = false;
    int rc = resident_capacity(pl, precision, &capacity, &edges_only);
    if (rc) return rc;
    ResidentArgs ra{};
    ra.W = pl.W;
    ra.H = pl.H;
    ra.lds_edges = edges_only ? 1 : 0;
    if (pl.tiles > capacity)
        return fail(HEAT_EINVAL, "the resident kernel needs all %lld tiles resident at once; this "
                    "shape fits %lld on the device (fewer cells per tile: a longer window, or "
                    "use HEAT_KERNEL_TB)", (long long)pl.tiles, (long long)capacity);
    const size_t words = (size_t)pl.tiles + 1;
    const size_t xwords =
        (size_t)resident_area_words(pl.tiles, pl.H, (int)storage_bytes(precision));
    const int64_t epochs = (nt + pl.T - 1) / pl.T;   // exchanges + 1
    if (!c.h) {
        HEAT_HIP(hipHostMalloc((void **)&c.h, sizeof(uint32_t), hipHostMallocDefault));
        *c.h = 0;
    }
    bool clear = false;
    // idle buffers: the last call waited for its stream
    if (c.cap < words) {
        if (c.d) HEAT_HIP(hipFree(c.d));
        c.d = nullptr;
        c.cap = 0;
        HEAT_HIP(hipMalloc((void **)&c.d, words * sizeof(uint32_t)));
        c.cap = words;
        clear = true;
    }
    if (c.xcap < xwords) {
        if (c.x) HEAT_HIP(hipFree(c.x));
        c.x = nullptr;
        c.xcap = 0;
        HEAT_HIP(hipMalloc((void **)&c.x, xwords * sizeof(uint64_t)));
        c.xcap = xwords;
        clear = true;
    }
    if (clear || (int64_t)c.base + epochs >= (int64_t(1) << 31)) {
        HEAT_HIP(launch_fill_u32(c.d, (int64_t)c.cap, 0u, st));
        HEAT_HIP(launch_fill_u32(reinterpret_cast<uint32_t *>(c.x), 2 * (int64_t)c.xcap, 0u, st));
        c.base = 0;
    }
    (void)b;   // the resident kernel keeps the state in registers and the ring
    ra.u = a;
    ra.N = N;
    ra.tiles = pl.tiles;
    ra.nt = nt;
    ra.T = pl.T;
    ra.r = r;
    ra.status = c.h;
    ra.flags = c.d + 1;
    ra.xa = c.x;
    ra.epoch_base = c.base;
    ra.spin_limit = resident_spin_limit();
    ra.part_in = sums ? sums->partial : nullptr;
    ra.part_out = sums ? sums->partial + pl.parts : nullptr;
    ra.vec_ok = (reinterpret_cast<uintptr_t>(a) & 15) == 0;
    HEAT_HIP(launch_resident(precision, ra, pl.K, pl.form, pl.wpg, pl.xd, st, nullptr));
    hipError_t e = sums ? launch_sum_partials(sums->partial, pl.parts, 2, sums->d_out, st)
                        : hipSuccess;
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(st);
        c.base += (uint32_t)epochs;   // counted on whatever happened, so no tag repeats
        return fail_hip(e, "resident kernel: checksum");
    }
    const ResidentPending p{&c, pl.tiles, epochs};
    if (defer) {
        *defer = p;
        return HEAT_OK;
    }
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        c.base += (uint32_t)epochs;   // counted on whatever happened, so no tag repeats
        return fail_hip(e, "resident kernel: wait");
    }
    return resident_settle(p);
}

static int run_rounds(const Plan &pl, int precision, void *a, void *b, int64_t N, double r,
                      int64_t nt, hipStream_t st, const SumArea *sums,
                      ResidentPending *defer = nullptr) {
    if (pl.kernel == HEAT_KERNEL_RESIDENT && nt > 0)
        return run_resident(pl, precision, a, b, N, r, nt, st, sums, defer);
    void *cur = a, *oth = b;
    const bool fused = sums && pl.kernel == HEAT_KERNEL_TB && nt > 0;
    if (sums && !fused) HEAT_HIP(launch_sum(precision, a, N, sums->partial, sums->d_out, st));
    if (pl.kernel == HEAT_KERNEL_STEP) {
        for (int64_t s = 0; s < nt; ++s) {
            HEAT_HIP(launch_step(precision, cur, oth, N, r, pl.wpg, st));
            std::swap(cur, oth);
        }
    } else {
        WindowLaunch w;
        w.precision = precision;
        w.K = pl.K;
        w.form = pl.form;
        w.N = N;
        w.H = pl.H;
        w.r = r;
        w.wpg = pl.wpg;
        w.xd = pl.xd;
        int64_t done = 0;
        while (done < nt) {
            w.steps = (int)std::min<int64_t>(pl.T, nt - done);
            w.src = cur;
            w.dst = oth;
            w.part_in = fused && done == 0 ? sums->partial : nullptr;
            w.part_out = fused && done + w.steps == nt ? sums->partial + pl.parts : nullptr;
            HEAT_HIP(launch_window(w, st));
            std::swap(cur, oth);
            done += w.steps;
        }
        if (fused) {
            // partial[0, parts): before the first round; [parts, 2 parts): after the last
            HEAT_HIP(launch_sum_partials(sums->partial, pl.parts, 2, sums->d_out, st));
        }
    }
    if (cur != a)
        HEAT_HIP(hipMemcpyAsync(a, cur, (size_t)N * storage_bytes(precision),
                                hipMemcpyDeviceToDevice, st));
    if (sums && !fused) HEAT_HIP(launch_sum(precision, a, N, sums->partial, sums->d_out + 1, st));
    return HEAT_OK;
}

struct DevBuf {   // stream-ordered scratch, freed on the same stream
    void *p = nullptr;
    hipStream_t st = nullptr;
    ~DevBuf() {
        if (p) (void)hipFreeAsync(p, st);
    }
};

// Checksum scratch per thread and device: device partials, and pinned host
// memory for the two sums, which the final reduction writes directly (no
// copy after it).  A call that asks for sums waits for its stream before it
// returns, so the next call from the same thread always finds the buffers
// idle.  Grown on demand and kept until the process ends (never freed: the
// runtime may be gone by thread exit), so a small ring's pass makes no
// allocation call.
struct SumCache {
    double *d = nullptr;   // device: partials
    size_t cap = 0;        // doubles held by d
    double *h = nullptr;   // pinned host: 2 doubles
};
static thread_local SumCache g_sum_cache[64];

static int sum_scratch(size_t doubles, SumCache **out) {
    int dev = 0;
    HEAT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(HEAT_EDEVICE, "device %d out of range", dev);
    SumCache &c = g_sum_cache[dev];
    if (!c.h) HEAT_HIP(hipHostMalloc((void **)&c.h, 2 * sizeof(double), hipHostMallocDefault));
    if (c.cap < doubles) {
        if (c.d) HEAT_HIP(hipFree(c.d));   // idle: the last call waited for its stream
        c.d = nullptr;
        c.cap = 0;
        HEAT_HIP(hipMalloc((void **)&c.d, doubles * sizeof(double)));
        c.cap = doubles;
    }
    *out = &c;
    return HEAT_OK;
}

// ============================================================ host staging
// heat_solve takes a pageable host array.  A plain copy of pageable memory
// runs through the runtime's own staging at a fraction of the PCIe rate, so
// large arrays go through pinned chunks instead: the array is cut into one
// contiguous slice per lane, and each lane (a host thread with its own
// stream and two pinned chunks) overlaps the host-side copy of one chunk
// with the DMA of the other.  The pinned chunks are allocated once per
// device (hipHostMalloc) and kept until the process ends; calls that stage
// at the same time take turns.  A copy may be a list of segments (the
// problems of a batch): the lanes then cut the segments' concatenation, and
// a chunk may hold pieces of several segments.
namespace {

constexpr size_t STAGE_CHUNK = size_t(8) << 20;        // bytes per pinned chunk
constexpr int STAGE_LANES = 8;                          // threads, each with 2 chunks
constexpr size_t STAGE_MIN_BYTES = size_t(64) << 20;    // smaller arrays: one plain copy

struct StageLane {
    char *buf[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipStream_t st = nullptr;
};

struct StagePool {
    std::mutex mu;
    bool ready = false;
    StageLane lane[STAGE_LANES];
};

StagePool g_stage[64];

// Allocate the device's pool on first use (caller holds pool.mu).  On
// failure the parts made so far are kept and the next call retries them.
hipError_t stage_pool_init(StagePool &pool) {
    if (pool.ready) return hipSuccess;
    for (StageLane &L : pool.lane) {
        for (int b = 0; b < 2; ++b) {
            if (!L.buf[b]) {
                hipError_t e = hipHostMalloc((void **)&L.buf[b], STAGE_CHUNK, hipHostMallocDefault);
                if (e != hipSuccess) return e;
            }
            if (!L.ev[b]) {
                hipError_t e = hipEventCreateWithFlags(&L.ev[b], hipEventDisableTiming);
                if (e != hipSuccess) return e;
            }
        }
        if (!L.st) {
            hipError_t e = hipStreamCreateWithFlags(&L.st, hipStreamNonBlocking);
            if (e != hipSuccess) return e;
        }
    }
    pool.ready = true;
    return hipSuccess;
}

// The pieces of segments that fall in the logical byte range [c0, c1): calls
// f(seg, offset in the segment, offset from c0, length) in order.
template <class F>
void for_pieces(const StageSeg *segs, const std::vector<size_t> &pre, size_t c0, size_t c1,
                F &&f) {
    size_t i = std::upper_bound(pre.begin(), pre.end(), c0) - pre.begin() - 1;
    for (; i + 1 < pre.size() && pre[i] < c1; ++i) {
        const size_t a = std::max(c0, pre[i]), b = std::min(c1, pre[i + 1]);
        if (b > a) f(segs[i], a - pre[i], a - c0, b - a);
    }
}

// One lane: the logical bytes [lo, hi) of the segments, host <-> device
// through its two chunks.
hipError_t stage_lane(StageLane &L, bool to_device, const StageSeg *segs,
                      const std::vector<size_t> &pre, size_t lo, size_t hi, int device) {
    hipError_t e = hipSetDevice(device);
    const size_t chunks = (hi - lo + STAGE_CHUNK - 1) / STAGE_CHUNK;
    auto c0 = [&](size_t k) { return lo + k * STAGE_CHUNK; };
    auto c1 = [&](size_t k) { return std::min(hi, lo + (k + 1) * STAGE_CHUNK); };
    if (to_device) {
        // host -> chunk k%2 (once the DMA of chunk k-2 has left it) -> device
        for (size_t k = 0; e == hipSuccess && k < chunks; ++k) {
            const int b = (int)(k & 1);
            if (k >= 2) e = hipEventSynchronize(L.ev[b]);
            if (e != hipSuccess) break;
            for_pieces(segs, pre, c0(k), c1(k), [&](const StageSeg &g, size_t so, size_t bo, size_t n) {
                std::memcpy(L.buf[b] + bo, (const char *)g.host + so, n);
            });
            for_pieces(segs, pre, c0(k), c1(k), [&](const StageSeg &g, size_t so, size_t bo, size_t n) {
                if (e == hipSuccess)
                    e = hipMemcpyAsync((char *)g.dev + so, L.buf[b] + bo, n, hipMemcpyHostToDevice,
                                       L.st);
            });
            if (e == hipSuccess) e = hipEventRecord(L.ev[b], L.st);
        }
    } else {
        // device -> chunk k%2, the DMA of chunk k+1 in flight while chunk k
        // is copied out to the host
        auto issue = [&](size_t k) {
            const int b = (int)(k & 1);
            hipError_t x = hipSuccess;
            for_pieces(segs, pre, c0(k), c1(k), [&](const StageSeg &g, size_t so, size_t bo, size_t n) {
                if (x == hipSuccess)
                    x = hipMemcpyAsync(L.buf[b] + bo, (const char *)g.dev + so, n,
                                       hipMemcpyDeviceToHost, L.st);
            });
            return x == hipSuccess ? hipEventRecord(L.ev[b], L.st) : x;
        };
        if (e == hipSuccess && chunks > 0) e = issue(0);
        for (size_t k = 0; e == hipSuccess && k < chunks; ++k) {
            if (k + 1 < chunks) e = issue(k + 1);
            if (e == hipSuccess) e = hipEventSynchronize(L.ev[k & 1]);
            if (e != hipSuccess) break;
            const int b = (int)(k & 1);
            for_pieces(segs, pre, c0(k), c1(k), [&](const StageSeg &g, size_t so, size_t bo, size_t n) {
                std::memcpy((char *)g.host + so, L.buf[b] + bo, n);
            });
        }
    }
    const hipError_t f = hipStreamSynchronize(L.st);
    return e != hipSuccess ? e : f;
}

}  // namespace

int stage_copies(bool to_device, const StageSeg *segs, size_t count, hipStream_t st) {
    // the device side may be stream-ordered memory or results of work on st
    HEAT_HIP(hipStreamSynchronize(st));
    std::vector<size_t> pre(count + 1, 0);
    for (size_t i = 0; i < count; ++i) pre[i + 1] = pre[i] + segs[i].bytes;
    const size_t total = pre[count];
    int device = 0;
    HEAT_HIP(hipGetDevice(&device));
    if (total < STAGE_MIN_BYTES || device < 0 || device >= 64) {
        for (size_t i = 0; i < count; ++i) {
            if (!segs[i].bytes) continue;
            if (to_device)
                HEAT_HIP(hipMemcpyAsync(segs[i].dev, segs[i].host, segs[i].bytes,
                                        hipMemcpyHostToDevice, st));
            else
                HEAT_HIP(hipMemcpyAsync(segs[i].host, segs[i].dev, segs[i].bytes,
                                        hipMemcpyDeviceToHost, st));
        }
        HEAT_HIP(hipStreamSynchronize(st));
        return HEAT_OK;
    }
    StagePool &pool = g_stage[device];
    std::lock_guard<std::mutex> lk(pool.mu);
    HEAT_HIP(stage_pool_init(pool));
    // lanes take slices of whole 4 KiB of the logical byte stream; the last
    // one takes the remainder
    const size_t slice = (total / STAGE_LANES + 4095) & ~size_t(4095);
    hipError_t err[STAGE_LANES];
    std::vector<std::thread> th;
    for (int t = 0; t < STAGE_LANES; ++t) {
        const size_t lo = std::min(total, (size_t)t * slice);
        const size_t hi = t + 1 == STAGE_LANES ? total : std::min(total, lo + slice);
        err[t] = hipSuccess;
        if (hi <= lo) continue;
        auto run = [&, t, lo, hi]() {
            err[t] = stage_lane(pool.lane[t], to_device, segs, pre, lo, hi, device);
        };
        if (t == 0) {
            continue;           // lane 0 runs on the calling thread below
        }
        try {
            th.emplace_back(run);
        } catch (...) {
            run();              // no thread to be had: this lane runs here
        }
    }
    err[0] = stage_lane(pool.lane[0], to_device, segs, pre, 0, std::min(total, slice), device);
    for (std::thread &x : th) x.join();
    for (hipError_t e : err)
        if (e != hipSuccess)
            return fail_hip(e, to_device ? "staged copy to device" : "staged copy to host");
    return HEAT_OK;
}

static bool config_is_auto(const heat_config *cfg) {
    return !cfg || !(cfg->kernel || cfg->cells_per_lane || cfg->steps_per_round ||
                     cfg->waves_per_group || cfg->register_form || cfg->exchange);
}

// Waves on the busiest SIMD of a resident plan, and its load efficiency.
static int64_t busiest_simd(const Plan &q, int cus) {
    const int64_t per_cu = (q.tiles + cus - 1) / cus;
    return (per_cu * q.wpg + 3) / 4;
}
static double load_efficiency(const Plan &q, int cus) {
    const int64_t busiest = busiest_simd(q, cus);
    return busiest > 0 ? (double)q.tiles * q.wpg / (4.0 * cus) / (double)busiest : 0.0;
}

static int device_cus(int *cus) {
    int dev = 0;
    HEAT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(HEAT_EDEVICE, "device %d out of range", dev);
    ResidentCache &c = g_resident_cache[dev];
    if (c.cus == 0) {
        hipDeviceProp_t prop;
        HEAT_HIP(hipGetDeviceProperties(&prop, dev));
        c.cus = prop.multiProcessorCount;
    }
    *cus = c.cus;
    return HEAT_OK;
}

// The fitting of resident_fit on a plan; false if no interval fits.
static bool fit_resident_plan(int64_t N, int64_t nt, int precision, const heat_config &c, int cus,
                              Plan *out, int *T_out = nullptr) {
    const int T0 = c.steps_per_round;
    int64_t best_load = 0;
    bool have = false;
    for (int T : {T0, 96, 64, 48, 32, 24, 16}) {
        if (T > T0 || 2 * T < T0 || (T != T0 && precision == HEAT_FP32C)) continue;
        if (have && T == T0) continue;
        heat_config f = c;
        f.steps_per_round = T;
        Plan q;
        if (make_plan(N, nt, precision, &f, &q) != HEAT_OK || q.kernel != HEAT_KERNEL_RESIDENT)
            continue;
        int64_t capacity = 0;
        if (resident_capacity(q, precision, &capacity) != HEAT_OK || q.tiles > capacity)
            continue;
        const int64_t load = busiest_simd(q, cus);
        if (!have || load < best_load) {
            *out = q;
            if (T_out) *T_out = T;
            best_load = load;
            have = true;
        }
    }
    return have;
}

int resident_fit(int64_t N, int64_t nt, int precision, const heat_config &c,
                 heat_config *fitted, double *eff) {
    int cus = 0;
    int rc = device_cus(&cus);
    if (rc) return rc;
    Plan q;
    int T = 0;
    if (!fit_resident_plan(N, nt, precision, c, cus, &q, &T))
        return fail(HEAT_EINVAL, "the resident shape cannot run %lld cells", (long long)N);
    *fitted = c;
    fitted->steps_per_round = T;
    *eff = load_efficiency(q, cus);
    return HEAT_OK;
}

// The last resident choice of each thread, kept until the tuning table
// changes (a loop of calls on one ring chooses once).
struct ResidentChoiceCache {
    bool valid = false, resident = false;
    int dev = -1, precision = -1;
    int64_t N = 0, nt = 0;
    uint64_t generation = 0;
    Plan plan;
};
static thread_local ResidentChoiceCache g_choice;

static void choose_resident(int64_t N, int64_t nt, int precision, Plan *pl);

// The plan a call runs: make_plan's, except that a call that waits for its
// result (`waits`) with an all-automatic configuration may take the resident
// kernel: every shape the tuning table records for N's quarter decade whose
// shortest winning run at N is no longer than nt is fitted to N
// (resident_fit), and the one whose gain at full SIMD load at N times its
// load efficiency at N is the largest is taken, if that is at least the
// margin (the shortest run and the gain interpolated between the points the
// tuner measured).  At the measured points this is the measured gain; in
// between, the model follows the tiles as they fall on the SIMDs.  The
// choice is cached per thread (g_choice).
static int choose_plan(int64_t N, int64_t nt, int precision, const heat_config *cfg, bool waits,
                       Plan *pl) {
    int rc = make_plan(N, nt, precision, cfg, pl);
    if (rc || !waits || nt < 1 || !config_is_auto(cfg)) return rc;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HEAT_OK;
    const uint64_t gen = tune_generation();
    ResidentChoiceCache &m = g_choice;
    if (!(m.valid && m.dev == dev && m.N == N && m.nt == nt && m.precision == precision &&
          m.generation == gen)) {
        Plan q = *pl;
        choose_resident(N, nt, precision, &q);
        m.valid = true;
        m.dev = dev;
        m.N = N;
        m.nt = nt;
        m.precision = precision;
        m.generation = gen;
        m.resident = q.kernel == HEAT_KERNEL_RESIDENT;
        m.plan = q;
    }
    if (m.resident) *pl = m.plan;
    return HEAT_OK;
}

// choose_plan's resident step: *pl is replaced where a recorded shape wins.
static void choose_resident(int64_t N, int64_t nt, int precision, Plan *pl) {
    ResidentChoice ch[RESIDENT_SHAPES];
    const int n = tuned_resident(N, precision, ch);
    int cus = 0;
    if (n == 0 || device_cus(&cus) != HEAT_OK || cus < 1) return;
    int64_t pts[RESIDENT_POINTS];
    resident_points(N, pts);
    double best_score = 0.0;
    Plan best;
    for (int i = 0; i < n; ++i) {
        const double min_nt = resident_interp(ch[i].min_nt, pts, N);
        if (min_nt <= 0.0 || (double)nt < min_nt) continue;
        Plan q;
        if (!fit_resident_plan(N, nt, precision, ch[i].c, cus, &q)) continue;
        // a shape recorded without its gains stands for the margin
        const bool recorded = ch[i].gain[0] > 0.0 || ch[i].gain[1] > 0.0 || ch[i].gain[2] > 0.0;
        const double score = recorded
                                 ? resident_interp(ch[i].gain, pts, N) * load_efficiency(q, cus)
                                 : RESIDENT_TUNE_MARGIN;
        if (score > best_score) {
            best_score = score;
            best = q;
        }
    }
    if (best_score >= RESIDENT_TUNE_MARGIN) *pl = best;
}

static int solve_dev_impl(void *d_u, void *d_work, int64_t N, int32_t nparts, double r, int64_t nt,
                          int32_t precision, const heat_config *cfg, hipStream_t st,
                          double *sum0_out, double *sum_out, bool waits = false) {
    int rc = check_problem(N, nparts, r, nt, precision);
    if (rc) return rc;
    if (!d_u) return fail(HEAT_EINVAL, "d_u is NULL");
    const size_t bytes = (size_t)N * storage_bytes(precision);
    if (d_work) {
        const char *a = (const char *)d_u, *w = (const char *)d_work;
        if (w < a + bytes && a < w + bytes) return fail(HEAT_EINVAL, "d_work overlaps d_u");
    }
    const bool want_sums = sum0_out || sum_out;
    Plan pl;
    rc = choose_plan(N, nt, precision, cfg, waits || want_sums, &pl);
    if (rc) return rc;
    rc = device_pool_setup();
    if (rc) return rc;
    DevBuf work;
    work.st = st;
    SumArea area;
    SumCache *cache = nullptr;
    if (want_sums) {
        const int64_t np = std::max<int64_t>(SUM_BLOCKS, 2 * pl.parts);
        rc = sum_scratch((size_t)np, &cache);
        if (rc) return rc;
        area.partial = cache->d;
        area.d_out = cache->h;   // the final reduction writes the pinned host words
    }
    void *b = d_work;
    // the resident kernel keeps the state in registers and needs no second buffer
    if (nt > 0 && !b && pl.kernel != HEAT_KERNEL_RESIDENT) {
        HEAT_HIP(hipMallocAsync(&work.p, bytes, st));
        b = work.p;
    }
    // one wait for the sums and the resident kernel's status together
    ResidentPending pend;
    rc = run_rounds(pl, precision, d_u, b, N, r, nt, st, want_sums ? &area : nullptr, &pend);
    if (rc) {
        // the cached scratch must be idle when this thread calls again
        if (want_sums || pend.c) (void)hipStreamSynchronize(st);
        if (pend.c) pend.c->base += (uint32_t)pend.epochs;
        return rc;
    }
    hipError_t e = hipSuccess;
    if (want_sums || pend.c) e = hipStreamSynchronize(st);
    if (pend.c) {
        // the epochs are counted on whatever happened, so no tag repeats
        if (e != hipSuccess) pend.c->base += (uint32_t)pend.epochs;
        else rc = resident_settle(pend);
    }
    if (e != hipSuccess) return fail_hip(e, "solve: wait");
    if (rc) return rc;
    if (want_sums) {
        if (sum0_out) *sum0_out = cache->h[0];
        if (sum_out) *sum_out = cache->h[1];
    }
    return HEAT_OK;
}

// ============================================================ no-alloc form
// Device scratch of heat_solve_dev_noalloc: the ping-pong state buffer and
// the checksum partials of one call, in one fixed array that the code object
// holds on every device the library runs on (until the process ends).  Host
// code never uses the array's name as an address: on each device the
// address is looked up once (hipGetSymbolAddress, with that device
// current) and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[HEAT_NOALLOC_SCRATCH_BYTES];

static std::once_flag g_scratch_once[64];
static void *g_scratch_ptr[64];
static hipError_t g_scratch_err[64];

static int noalloc_scratch(void **out) {
    int dev = 0;
    HEAT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(HEAT_EDEVICE, "device %d out of range", dev);
    std::call_once(g_scratch_once[dev], [&]() {
        g_scratch_err[dev] = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
    });
    if (g_scratch_err[dev] != hipSuccess)
        return fail_hip(g_scratch_err[dev], "hipGetSymbolAddress(scratch)");
    *out = g_scratch_ptr[dev];
    return HEAT_OK;
}

// Bytes of scratch a call needs: the state buffer (whole 256-byte units),
// then the checksum partials (max(SUM_BLOCKS, 2 * parts) doubles).
static size_t noalloc_bytes(const Plan &pl, int64_t N, int precision, int64_t nt, bool sums,
                            size_t *partial_off) {
    const size_t work = nt > 0 ? ((size_t)N * storage_bytes(precision) + 255) & ~size_t(255) : 0;
    *partial_off = work;
    const size_t np = sums ? (size_t)std::max<int64_t>(SUM_BLOCKS, 2 * pl.parts) : 0;
    return work + np * sizeof(double);
}

static int solve_dev_noalloc_impl(void *d_u, int64_t N, int32_t nparts, double r, int64_t nt,
                                  int32_t precision, hipStream_t st, double *d_sums_out) {
    int rc = check_problem(N, nparts, r, nt, precision);
    if (rc) return rc;
    if (!d_u) return fail(HEAT_EINVAL, "d_u is NULL");
    Plan pl;
    rc = make_plan(N, nt, precision, nullptr, &pl);
    if (rc) return rc;
    if (pl.kernel == HEAT_KERNEL_RESIDENT) {
        // it waits for the stream and keeps its own counters: take the round
        // kernel with the same shape (the same results)
        heat_config c{HEAT_KERNEL_TB, pl.K, 0, 0, pl.form, 0};
        rc = make_plan(N, nt, precision, &c, &pl);
        if (rc) return rc;
    }
    size_t partial_off = 0;
    const size_t need = noalloc_bytes(pl, N, precision, nt, d_sums_out != nullptr, &partial_off);
    if (need > (size_t)HEAT_NOALLOC_SCRATCH_BYTES)
        return fail(HEAT_EINVAL, "ring of %lld cells needs %zu bytes of scratch; the static "
                    "scratch holds %zu", (long long)N, need, (size_t)HEAT_NOALLOC_SCRATCH_BYTES);
    void *base = nullptr;
    rc = noalloc_scratch(&base);
    if (rc) return rc;
    SumArea area;
    if (d_sums_out) {
        area.partial = (double *)((char *)base + partial_off);
        area.d_out = d_sums_out;
    }
    return run_rounds(pl, precision, d_u, nt > 0 ? base : nullptr, N, r, nt, st,
                      d_sums_out ? &area : nullptr);
}

}  // namespace heat

using namespace heat;

// ================================================================== C ABI

extern "C" {

const char *heat_last_error(void) { return heat::g_err; }

// The build compiles in the sha256 of the sources it compiled (build.py,
// source_digest), so a caller can tell a library built from other sources.
#ifndef HEAT_SOURCE_SHA256
#define HEAT_SOURCE_SHA256 "unknown"
#endif
const char *heat_version(void) { return "heat-mi355x 0.2 (gfx950) src " HEAT_SOURCE_SHA256; }

int heat_device_info(int32_t *cus, int32_t *lds_bytes, int32_t *wave_size, int32_t *clock_khz,
                     size_t *mem_total, size_t *mem_free) {
    int dev = 0;
    HEAT_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HEAT_HIP(hipGetDeviceProperties(&prop, dev));
    if (cus) *cus = prop.multiProcessorCount;
    if (lds_bytes) *lds_bytes = (int32_t)prop.sharedMemPerBlock;
    if (wave_size) *wave_size = prop.warpSize;
    if (clock_khz) *clock_khz = prop.clockRate;
    if (mem_total || mem_free) {
        size_t f = 0, t = 0;
        HEAT_HIP(hipMemGetInfo(&f, &t));
        if (mem_total) *mem_total = t;
        if (mem_free) *mem_free = f;
    }
    return HEAT_OK;
}

int heat_plan(int64_t N, int64_t nt, int32_t precision, const heat_config *cfg,
              heat_plan_info *out) {
    int rc = check_problem(N, 1, 0.25, nt, precision);
    if (rc) return rc;
    if (!out) return fail(HEAT_EINVAL, "out is NULL");
    Plan pl;
    rc = choose_plan(N, nt, precision, cfg, true, &pl);
    if (rc) return rc;
    out->kernel = pl.kernel;
    out->cells_per_lane = pl.K;
    out->steps_per_round = pl.T;
    out->waves_per_group = pl.wpg;
    out->register_form = pl.form;
    out->exchange_steps = pl.kernel != HEAT_KERNEL_STEP && pl.xd ? pl.K / pl.xd : 0;
    out->tile_cells = pl.W;
    out->tiles = pl.tiles;
    out->rounds = pl.rounds;
    return HEAT_OK;
}

int heat_solve_dev_cfg(void *d_u, void *d_work, int64_t N, int32_t nparts, double r, int64_t nt,
                       int32_t precision, const heat_config *cfg, void *hip_stream,
                       double *sum0_out, double *sum_out) {
    return solve_dev_impl(d_u, d_work, N, nparts, r, nt, precision, cfg, (hipStream_t)hip_stream,
                          sum0_out, sum_out);
}

int heat_solve_dev(void *d_u, int64_t N, int32_t nparts, double r, int64_t nt, int32_t precision,
                   void *hip_stream, double *sum0_out, double *sum_out) {
    return solve_dev_impl(d_u, nullptr, N, nparts, r, nt, precision, nullptr,
                          (hipStream_t)hip_stream, sum0_out, sum_out);
}

int heat_solve_dev_noalloc(void *d_u, int64_t N, int32_t nparts, double r, int64_t nt,
                           int32_t precision, void *hip_stream, double *d_sums_out) {
    return solve_dev_noalloc_impl(d_u, N, nparts, r, nt, precision, (hipStream_t)hip_stream,
                                  d_sums_out);
}

int heat_solve(double *u, int64_t N, int32_t nparts, double r, int64_t nt) {
    if (!u) return fail(HEAT_EINVAL, "u is NULL");
    int rc = check_problem(N, nparts, r, nt, HEAT_FP64);
    if (rc) return rc;
    hipStream_t st = nullptr;
    HEAT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    void *d = nullptr;
    const size_t bytes = (size_t)N * sizeof(double);
    hipError_t e = hipMalloc(&d, bytes);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(st);
        return fail_hip(e, "hipMalloc(state)");
    }
    const StageSeg seg{d, u, bytes};
    rc = stage_copies(true, &seg, 1, st);
    if (!rc) rc = solve_dev_impl(d, nullptr, N, nparts, r, nt, HEAT_FP64, nullptr, st, nullptr,
                                 nullptr, true);
    if (!rc) rc = stage_copies(false, &seg, 1, st);
    e = hipStreamSynchronize(st);
    if (!rc && e != hipSuccess) rc = fail_hip(e, "hipStreamSynchronize");
    (void)hipFree(d);
    (void)hipStreamDestroy(st);
    return rc;
}

int heat_copy_dev(const void *d_src, void *d_dst, size_t bytes, void *hip_stream) {
    if (!d_src || !d_dst) return fail(HEAT_EINVAL, "NULL pointer");
    if ((bytes & 15) || ((uintptr_t)d_src & 15) || ((uintptr_t)d_dst & 15))
        return fail(HEAT_EINVAL, "copy needs 16-byte sizes and alignment");
    if (bytes == 0) return HEAT_OK;
    HEAT_HIP(launch_copy(d_src, d_dst, bytes, (hipStream_t)hip_stream));
    return HEAT_OK;
}

int heat_checksum_dev(const void *d_u, int64_t N, int32_t precision, void *hip_stream,
                      double *sum_out) {
    if (!d_u || !sum_out) return fail(HEAT_EINVAL, "NULL pointer");
    if (N < 1) return fail(HEAT_EINVAL, "N must be >= 1");
    if (precision != HEAT_FP64 && precision != HEAT_FP32 && precision != HEAT_FP32C)
        return fail(HEAT_EINVAL, "unknown precision %d", precision);
    int rc = device_pool_setup();
    if (rc) return rc;
    hipStream_t st = (hipStream_t)hip_stream;
    DevBuf sums;
    sums.st = st;
    HEAT_HIP(hipMallocAsync(&sums.p, (SUM_BLOCKS + 1) * sizeof(double), st));
    double *partial = (double *)sums.p;
    HEAT_HIP(launch_sum(precision, d_u, N, partial, partial + SUM_BLOCKS, st));
    HEAT_HIP(hipMemcpyAsync(sum_out, partial + SUM_BLOCKS, sizeof(double), hipMemcpyDeviceToHost,
                            st));
    HEAT_HIP(hipStreamSynchronize(st));
    return HEAT_OK;
}

}  // extern "C"
