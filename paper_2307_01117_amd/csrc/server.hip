// server.hip -- serving form: a continuous-batching request loop.
//
// Requests (heat problems of different N, nt, r and precision) arrive through
// heat_submit from any thread.  A scheduler thread admits them in arrival
// order while the device arena has room for their footprint and a slot is
// free, and advances every resident request together: each tick is a short
// sequence of round launches (the batching form's k_batch_round) over all
// active requests, so requests that arrive while others run join at the next
// tick and their work shares the device.  Copy threads move request data
// host->device at admission (one thread, its own stream) and device->host at
// completion (STAGE_OUT_LANES threads), off the scheduler's path and past
// each other (measured on MI355X with the serving mix: one thread for both
// directions saturated at 3,700 GCUP/s, two at 5,050).  The device->host
// copies are issued to the DMA engines through ROCr (a HIP copy to host
// memory runs as a blit kernel on the compute units, beside the rounds):
// each stage-out lane owns two pinned chunks and copies a result chunk by
// chunk, the DMA of one chunk overlapping the host-side copy of the other.
// A request's rounds are exactly those it would run alone (same T rule,
// same buffers, same order), so its result is bit-identical alone and in
// any mix.
#include <hip/hip_runtime.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include <algorithm>
#include <cmath>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "arena.h"
#include "heat_batch.h"
#include "heat_internal.h"

namespace heat {

using Clock = std::chrono::steady_clock;

// ------------------------------------------------------------------ arena
// One device allocation; offsets are handed out by ArenaBook (arena.h).
class Arena {
  public:
    int init(size_t bytes) {
        HEAT_HIP(hipMalloc(&base_, bytes));
        book_.reset(bytes);
        return HEAT_OK;
    }
    void destroy() {
        if (base_) (void)hipFree(base_);
        base_ = nullptr;
    }
    bool alloc(size_t bytes, size_t *off) { return book_.alloc(bytes, off); }
    void release(size_t off, size_t bytes) { book_.release(off, bytes); }
    static size_t round(size_t b) { return ArenaBook::round(b); }
    char *base() const { return (char *)base_; }
    size_t cap() const { return book_.cap(); }
    size_t used() const { return book_.used(); }
    size_t peak() const { return book_.peak(); }

  private:
    void *base_ = nullptr;
    ArenaBook book_;
};

enum ReqState { QUEUED, STAGING, READY, ACTIVE, DRAINING, DONE, FAILED, CANCELLED };
static bool finished_state(int st) { return st == DONE || st == FAILED || st == CANCELLED; }

struct Req {
    uint64_t ticket = 0;
    heat_problem *p = nullptr;
    heat_ring ring{};
    BatchRing br{};
    size_t off = 0, bytes = 0;
    double *d_sums = nullptr;          // [sum0, sum_nt] on the device
    double shift = 0.0;                // FP32 forms: state held as offsets from it
    int state = QUEUED;
    int rc = HEAT_OK;
    std::string msg;                   // error text, kept for the thread that polls
    bool holds = false;                // owns an arena block and a slot
    bool cancel = false;
    hipEvent_t fin = nullptr;          // compute stream passed its final kernels
    Clock::time_point t_submit;
};

// Footprint: state (N x storage) + scratch wide enough to stage binary64
// input (N x max(storage, 8)) + the two sums.
static size_t footprint(int64_t N, int precision) {
    const size_t es = storage_bytes(precision);
    return Arena::round((size_t)N * es) + Arena::round((size_t)N * std::max<size_t>(es, 8)) + 256;
}

// Rounds per tick: every active request advances this many rounds (or what
// it has left).  Short ticks bound the admission delay, and every round of a
// tick is a launch per kernel class, so later rounds that hold only a few
// rings leave the GPU partly idle: on MI355X with the serving mix, ticks of
// 320+ steps fell behind 1,000 requests/s that 2-round ticks sustain.
// HEAT_SERVER_TICK_STEPS (optional) instead sizes ticks in steps.
constexpr int32_t TICK_ROUNDS = 2;

// Cells per lane of a ring served at light load.  A tick's rounds are
// launches that a mix of requests fills only partly, so a round lasts about
// as long as its slowest tile, and a 64-cell tile takes twice as long as a
// 32-cell one; the batching form, which fills the GPU, uses wider classes
// (and so does the server under load, see SERVER_BUSY_SLOTS).  Measured on MI355X with the serving mix at 1,000
// requests/s: p50 / p99 13.4 / 63.7 ms with 32-cell lanes against 25.6 /
// 75.9 ms with the batching form's classes, at the same throughput.
constexpr int SERVER_CELLS_PER_LANE = 32;
constexpr int TABLE_GROUPS = 9;        // (precision, kernel class) round tables per tick
// Requests admitted while more than this many are resident take the batching
// form's classes (64-cell lanes, 4-wave tiles for the longest rings): under
// load throughput decides latency, and those classes carry more cell updates
// per launch; at light load every request keeps 32-cell lanes.  A request
// keeps its class for life, and no class changes a result.
constexpr int32_t SERVER_BUSY_SLOTS = 64;

// ------------------------------------------------------- DMA stage-out
// Device -> host copies on the DMA engines: hsa_amd_memory_async_copy with
// the host's CPU agent as destination runs on an SDMA engine (ROCr keeps
// blit kernels for copies within one agent).  Its destination must be memory
// the GPU can reach, so results go through pinned chunks; the source must be
// released to system scope first, which the completion event of a request's
// last kernels does (hipEventReleaseToSystem).
constexpr int STAGE_OUT_LANES = 2;
constexpr size_t STAGE_OUT_CHUNK = size_t(8) << 20;
constexpr int64_t DMA_WAIT_NS = int64_t(60) * 1000 * 1000 * 1000;   // a copy stuck this long fails

struct DmaAgents {
    hsa_agent_t gpu{}, cpu{};
    bool gpu_found = false, cpu_found = false;
    uint32_t bdf = 0, domain = 0;
};

static hsa_status_t find_agents(hsa_agent_t a, void *data) {
    DmaAgents *d = (DmaAgents *)data;
    hsa_device_type_t t;
    if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &t) != HSA_STATUS_SUCCESS)
        return HSA_STATUS_SUCCESS;
    if (t == HSA_DEVICE_TYPE_CPU && !d->cpu_found) {
        d->cpu = a;
        d->cpu_found = true;
    } else if (t == HSA_DEVICE_TYPE_GPU && !d->gpu_found) {
        uint32_t bdf = 0, dom = 0;
        if (hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_BDFID, &bdf) ==
                HSA_STATUS_SUCCESS &&
            hsa_agent_get_info(a, (hsa_agent_info_t)HSA_AMD_AGENT_INFO_DOMAIN, &dom) ==
                HSA_STATUS_SUCCESS &&
            bdf == d->bdf && dom == d->domain) {
            d->gpu = a;
            d->gpu_found = true;
        }
    }
    return HSA_STATUS_SUCCESS;
}

// One stage-out lane: two pinned chunks, a pinned landing spot for a
// request's two sums, and a completion signal for each.
struct OutLane {
    char *buf[2] = {nullptr, nullptr};
    double *sums = nullptr;
    hsa_signal_t sig[2] = {{0}, {0}};
    hsa_signal_t sig_sums = {0};
    std::thread th;
};

static int hsa_fail(hsa_status_t st, const char *what) {
    const char *msg = nullptr;
    if (hsa_status_string(st, &msg) != HSA_STATUS_SUCCESS || !msg) msg = "unknown";
    return fail(HEAT_EDEVICE, "%s: %s", what, msg);
}

// Start a DMA copy of n bytes from device memory to pinned host memory.
static int dma_start(const DmaAgents &ag, void *dst, const void *src, size_t n,
                     hsa_signal_t sig) {
    hsa_signal_store_relaxed(sig, 1);
    const hsa_status_t st = hsa_amd_memory_async_copy(dst, ag.cpu, src, ag.gpu, n, 0, nullptr, sig);
    return st == HSA_STATUS_SUCCESS ? HEAT_OK : hsa_fail(st, "hsa_amd_memory_async_copy");
}

// Wait for a copy started by dma_start (bounded: a copy that does not end
// within DMA_WAIT_NS fails instead of hanging the lane).
static int dma_wait(hsa_signal_t sig) {
    const auto t0 = std::chrono::steady_clock::now();
    while (true) {
        const hsa_signal_value_t v = hsa_signal_wait_scacquire(
            sig, HSA_SIGNAL_CONDITION_LT, 1, 100 * 1000 * 1000, HSA_WAIT_STATE_BLOCKED);
        if (v < 0) return fail(HEAT_EDEVICE, "DMA copy to host failed");
        if (v == 0) return HEAT_OK;
        if (std::chrono::duration_cast<std::chrono::nanoseconds>(
                std::chrono::steady_clock::now() - t0).count() > DMA_WAIT_NS)
            return fail(HEAT_EDEVICE, "DMA copy to host did not finish");
    }
}

// Host memory the GPU can reach (pinned by hipHostMalloc or registered):
// the DMA may write it directly.
static bool gpu_reachable_host(const void *p) {
    hipPointerAttribute_t a;
    const hipError_t e = hipPointerGetAttributes(&a, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();   // pageable memory: not an error here
        return false;
    }
    return a.type == hipMemoryTypeHost;
}

// Copy n bytes of device memory into a host array: straight into it when
// the GPU can reach it, otherwise through the lane's two pinned chunks, the
// DMA of chunk k+1 running while chunk k is copied out.
static int dma_to_host(const DmaAgents &ag, OutLane &L, void *host, const void *dev, size_t n) {
    if (n > 0 && gpu_reachable_host(host)) {
        int rc = dma_start(ag, host, dev, n, L.sig[0]);
        if (rc == HEAT_OK) rc = dma_wait(L.sig[0]);
        return rc;
    }
    const size_t chunks = (n + STAGE_OUT_CHUNK - 1) / STAGE_OUT_CHUNK;
    auto len = [&](size_t k) { return std::min(STAGE_OUT_CHUNK, n - k * STAGE_OUT_CHUNK); };
    int rc = chunks > 0 ? dma_start(ag, L.buf[0], dev, len(0), L.sig[0]) : HEAT_OK;
    bool next_in_flight = false;
    for (size_t k = 0; rc == HEAT_OK && k < chunks; ++k) {
        const int b = (int)(k & 1);
        next_in_flight = false;
        if (k + 1 < chunks) {
            rc = dma_start(ag, L.buf[b ^ 1], (const char *)dev + (k + 1) * STAGE_OUT_CHUNK,
                           len(k + 1), L.sig[b ^ 1]);
            next_in_flight = rc == HEAT_OK;
        }
        const int rw = dma_wait(L.sig[b]);
        if (rc == HEAT_OK) rc = rw;
        if (rc == HEAT_OK) std::memcpy((char *)host + k * STAGE_OUT_CHUNK, L.buf[b], len(k));
    }
    // a failed wait may leave the next chunk's copy in flight: let it end
    // before the lane's chunks are reused
    if (rc != HEAT_OK && next_in_flight) {
        for (int b = 0; b < 2; ++b) (void)dma_wait(L.sig[b]);
    }
    return rc;
}

}  // namespace heat

using namespace heat;

struct heat_server {
    std::mutex mu;
    std::condition_variable cv_sched, cv_in, cv_out, cv_done;
    std::deque<Req *> queue, h2d, d2h;
    std::vector<Req *> ready, active;
    std::unordered_map<uint64_t, Req *> reqs;
    Arena arena;
    int device = 0;
    int32_t max_slots = 4096, max_queue = 65536, slots_used = 0;
    int32_t tick_steps = 0;   // 0: TICK_ROUNDS rounds per tick
    hipStream_t compute = nullptr, copy_in = nullptr;
    double *d_partial = nullptr;
    // round tables, double-buffered across ticks (TABLE_GROUPS groups each)
    size_t table_slot_bytes = 0;
    char *d_tables = nullptr, *h_tables = nullptr;
    hipEvent_t table_ev[2] = {nullptr, nullptr};
    uint64_t tick = 0, next_ticket = 1;
    bool stop = false;
    int fatal = HEAT_OK;
    std::thread sched, stager_in;
    DmaAgents dma;
    bool hsa_up = false;
    OutLane out[STAGE_OUT_LANES];
    heat_server_stats st{};
};

static void finish_locked(heat_server *s, Req *q, int state, int rc) {
    if (q->holds) {
        s->arena.release(q->off, q->bytes);
        q->holds = false;
        --s->slots_used;
    }
    q->state = state;
    q->rc = rc;
    if (rc < 0 && rc != HEAT_ECANCELED) q->msg = heat_last_error();
    if (q->fin) {
        (void)hipEventDestroy(q->fin);
        q->fin = nullptr;
    }
    if (state == CANCELLED) ++s->st.cancelled;
    s->cv_done.notify_all();
    s->cv_sched.notify_one();
}

// After a device error: fail every request the scheduler still holds --
// resident, staged, waiting for its stage-in, or queued -- and release their
// blocks.  The caller has waited for the compute stream, so no kernel still
// writes the arena; a stage-in in progress fails its request itself when it
// ends (stage_in_loop checks `fatal`).
static void fail_all_locked(heat_server *s, int rc) {
    auto fail_list = [&](auto &list) {
        for (Req *q : list) {
            q->p->status = rc;
            finish_locked(s, q, FAILED, rc);
        }
        list.clear();
    };
    fail_list(s->active);
    fail_list(s->ready);
    fail_list(s->h2d);
    fail_list(s->queue);
    s->st.active = 0;
    s->st.queued = 0;
}

// ------------------------------------------------------------ copy threads
// Stage-in and stage-out run on threads and streams of their own: the two
// directions overlap on the DMA engines, and a stage-out that waits for its
// request's last round never holds up the next request's stage-in.  Each
// loop drains its queue before it honours `stop`.
static void stage_out_loop(heat_server *s, int lane) {
    (void)hipSetDevice(s->device);
    OutLane &L = s->out[lane];
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv_out.wait(lk, [&] { return s->stop || !s->d2h.empty(); });
        if (s->d2h.empty()) break;
        Req *q = s->d2h.front();
        s->d2h.pop_front();
        lk.unlock();
        const int64_t N = q->ring.N;
        int rc = HEAT_OK;
        hipError_t e = hipEventSynchronize(q->fin);
        if (e != hipSuccess) rc = fail_hip(e, "server stage-out (wait for the last round)");
        // FP32 forms were widened exactly into the scratch buffer
        const void *src = q->ring.precision == HEAT_FP64 ? q->ring.d_u : q->ring.d_work;
        bool sums_in_flight = false;
        if (rc == HEAT_OK) {
            rc = dma_start(s->dma, L.sums, q->d_sums, 2 * sizeof(double), L.sig_sums);
            sums_in_flight = rc == HEAT_OK;
        }
        if (rc == HEAT_OK) rc = dma_to_host(s->dma, L, q->p->u_out, src, (size_t)N * 8);
        if (sums_in_flight) {
            const int rw = dma_wait(L.sig_sums);
            if (rc == HEAT_OK) rc = rw;
        }
        const std::string msg = rc ? heat_last_error() : "";
        lk.lock();
        if (rc == HEAT_OK) {
            // sums of the stored offsets, plus N*shift for the shifted forms
            const double base = q->ring.precision == HEAT_FP64 ? 0.0 : (double)N * q->shift;
            q->p->sum0 = base + L.sums[0];
            q->p->sum_nt = base + L.sums[1];
            q->p->status = HEAT_OK;
            q->p->latency_s =
                std::chrono::duration<double>(Clock::now() - q->t_submit).count();
            ++s->st.completed;
            s->st.cell_updates += (uint64_t)(q->ring.N * q->ring.nt);
            finish_locked(s, q, DONE, HEAT_OK);
        } else {
            q->p->status = HEAT_EDEVICE;
            (void)fail(HEAT_EDEVICE, "server stage-out: %s", msg.c_str());
            finish_locked(s, q, FAILED, HEAT_EDEVICE);
        }
    }
}

static void stage_in_loop(heat_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        s->cv_in.wait(lk, [&] { return s->stop || !s->h2d.empty(); });
        if (s->h2d.empty()) break;
        Req *q = s->h2d.front();
        s->h2d.pop_front();
        lk.unlock();
        const int64_t N = q->ring.N;
        // binary64 input lands in the state buffer (FP64) or in the scratch
        // buffer, to be rounded to binary32 on the compute stream
        void *dst = q->ring.precision == HEAT_FP64 ? q->ring.d_u : q->ring.d_work;
        hipError_t e = hipMemcpyAsync(dst, q->p->u0, (size_t)N * 8, hipMemcpyHostToDevice, s->copy_in);
        if (e == hipSuccess) e = hipStreamSynchronize(s->copy_in);
        lk.lock();
        if (e != hipSuccess) {
            q->p->status = HEAT_EDEVICE;
            finish_locked(s, q, FAILED, fail_hip(e, "server stage-in"));
        } else if (s->fatal) {
            q->p->status = s->fatal;
            finish_locked(s, q, FAILED, fail(s->fatal, "server failed earlier: device error"));
        } else if (q->cancel) {
            finish_locked(s, q, CANCELLED, HEAT_ECANCELED);
        } else {
            q->state = READY;
            s->ready.push_back(q);
            s->cv_sched.notify_one();
        }
    }
}

// ------------------------------------------------------------ scheduler
static int run_tick(heat_server *s, std::vector<Req *> &act, uint64_t tick) {
    // group by precision and kernel class; every ring advances the rounds
    // that cover the tick's steps
    std::vector<BatchRing> groups[TABLE_GROUPS];
    for (Req *q : act)
        groups[q->ring.precision * 3 + (q->br.G > 1 ? 2 : (q->br.K == 64))].push_back(q->br);
    const int slot = (int)(tick & 1);
    HEAT_HIP(hipEventSynchronize(s->table_ev[slot]));   // the tick that used this slot is done
    char *dt = s->d_tables + slot * s->table_slot_bytes;
    char *ht = s->h_tables + slot * s->table_slot_bytes;
    const size_t per_group = s->table_slot_bytes / TABLE_GROUPS;
    for (int g = 0; g < TABLE_GROUPS; ++g) {
        if (groups[g].empty()) continue;
        BatchLaunch L;
        int rc = L.build(groups[g], g / 3, s->tick_steps ? 0 : TICK_ROUNDS, s->tick_steps);
        if (!rc) rc = L.enqueue_rounds(dt + g * per_group, ht + g * per_group, s->compute);
        if (rc) return rc;
    }
    HEAT_HIP(hipEventRecord(s->table_ev[slot], s->compute));
    return HEAT_OK;
}

static void sched_loop(heat_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        // admission in arrival order while memory and slots allow
        while (!s->stop && !s->fatal && !s->queue.empty() && s->slots_used < s->max_slots) {
            Req *q = s->queue.front();
            size_t off = 0;
            if (!s->arena.alloc(q->bytes, &off)) break;
            s->queue.pop_front();
            ++s->slots_used;
            q->holds = true;
            q->off = off;
            char *b = s->arena.base() + off;
            const size_t es = storage_bytes(q->ring.precision);
            q->ring.d_u = b;
            q->ring.d_work = b + Arena::round((size_t)q->ring.N * es);
            q->d_sums = (double *)(b + Arena::round((size_t)q->ring.N * es) +
                                   Arena::round((size_t)q->ring.N * std::max<size_t>(es, 8)));
            if (s->slots_used > SERVER_BUSY_SLOTS)
                describe_ring_batch(q->ring, &q->br);
            else
                describe_ring(q->ring, &q->br, SERVER_CELLS_PER_LANE);
            q->state = STAGING;
            ++s->st.admitted;
            s->h2d.push_back(q);
            s->cv_in.notify_one();
        }
        s->st.hbm_in_use = s->arena.used();
        s->st.hbm_peak = s->arena.peak();
        s->st.queued = (int32_t)s->queue.size();
        if (s->stop) break;
        std::vector<Req *> fresh;
        fresh.swap(s->ready);
        // drop cancelled residents once the device no longer touches them
        bool any_cancel = false;
        for (Req *q : s->active) any_cancel |= q->cancel;
        for (Req *q : fresh) any_cancel |= q->cancel;
        if (any_cancel) {
            lk.unlock();
            (void)hipStreamSynchronize(s->compute);
            lk.lock();
            auto drop = [&](std::vector<Req *> &v) {
                v.erase(std::remove_if(v.begin(), v.end(),
                                       [&](Req *q) {
                                           if (!q->cancel) return false;
                                           finish_locked(s, q, CANCELLED, HEAT_ECANCELED);
                                           return true;
                                       }),
                        v.end());
            };
            drop(s->active);
            drop(fresh);
        }
        if (s->active.empty() && fresh.empty()) {
            s->st.active = 0;
            s->cv_sched.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        lk.unlock();
        int rc = HEAT_OK;
        // newly staged requests: round FP32 inputs, take the initial sum
        for (Req *q : fresh) {
            hipError_t e = hipSuccess;
            if (q->ring.precision != HEAT_FP64)
                e = launch_f64_to_f32((const double *)q->ring.d_work, (float *)q->ring.d_u,
                                      q->ring.N, s->compute, q->shift);
            if (e == hipSuccess)
                e = launch_sum(q->ring.precision, q->ring.d_u, q->ring.N, s->d_partial, q->d_sums,
                               s->compute);
            if (e != hipSuccess) rc = fail_hip(e, "server admit");
        }
        lk.lock();
        for (Req *q : fresh) {
            q->state = ACTIVE;
            s->active.push_back(q);
        }
        std::vector<Req *> act = s->active;
        const uint64_t tick = s->tick++;
        s->st.active = (int32_t)act.size();
        lk.unlock();
        if (!rc) rc = run_tick(s, act, tick);
        // progress bookkeeping and completions (all enqueued after the tick)
        std::vector<Req *> finished;
        for (Req *q : act) {
            q->br.round0 += scheduled_rounds(q->br, s->tick_steps ? 0 : TICK_ROUNDS, s->tick_steps);
            if (q->br.round0 >= q->br.rounds + q->br.copy_round) finished.push_back(q);
        }
        for (Req *q : finished) {
            hipError_t e = launch_sum(q->ring.precision, q->ring.d_u, q->ring.N, s->d_partial,
                                      q->d_sums + 1, s->compute);
            if (e == hipSuccess && q->ring.precision != HEAT_FP64)
                e = launch_f32_to_f64((const float *)q->ring.d_u, (double *)q->ring.d_work,
                                      q->ring.N, s->compute, q->shift);
            // system-scope release: the DMA engines read the result from memory
            if (e == hipSuccess)
                e = hipEventCreateWithFlags(&q->fin, hipEventDisableTiming | hipEventReleaseToSystem);
            if (e == hipSuccess) e = hipEventRecord(q->fin, s->compute);
            if (e != hipSuccess && !rc) rc = fail_hip(e, "server complete");
        }
        lk.lock();
        ++s->st.ticks;
        if (rc) {
            // A device error poisons the server: no more admissions; once the
            // compute stream has drained (the tick's kernels may still be
            // writing the arena) every request it holds fails and its block
            // is released.
            s->fatal = rc;
            const std::string msg = heat_last_error();
            lk.unlock();
            (void)hipStreamSynchronize(s->compute);
            lk.lock();
            (void)fail(rc, "%s", msg.c_str());
            fail_all_locked(s, rc);
            continue;
        }
        for (Req *q : finished) {
            s->active.erase(std::find(s->active.begin(), s->active.end(), q));
            q->state = DRAINING;
            s->d2h.push_back(q);
        }
        if (!finished.empty()) s->cv_out.notify_one();
    }
}

// DMA agents of the server's device and the stage-out lanes' pinned chunks
// and signals (ROCr is initialised here and shut down in release_out_lanes;
// ROCr counts its initialisations, HIP holds its own).
static int setup_out_lanes(heat_server *s) {
    hipDeviceProp_t prop;
    HEAT_HIP(hipGetDeviceProperties(&prop, s->device));
    s->dma.bdf = ((uint32_t)prop.pciBusID << 8) | ((uint32_t)prop.pciDeviceID << 3);
    s->dma.domain = (uint32_t)prop.pciDomainID;
    hsa_status_t st = hsa_init();
    if (st != HSA_STATUS_SUCCESS) return hsa_fail(st, "hsa_init");
    s->hsa_up = true;
    st = hsa_iterate_agents(find_agents, &s->dma);
    if (st != HSA_STATUS_SUCCESS) return hsa_fail(st, "hsa_iterate_agents");
    if (!s->dma.gpu_found || !s->dma.cpu_found)
        return fail(HEAT_EDEVICE, "no ROCr agent for device %d (PCI %x:%x) or the host",
                    s->device, s->dma.domain, s->dma.bdf);
    for (OutLane &L : s->out) {
        for (int b = 0; b < 2; ++b) {
            HEAT_HIP(hipHostMalloc((void **)&L.buf[b], STAGE_OUT_CHUNK, hipHostMallocDefault));
            if ((st = hsa_signal_create(0, 0, nullptr, &L.sig[b])) != HSA_STATUS_SUCCESS)
                return hsa_fail(st, "hsa_signal_create");
        }
        HEAT_HIP(hipHostMalloc((void **)&L.sums, 2 * sizeof(double), hipHostMallocDefault));
        if ((st = hsa_signal_create(0, 0, nullptr, &L.sig_sums)) != HSA_STATUS_SUCCESS)
            return hsa_fail(st, "hsa_signal_create");
    }
    return HEAT_OK;
}

static void release_out_lanes(heat_server *s) {
    for (OutLane &L : s->out) {
        for (int b = 0; b < 2; ++b) {
            if (L.buf[b]) (void)hipHostFree(L.buf[b]);
            if (L.sig[b].handle) (void)hsa_signal_destroy(L.sig[b]);
            L.buf[b] = nullptr;
            L.sig[b].handle = 0;
        }
        if (L.sums) (void)hipHostFree(L.sums);
        if (L.sig_sums.handle) (void)hsa_signal_destroy(L.sig_sums);
        L.sums = nullptr;
        L.sig_sums.handle = 0;
    }
    if (s->hsa_up) (void)hsa_shut_down();
    s->hsa_up = false;
}

// ================================================================== C ABI

extern "C" {

int heat_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t max_queue,
                       heat_server **out) {
    if (!out) return fail(HEAT_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_slots < 0 || max_queue < 0) return fail(HEAT_EINVAL, "negative limits");
    heat_server *s = new heat_server();
    s->max_slots = max_slots ? max_slots : 4096;
    s->max_queue = max_queue ? max_queue : 65536;
    if (const char *ts = std::getenv("HEAT_SERVER_TICK_STEPS")) {
        const long v = std::strtol(ts, nullptr, 10);
        if (v >= 1 && v <= (1 << 20)) s->tick_steps = (int32_t)v;
    }
    int rc = HEAT_OK;
    auto bail = [&](int code) {
        if (s->d_partial) (void)hipFree(s->d_partial);
        if (s->d_tables) (void)hipFree(s->d_tables);
        if (s->h_tables) (void)hipHostFree(s->h_tables);
        for (hipEvent_t &e : s->table_ev)
            if (e) (void)hipEventDestroy(e);
        if (s->compute) (void)hipStreamDestroy(s->compute);
        if (s->copy_in) (void)hipStreamDestroy(s->copy_in);
        release_out_lanes(s);
        s->arena.destroy();
        delete s;
        return code;
    };
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) return bail(fail_hip(e, "hipGetDevice"));
    size_t fr = 0, tot = 0;
    e = hipMemGetInfo(&fr, &tot);
    if (e != hipSuccess) return bail(fail_hip(e, "hipMemGetInfo"));
    size_t budget = hbm_budget_bytes ? hbm_budget_bytes : (size_t)(0.8 * (double)fr);
    budget &= ~size_t(255);
    if (budget < (1u << 20)) return bail(fail(HEAT_EINVAL, "budget below 1 MiB"));
    if ((rc = s->arena.init(budget))) return bail(rc);
    if ((e = hipStreamCreateWithFlags(&s->compute, hipStreamNonBlocking)) != hipSuccess)
        return bail(fail_hip(e, "hipStreamCreate"));
    if ((e = hipStreamCreateWithFlags(&s->copy_in, hipStreamNonBlocking)) != hipSuccess)
        return bail(fail_hip(e, "hipStreamCreate"));
    if ((rc = setup_out_lanes(s))) return bail(rc);
    if ((e = hipMalloc((void **)&s->d_partial, SUM_BLOCKS * sizeof(double))) != hipSuccess)
        return bail(fail_hip(e, "hipMalloc(partials)"));
    const size_t group = Arena::round((size_t)s->max_slots * sizeof(BatchRing)) +
                         Arena::round(((size_t)s->max_slots + 1) * 8);
    s->table_slot_bytes = TABLE_GROUPS * group;
    if ((e = hipMalloc((void **)&s->d_tables, 2 * s->table_slot_bytes)) != hipSuccess)
        return bail(fail_hip(e, "hipMalloc(tables)"));
    if ((e = hipHostMalloc((void **)&s->h_tables, 2 * s->table_slot_bytes, 0)) != hipSuccess)
        return bail(fail_hip(e, "hipHostMalloc(tables)"));
    for (hipEvent_t &ev : s->table_ev) {
        if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
            return bail(fail_hip(e, "hipEventCreate"));
        if ((e = hipEventRecord(ev, s->compute)) != hipSuccess)
            return bail(fail_hip(e, "hipEventRecord"));
    }
    s->st.hbm_budget = budget;
    s->sched = std::thread(sched_loop, s);
    s->stager_in = std::thread(stage_in_loop, s);
    for (int i = 0; i < STAGE_OUT_LANES; ++i) s->out[i].th = std::thread(stage_out_loop, s, i);
    *out = s;
    return HEAT_OK;
}

int heat_submit(heat_server *s, heat_problem *p, uint64_t *ticket) {
    if (!s || !p || !ticket) return fail(HEAT_EINVAL, "NULL argument");
    heat_ring g{p->N, p->nt, p->r, p->precision, p->nparts, (void *)16, (void *)16};
    int rc = validate_ring(g);
    if (rc) return rc;
    if (!p->u0 || !p->u_out) return fail(HEAT_EINVAL, "u0/u_out is NULL");
    if (!std::isfinite(p->shift)) return fail(HEAT_EINVAL, "shift must be finite");
    const size_t bytes = footprint(p->N, p->precision);
    std::lock_guard<std::mutex> lk(s->mu);
    ++s->st.submitted;
    if (s->fatal) return fail(s->fatal, "server failed earlier: device error");
    if (bytes > s->arena.cap()) {
        ++s->st.rejected;
        return fail(HEAT_ENOMEM, "request needs %zu bytes, budget is %zu", bytes, s->arena.cap());
    }
    if ((int64_t)s->queue.size() >= s->max_queue) {
        ++s->st.rejected;
        return fail(HEAT_EBUSY, "admission queue full (%d)", s->max_queue);
    }
    Req *q = new Req();
    q->ticket = s->next_ticket++;
    q->p = p;
    q->shift = p->precision == HEAT_FP64 ? 0.0 : p->shift;
    q->ring = g;
    q->ring.d_u = q->ring.d_work = nullptr;
    q->bytes = bytes;
    q->t_submit = Clock::now();
    p->status = HEAT_PENDING;
    s->reqs[q->ticket] = q;
    s->queue.push_back(q);
    *ticket = q->ticket;
    s->cv_sched.notify_one();
    return HEAT_OK;
}

static int consume_locked(heat_server *s, std::unordered_map<uint64_t, Req *>::iterator it) {
    Req *q = it->second;
    const int rc = q->state == DONE ? HEAT_OK : q->rc;
    const std::string msg = q->msg;
    s->reqs.erase(it);
    delete q;
    if (rc == HEAT_ECANCELED) return fail(rc, "request was cancelled");
    if (rc < 0) return fail(rc, "request failed: %s", msg.c_str());
    return rc;
}

int heat_poll(heat_server *s, uint64_t ticket) {
    if (!s) return fail(HEAT_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(HEAT_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    if (finished_state(it->second->state)) return consume_locked(s, it);
    return HEAT_PENDING;
}

// Wait until `ticket` is finished or gone.  Another thread may consume the
// ticket (poll, wait, cancel) and free its request meanwhile, so the request
// is looked up again on every wake and never held across the wait.  Returns
// the ticket's entry, or end() when another call consumed it.
static std::unordered_map<uint64_t, Req *>::iterator
wait_finished_locked(heat_server *s, std::unique_lock<std::mutex> &lk, uint64_t ticket) {
    auto it = s->reqs.find(ticket);
    s->cv_done.wait(lk, [&] {
        it = s->reqs.find(ticket);
        return it == s->reqs.end() || finished_state(it->second->state);
    });
    return it;
}

int heat_wait(heat_server *s, uint64_t ticket) {
    if (!s) return fail(HEAT_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    if (!s->reqs.count(ticket))
        return fail(HEAT_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    auto it = wait_finished_locked(s, lk, ticket);
    if (it == s->reqs.end())
        return fail(HEAT_ENOENT, "ticket %llu was consumed by another call", (unsigned long long)ticket);
    return consume_locked(s, it);
}

int heat_cancel(heat_server *s, uint64_t ticket) {
    if (!s) return fail(HEAT_EINVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return fail(HEAT_ENOENT, "unknown ticket %llu", (unsigned long long)ticket);
    Req *q = it->second;
    if (q->state == QUEUED) {
        s->queue.erase(std::find(s->queue.begin(), s->queue.end(), q));
        q->state = CANCELLED;
        ++s->st.cancelled;
    } else if (!finished_state(q->state)) {
        // resident: the scheduler (or the stage-in thread) lets go of it; a request
        // already draining completes normally
        q->cancel = true;
        s->cv_sched.notify_one();
        it = wait_finished_locked(s, lk, ticket);
        if (it == s->reqs.end())
            return fail(HEAT_ENOENT, "ticket %llu was consumed by another call",
                        (unsigned long long)ticket);
        q = it->second;
    }
    q->p->status = HEAT_ECANCELED;
    s->reqs.erase(it);
    delete q;
    s->cv_done.notify_all();   // other waiters on this ticket find it gone
    return HEAT_OK;
}

int heat_server_get_stats(heat_server *s, heat_server_stats *out) {
    if (!s || !out) return fail(HEAT_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    s->st.hbm_in_use = s->arena.used();
    s->st.hbm_peak = s->arena.peak();
    s->st.queued = (int32_t)s->queue.size();
    *out = s->st;
    return HEAT_OK;
}

int heat_server_destroy(heat_server *s) {
    if (!s) return HEAT_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_sched.notify_all();
        s->cv_in.notify_all();
        s->cv_out.notify_all();
    }
    if (s->sched.joinable()) s->sched.join();
    if (s->stager_in.joinable()) s->stager_in.join();
    for (OutLane &L : s->out)
        if (L.th.joinable()) L.th.join();
    (void)hipStreamSynchronize(s->compute);
    (void)hipStreamSynchronize(s->copy_in);
    for (auto &kv : s->reqs) {
        Req *q = kv.second;
        if (q->fin) (void)hipEventDestroy(q->fin);
        if (q->state != DONE && q->state != FAILED) q->p->status = HEAT_ECANCELED;
        delete q;
    }
    s->reqs.clear();
    (void)hipFree(s->d_partial);
    (void)hipFree(s->d_tables);
    (void)hipHostFree(s->h_tables);
    for (hipEvent_t &e : s->table_ev) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(s->compute);
    (void)hipStreamDestroy(s->copy_in);
    release_out_lanes(s);
    s->arena.destroy();
    delete s;
    return HEAT_OK;
}

}  // extern "C"
