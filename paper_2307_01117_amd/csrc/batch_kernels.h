// batch_kernels.h -- kernels of the batching form as templates: one round of
// many rings per launch (k_batch_round, and k_batch_round_x whose workgroup
// waves share a tile), the persistent flag-synchronised variant (k_batch),
// and their launchers.  The per-tile work is window_tile.  batch_kernels.hip
// instantiates them for binary64 and binary32, kernels_f32c.hip for the
// compensated form (built with its own instruction scheduler); no other file
// may instantiate them.
#pragma once

#include <hip/hip_runtime.h>

#include "heat_device.h"
#include "heat_internal.h"
#include "window.h"

namespace heat {

// =============================================================== BATCHING
// One persistent launch for many rings.  Work items (round k, ring p, tile t)
// are numbered round-major: all tiles of all rings still running in round 0,
// then round 1, ...  Rings are sorted by their number of rounds (descending)
// so the rings alive in round k are a prefix.  Item (k, p, t) reads tiles
// t-1, t, t+1 of ring p as written in round k-1, so it waits until their
// epoch counters reach k; when done it raises its own counter to k + 1
// (together with the other tiles of its chunk in the same ring and round).
// Items are claimed in increasing order from one atomic counter, and every
// item waits only on items with smaller numbers, which were claimed earlier
// by running wavefronts: the earliest unfinished item can always proceed, so
// the launch drains.  A wait longer than spin_limit sets status[0] and every
// wavefront leaves, so a bug can never hang the device.

__device__ __forceinline__ int64_t upper_bound_i64(const int64_t *a, int64_t n, int64_t x) {
    // first index i in [0, n) with a[i] > x (n if none)
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= x)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// Spin until the epoch counter *f reaches `need`.  The polls are relaxed
// (coherent at agent scope, no cache maintenance): an acquiring poll would
// invalidate the XCD's L2 on every iteration, under the feet of the waves
// that are working.  The caller issues one acquire fence after all of an
// item's waits; with the writer's release fence before its counter store,
// that orders the tile data after the counters.
__device__ __forceinline__ bool wait_epoch(const BatchPlanDev &plan, const uint32_t *f,
                                           uint32_t need) {
    int64_t spins = 0;
    while (true) {
        const uint32_t v = __hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (__builtin_amdgcn_readfirstlane(v) >= need) break;
        if (++spins > plan.spin_limit) {
            __hip_atomic_store(plan.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        if ((spins & 63) == 0 &&
            __hip_atomic_load(plan.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
    return true;
}

template <class P, int K>
__global__ void __launch_bounds__(256) k_batch(BatchPlanDev plan) {
    using T = typename P::T;
    const int lane = threadIdx.x & 63;
    while (true) {
        unsigned long long x0 = 0;
        if (lane == 0) x0 = atomicAdd(plan.work, (unsigned long long)plan.chunk);
        x0 = __shfl(x0, 0);
        if ((int64_t)x0 >= plan.total_items) return;
        if (__hip_atomic_load(plan.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
            return;
        int64_t x = (int64_t)x0;
        const int64_t x_end = x + plan.chunk < plan.total_items ? x + plan.chunk : plan.total_items;
        // decode the first item, then walk forward
        int64_t k = upper_bound_i64(plan.round_start, plan.max_rounds + 1, x) - 1;
        int64_t y = x - plan.round_start[k];
        int64_t p = upper_bound_i64(plan.tile_prefix, plan.active[k] + 1, y) - 1;
        int64_t t = y - plan.tile_prefix[p];
        // Tiles computed but not yet published: [pub_lo, pub_lo + pub_n) of
        // one ring in one round.  They are published together (one release
        // fence, then their counters) at the end of the chunk, or before the
        // walk moves on to another ring or round: an item waits only for
        // tiles of the previous round, so never for its own unpublished ones.
        uint32_t *pub_fl = nullptr;
        uint32_t pub_epoch = 0;
        int64_t pub_lo = 0, pub_n = 0;
        auto publish = [&]() {
            if (pub_n == 0) return;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_wave_barrier();
            if (lane == 0)
                for (int64_t i = 0; i < pub_n; ++i)
                    __hip_atomic_store(pub_fl + pub_lo + i, pub_epoch, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            pub_n = 0;
        };
        for (; x < x_end; ++x) {
            const BatchRing &R = plan.rings[p];
            const int64_t tiles = R.tiles;
            uint32_t *fl = plan.flags + R.flag_base;
            const uint32_t need = (uint32_t)k;
            if (pub_n && (pub_fl != fl || pub_epoch != (uint32_t)(k + 1))) publish();
            // Wait for every tile whose cells lie within H of this tile on
            // the ring: exactly the tiles this window reads (read after
            // write) and the tiles whose windows read this tile's cells in
            // the other buffer (write after read; the relation is symmetric).
            // With a last tile shorter than H this reaches two tiles away.
            if (!wait_epoch(plan, fl + t, need)) return;
            const int64_t last_len = R.N - (tiles - 1) * R.W;
            bool ok = true;
            int64_t acc = 0, q = t;
            for (int64_t g = 0; ok && g + 1 < tiles && acc < R.H; ++g) {
                q = q == 0 ? tiles - 1 : q - 1;
                ok = wait_epoch(plan, fl + q, need);
                acc += q == tiles - 1 ? last_len : R.W;
            }
            acc = 0;
            q = t;
            for (int64_t g = 0; ok && g + 1 < tiles && acc < R.H; ++g) {
                q = q + 1 == tiles ? 0 : q + 1;
                ok = wait_epoch(plan, fl + q, need);
                acc += q == tiles - 1 ? last_len : R.W;
            }
            if (!ok) return;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // one for all the waits above
            const int64_t b = t * R.W;
            if (k < R.rounds) {
                const T *src = reinterpret_cast<const T *>(R.buf[k & 1]);
                T *dst = reinterpret_cast<T *>(R.buf[(k + 1) & 1]);
                const int64_t done = k * (int64_t)R.T;
                const int steps = (int)((R.nt - done) < R.T ? (R.nt - done) : R.T);
                window_tile<P, K, FORM_ALTERNATING>(src, dst, R.N, R.H, steps, R.r, b, R.W,
                                                    R.vec_ok != 0, lane);
            } else {
                // copy-back round: the final state sits in buf[1]
                const T *src = reinterpret_cast<const T *>(R.buf[1]);
                T *dst = reinterpret_cast<T *>(R.buf[0]);
                const int64_t wlen = (R.N - b) < R.W ? (R.N - b) : R.W;
                for (int64_t i = lane; i < wlen; i += 64) dst[b + i] = src[b + i];
            }
            // published with the chunk's other tiles of this ring and round
            // (the release fence there orders their stores before the
            // counters, which then need no release of their own)
            if (pub_n == 0) {
                pub_fl = fl;
                pub_epoch = (uint32_t)(k + 1);
                pub_lo = t;
            }
            ++pub_n;
            // next item in numbering order
            if (++t == tiles) {
                t = 0;
                if (++p == plan.active[k]) {
                    p = 0;
                    ++k;
                }
            }
        }
        publish();
    }
}

// ========================================================= ROUND-BATCHING
// One launch advances every ring still running by one round: the flat item
// list is the tiles of the active rings (rings sorted by rounds, so the
// active ones are a prefix), one wavefront per tile.  The kernel boundary is
// the round barrier, so no flags or cross-wave waits are needed.  Item ids
// are wave-uniform, so the ring lookup runs on the scalar unit.

template <class P, int K, int FORM>
__global__ void __launch_bounds__(256)
k_batch_round(const BatchRing *__restrict__ rings, const int64_t *__restrict__ tile_prefix,
              int32_t k, int32_t active, int64_t items) {
    using T = typename P::T;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t id = xcd_remap(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + wave;
    if (id >= items) return;
    const int64_t p = upper_bound_i64(tile_prefix, (int64_t)active + 1, id) - 1;
    const int64_t t = id - tile_prefix[p];
    const BatchRing &R = rings[p];
    const int64_t b = t * R.W;
    const int32_t kk = R.round0 + k;   // this ring's own round index
    if (kk < R.rounds) {
        const T *src = reinterpret_cast<const T *>(R.buf[kk & 1]);
        T *dst = reinterpret_cast<T *>(R.buf[(kk + 1) & 1]);
        const int64_t done = (int64_t)kk * R.T;
        const int steps = (int)((R.nt - done) < R.T ? (R.nt - done) : R.T);
        window_tile<P, K, FORM>(src, dst, R.N, R.H, steps, R.r, b, R.W, R.vec_ok != 0, lane);
    } else {
        // copy-back round: after an odd number of rounds the state sits in buf[1]
        const T *src = reinterpret_cast<const T *>(R.buf[1]);
        T *dst = reinterpret_cast<T *>(R.buf[0]);
        const int64_t wlen = (R.N - b) < R.W ? (R.N - b) : R.W;
        for (int64_t i = lane; i < wlen; i += 64) dst[b + i] = src[b + i];
    }
}

// Same round over tiles shared by the G waves of a workgroup (one tile per
// workgroup, edge cells swapped through LDS; see window.h).
template <class P, int K, int FORM>
__global__ void __launch_bounds__(256)
k_batch_round_x(const BatchRing *__restrict__ rings, const int64_t *__restrict__ tile_prefix,
                int32_t k, int32_t active, int64_t items) {
    using T = typename P::T;
    extern __shared__ __align__(16) unsigned char heat_batch_xlds[];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int G = blockDim.x >> 6;
    const int64_t id = xcd_remap(blockIdx.x, gridDim.x);   // one tile per workgroup
    if (id >= items) return;
    const int64_t p = upper_bound_i64(tile_prefix, (int64_t)active + 1, id) - 1;
    const int64_t t = id - tile_prefix[p];
    const BatchRing &R = rings[p];
    const int64_t b = t * R.W;
    const int32_t kk = R.round0 + k;
    if (kk < R.rounds) {
        const T *src = reinterpret_cast<const T *>(R.buf[kk & 1]);
        T *dst = reinterpret_cast<T *>(R.buf[(kk + 1) & 1]);
        const int64_t done = (int64_t)kk * R.T;
        const int steps = (int)((R.nt - done) < R.T ? (R.nt - done) : R.T);
        window_tile<P, K, FORM, 4>(src, dst, R.N, R.H, steps, R.r, b, R.W, R.vec_ok != 0,
                                      lane, nullptr, nullptr, 0, G, wave,
                                      reinterpret_cast<T *>(heat_batch_xlds));
    } else {
        const T *src = reinterpret_cast<const T *>(R.buf[1]);
        T *dst = reinterpret_cast<T *>(R.buf[0]);
        const int64_t wlen = (R.N - b) < R.W ? (R.N - b) : R.W;
        for (int64_t i = threadIdx.x; i < wlen; i += blockDim.x) dst[b + i] = src[b + i];
    }
}

template <class P, int K>
inline hipError_t launch_batch_t(const BatchPlanDev &plan, int grid, int wpg, hipStream_t st) {
    hipLaunchKernelGGL((k_batch<P, K>), dim3(grid), dim3(64 * wpg), 0, st, plan);
    return hipGetLastError();
}

template <class P, int K, int FORM>
inline hipError_t launch_batch_round_t(const BatchRing *rings, const int64_t *tile_prefix, int k,
                                       int active, int64_t items, int wpg, hipStream_t st) {
    const int64_t blocks = (items + wpg - 1) / wpg;
    hipLaunchKernelGGL((k_batch_round<P, K, FORM>), dim3((unsigned)blocks), dim3(64 * wpg), 0, st,
                       rings, tile_prefix, k, active, items);
    return hipGetLastError();
}

template <class P, int K, int FORM>
inline hipError_t launch_batch_round_x(const BatchRing *rings, const int64_t *tile_prefix, int k,
                                       int active, int64_t items, int G, hipStream_t st) {
    const unsigned lds = (unsigned)exchange_lds_bytes<P>(K, G, 4);
    hipLaunchKernelGGL((k_batch_round_x<P, K, FORM>), dim3((unsigned)items), dim3(64 * G), lds, st,
                       rings, tile_prefix, k, active, items);
    return hipGetLastError();
}

template <class P, int K>
inline int occupancy_blocks(int wpg) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<P, K>, 64 * wpg, 0) != hipSuccess)
        return 0;
    return nb;
}

}  // namespace heat
