// kernels.hip -- HIP kernels (gfx950, wave64) of the periodic 1D heat stencil
// and their host launchers.
//
// Operation: the explicit-Euler step of the paper's Eq. (heat:discrete) on a
// periodic ring (Section 2), applied nt times with a Jacobi double buffer.
// The paper's per-step ghost-zone exchange between segments (Section 2, last
// paragraph) appears here at three levels:
//   * between lanes of a wavefront: DPP rotates (no memory traffic);
//   * between tiles of one round: overlapping windows read from HBM;
//   * between rounds: the kernel boundary (plain form) or per-tile epoch
//     counters (fused batch form).
#include <hip/hip_runtime.h>

#include "heat_device.h"
#include "heat_internal.h"

namespace heat {

// ====================================================================== TB
// Window of one wavefront: lane L holds cells [L*K, L*K + K) of a window of
// 64*K cells that starts at ring position g0 = b - H.  After `steps` <= H
// steps the cells [H, 64*K - H) are exact; they are the tile's output
// [b, b + W).  Rings shorter than the window are handled by reading the
// window modulo N (the periodic extension evolves exactly like the ring).

template <class P, int K>
__device__ __forceinline__ void window_load(const typename P::T *__restrict__ src, int64_t N,
                                            int64_t g0, bool fast, int lane,
                                            typename P::T (&v)[K]) {
    using T = typename P::T;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = P::VEC;
    if (fast) {
        const VT *p = reinterpret_cast<const VT *>(src + g0 + (int64_t)lane * K);
#pragma unroll
        for (int j = 0; j < K / VEC; ++j) {
            VT x = p[j];
            const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
            for (int k = 0; k < VEC; ++k) v[j * VEC + k] = xs[k];
        }
    } else {
        // Windows that wrap the ring (or overhang a short ring) gather cell by
        // cell.  Groups of 8 loads are fenced off from each other so the
        // addresses of the whole window are never live at once: this path is
        // rare, and its register peak would otherwise set the whole kernel's
        // occupancy.
#pragma unroll
        for (int j = 0; j < K; ++j) {
            v[j] = src[wrap_index(g0 + (int64_t)lane * K + j, N)];
            if ((j & 7) == 7) __builtin_amdgcn_sched_barrier(0);
        }
    }
}

template <class P, int K>
__device__ __forceinline__ void window_store(typename P::T *__restrict__ dst, int64_t b, int H,
                                             int64_t W, int64_t wlen, bool fast, int lane,
                                             const typename P::T (&v)[K]) {
    using T = typename P::T;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = P::VEC;
    const int64_t g0 = b - H;
    if (fast) {
        // H and W are multiples of 4, so a 16-byte group never straddles the
        // output boundaries.
        VT *p = reinterpret_cast<VT *>(dst + g0 + (int64_t)lane * K);
#pragma unroll
        for (int j = 0; j < K / VEC; ++j) {
            const int pos = lane * K + j * VEC;
            if (pos >= H && pos < H + W) {
                VT x;
                T *xs = reinterpret_cast<T *>(&x);
#pragma unroll
                for (int k = 0; k < VEC; ++k) xs[k] = v[j * VEC + k];
                p[j] = x;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int pos = lane * K + j;
            if (pos >= H && pos < H + wlen) dst[b + (pos - H)] = v[j];
        }
    }
}

// Process one tile: output cells [b, b + min(W, N - b)).  PP selects the
// ping-pong register form (no register rotation, twice the state registers).
// binary64 sum of the cells this tile owns (window positions [H, H + wlen)),
// lane by lane in index order, then a fixed butterfly over the wave; lane 0's
// value is returned.
template <int K, class T>
__device__ __forceinline__ double tile_sum(const T (&v)[K], int lane, int H, int64_t wlen) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int pos = lane * K + j;
        if (pos >= H && pos < H + wlen) s += (double)v[j];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    return s;
}

// Register forms of the T-step loop.
enum RegForm { FORM_INPLACE = 1, FORM_PINGPONG = 2, FORM_ALTERNATING = 3 };

// part_in / part_out (may be NULL): per-tile binary64 sums of the state
// before and after the round, written at index `tile` -- the conservation
// checksum fused into the first and last rounds (no extra pass over HBM).
template <class P, int K, int FORM>
__device__ __forceinline__ void window_tile(const typename P::T *__restrict__ src,
                                            typename P::T *__restrict__ dst, int64_t N, int H,
                                            int steps, typename P::T r, int64_t b, int64_t W,
                                            bool vec_ok, int lane, double *part_in = nullptr,
                                            double *part_out = nullptr, int64_t tile = 0) {
    using T = typename P::T;
    constexpr int WIN = 64 * K;
    const int64_t g0 = b - H;
    const int64_t wlen = (N - b) < W ? (N - b) : W;
    const bool fast = vec_ok && g0 >= 0 && g0 + WIN <= N && wlen == W;
    T v[K];
    window_load<P, K>(src, N, g0, fast, lane, v);
    if (part_in) {
        const double s = tile_sum<K>(v, lane, H, wlen);
        if (lane == 0) part_in[tile] = s;
    }
    if constexpr (P::COMP) {
        T e[K];
#pragma unroll
        for (int j = 0; j < K; ++j) e[j] = T(0);
        if constexpr (FORM == FORM_PINGPONG) {
            T v2[K], e2[K];
            int s = 0;
            for (; s + 2 <= steps; s += 2) {
                window_step_comp_pp<K>(v, e, v2, e2, r);
                window_step_comp_pp<K>(v2, e2, v, e, r);
            }
            if (s < steps) window_step_comp<K>(v, e, r);
        } else if constexpr (FORM == FORM_ALTERNATING) {
            int s = 0;
            for (; s + 2 <= steps; s += 2) {
                window_step_comp<K>(v, e, r);
                window_step_comp_bwd<K>(v, e, r);
            }
            if (s < steps) window_step_comp<K>(v, e, r);
        } else {
            for (int s = 0; s < steps; ++s) window_step_comp<K>(v, e, r);
        }
#pragma unroll
        for (int j = 0; j < K; ++j) v[j] = v[j] + e[j];   // fold: u := fl32(u + e)
    } else {
        if constexpr (FORM == FORM_PINGPONG) {
            T v2[K];
            int s = 0;
            for (; s + 2 <= steps; s += 2) {
                window_step_pp<K>(v, v2, r);
                window_step_pp<K>(v2, v, r);
            }
            if (s < steps) window_step<K>(v, r);
        } else if constexpr (FORM == FORM_ALTERNATING) {
            int s = 0;
            for (; s + 2 <= steps; s += 2) {
                window_step<K>(v, r);
                window_step_bwd<K>(v, r);
            }
            if (s < steps) window_step<K>(v, r);
        } else {
            for (int s = 0; s < steps; ++s) window_step<K>(v, r);
        }
    }
    if (part_out) {
        const double s = tile_sum<K>(v, lane, H, wlen);
        if (lane == 0) part_out[tile] = s;
    }
    window_store<P, K>(dst, b, H, W, wlen, fast, lane, v);
}

template <class P, int K, int FORM>
__global__ void __launch_bounds__(512)
k_window(const typename P::T *__restrict__ src, typename P::T *__restrict__ dst, int64_t N,
         int32_t H, int32_t steps, double r, int64_t tiles, int32_t vec_ok, double *part_in,
         double *part_out) {
    const int lane = threadIdx.x & 63;
    const int wpg = blockDim.x >> 6;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t tile = blk * wpg + (threadIdx.x >> 6);
    if (tile >= tiles) return;
    const int64_t W = 64 * K - 2 * (int64_t)H;
    window_tile<P, K, FORM>(src, dst, N, H, steps, (typename P::T)r, tile * W, W, vec_ok != 0,
                            lane, part_in, part_out, tile);
}

// ==================================================================== STEP
// One step per launch.  Wave chunk = U vectors of 16 bytes per lane, laid out
// so that every load instruction is fully coalesced: vector u of lane L holds
// cells base + u*64*VEC + L*VEC + [0, VEC).  Neighbours inside the chunk come
// from the adjacent lanes (DPP); the two cells just outside the chunk are
// read by lanes 0 and 63.

constexpr int STEP_U = 4;

template <class P>
__global__ void __launch_bounds__(512)
k_step(const typename P::T *__restrict__ src, typename P::T *__restrict__ dst, int64_t N, double r_in,
       int64_t chunks, int32_t vec_ok) {
    using T = typename P::T;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = P::VEC;
    constexpr int U = STEP_U;
    constexpr int64_t CH = 64 * VEC * U;
    const int lane = threadIdx.x & 63;
    const int wpg = blockDim.x >> 6;
    const int64_t chunk = xcd_remap(blockIdx.x, gridDim.x) * wpg + (threadIdx.x >> 6);
    if (chunk >= chunks) return;
    const T r = (T)r_in;
    const int64_t base = chunk * CH;
    if (vec_ok && base + CH <= N) {
        T c[U][VEC];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            VT x = *reinterpret_cast<const VT *>(src + base + u * 64 * VEC + lane * VEC);
            const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
            for (int k = 0; k < VEC; ++k) c[u][k] = xs[k];
        }
        T edge = T(0);
        if (lane == 0) edge = src[base == 0 ? N - 1 : base - 1];
        if (lane == 63) edge = src[base + CH == N ? 0 : base + CH];
        T prev_last[U], next_first[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            prev_last[u] = from_prev(c[u][VEC - 1]);
            next_first[u] = from_next(c[u][0]);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T left = lane == 0 ? (u == 0 ? edge : prev_last[u - 1]) : prev_last[u];
            const T right = lane == 63 ? (u == U - 1 ? edge : next_first[u + 1]) : next_first[u];
            VT y;
            T *ys = reinterpret_cast<T *>(&y);
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                const T l = k == 0 ? left : c[u][k - 1];
                const T q = k == VEC - 1 ? right : c[u][k + 1];
                ys[k] = cell_update(l, c[u][k], q, r);
            }
            *reinterpret_cast<VT *>(dst + base + u * 64 * VEC + lane * VEC) = y;
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u) {
#pragma unroll
            for (int k = 0; k < VEC; ++k) {
                const int64_t i = base + u * 64 * VEC + lane * VEC + k;
                if (i < N) {
                    const T l = src[i == 0 ? N - 1 : i - 1];
                    const T q = src[i == N - 1 ? 0 : i + 1];
                    dst[i] = cell_update(l, src[i], q, r);
                }
            }
        }
    }
}

// ===================================================================== SUM
// binary64 sum with a fixed shape: block b owns [b*N/G, (b+1)*N/G), each
// thread keeps a Neumaier-compensated sum of its strided elements, the block
// adds the 256 thread totals in a fixed tree, a second one-block pass does
// the same over the G partials.  Same N -> same order -> same bits.

__device__ __forceinline__ void neumaier_add(double &s, double &c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

__device__ __forceinline__ double block_tree_sum(double v) {
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// Slices start on multiples of 4 elements so the body can use 16-byte
// (binary64) or 16-byte (binary32, 4 at a time) loads when aligned.
template <class T>
__global__ void __launch_bounds__(256) k_sum_partial(const T *__restrict__ u, int64_t N,
                                                     double *__restrict__ partial, int32_t vec_ok) {
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t lo = ((b * N) / G) & ~int64_t(3);
    const int64_t hi = b + 1 == G ? N : (((b + 1) * N) / G) & ~int64_t(3);
    double s = 0.0, c = 0.0;
    if (vec_ok) {
        using VT = typename Vec16<T>::type;
        constexpr int VEC = 16 / sizeof(T);
        const int64_t nv = (hi - lo) / VEC;
        const VT *p = reinterpret_cast<const VT *>(u + lo);
        for (int64_t i = threadIdx.x; i < nv; i += 256) {
            VT x = p[i];
            const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
            for (int k = 0; k < VEC; ++k) neumaier_add(s, c, (double)xs[k]);
        }
        for (int64_t i = lo + nv * VEC + threadIdx.x; i < hi; i += 256) neumaier_add(s, c, (double)u[i]);
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) neumaier_add(s, c, (double)u[i]);
    }
    const double tot = block_tree_sum(s + c);
    if (threadIdx.x == 0) partial[b] = tot;
}

__global__ void __launch_bounds__(256) k_sum_final(const double *__restrict__ partial, int64_t G,
                                                   double *__restrict__ out) {
    double s = 0.0, c = 0.0;
    for (int64_t i = threadIdx.x; i < G; i += 256) neumaier_add(s, c, partial[i]);
    const double tot = block_tree_sum(s + c);
    if (threadIdx.x == 0) out[0] = tot;
}

// ================================================================= CONVERT

__global__ void k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (float)a[i];   // round to nearest even
}

__global__ void k_f32_to_f64(const float *__restrict__ a, double *__restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = (double)a[i];  // exact
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// =============================================================== BATCHING
// One persistent launch for many rings.  Work items (round k, ring p, tile t)
// are numbered round-major: all tiles of all rings still running in round 0,
// then round 1, ...  Rings are sorted by their number of rounds (descending)
// so the rings alive in round k are a prefix.  Item (k, p, t) reads tiles
// t-1, t, t+1 of ring p as written in round k-1, so it waits until their
// epoch counters reach k; when done it raises its own counter to k + 1.
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

__device__ __forceinline__ bool wait_epoch(const BatchPlanDev &plan, const uint32_t *f,
                                           uint32_t need) {
    int64_t spins = 0;
    while (true) {
        const uint32_t v = __hip_atomic_load(f, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
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
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
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
        for (; x < x_end; ++x) {
            const BatchRing &R = plan.rings[p];
            const int64_t tiles = R.tiles;
            uint32_t *fl = plan.flags + R.flag_base;
            const uint32_t need = (uint32_t)k;
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
            const int64_t b = t * R.W;
            if (k < R.rounds) {
                const T *src = reinterpret_cast<const T *>(R.buf[k & 1]);
                T *dst = reinterpret_cast<T *>(R.buf[(k + 1) & 1]);
                const int64_t done = k * (int64_t)R.T;
                const int steps = (int)((R.nt - done) < R.T ? (R.nt - done) : R.T);
                window_tile<P, K, FORM_ALTERNATING>(src, dst, R.N, R.H, steps, (T)R.r, b, R.W,
                                                    R.vec_ok != 0, lane);
            } else {
                // copy-back round: the final state sits in buf[1]
                const T *src = reinterpret_cast<const T *>(R.buf[1]);
                T *dst = reinterpret_cast<T *>(R.buf[0]);
                const int64_t wlen = (R.N - b) < R.W ? (R.N - b) : R.W;
                for (int64_t i = lane; i < wlen; i += 64) dst[b + i] = src[b + i];
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_wave_barrier();
            if (lane == 0)
                __hip_atomic_store(fl + t, (uint32_t)(k + 1), __ATOMIC_RELEASE,
                                   __HIP_MEMORY_SCOPE_AGENT);
            // next item in numbering order
            if (++t == tiles) {
                t = 0;
                if (++p == plan.active[k]) {
                    p = 0;
                    ++k;
                }
            }
        }
    }
}

// ==================================================================== COPY
// Bandwidth probe: every wave moves U 16-byte vectors per lane, coalesced,
// exactly like the fast path of k_step without the arithmetic.

__global__ void __launch_bounds__(256) k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                              int64_t nvec) {
    constexpr int U = STEP_U;
    const int lane = threadIdx.x & 63;
    const int64_t chunk = xcd_remap(blockIdx.x, gridDim.x) * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int64_t base = chunk * 64 * U;
    uint4 x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * 64 + lane;
        if (i < nvec) x[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = base + u * 64 + lane;
        if (i < nvec) dst[i] = x[u];
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
        window_tile<P, K, FORM>(src, dst, R.N, R.H, steps, (T)R.r, b, R.W, R.vec_ok != 0, lane);
    } else {
        // copy-back round: after an odd number of rounds the state sits in buf[1]
        const T *src = reinterpret_cast<const T *>(R.buf[1]);
        T *dst = reinterpret_cast<T *>(R.buf[0]);
        const int64_t wlen = (R.N - b) < R.W ? (R.N - b) : R.W;
        for (int64_t i = lane; i < wlen; i += 64) dst[b + i] = src[b + i];
    }
}

// ================================================================ LAUNCHERS

static inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

template <class P, int K, int FORM>
static hipError_t launch_window_t(const WindowLaunch &a, hipStream_t st) {
    using T = typename P::T;
    const int64_t W = 64 * K - 2 * (int64_t)a.H;
    const int64_t tiles = (a.N + W - 1) / W;
    const int64_t blocks = (tiles + a.wpg - 1) / a.wpg;
    const int vec_ok = aligned16(a.src) && aligned16(a.dst);
    hipLaunchKernelGGL((k_window<P, K, FORM>), dim3((unsigned)blocks), dim3(64 * a.wpg), 0, st,
                       reinterpret_cast<const T *>(a.src), reinterpret_cast<T *>(a.dst), a.N, a.H,
                       a.steps, a.r, tiles, vec_ok, a.part_in, a.part_out);
    return hipGetLastError();
}

// Shapes that cannot hold their state in registers (they would spill).
template <class P, int K, int FORM>
constexpr bool shape_fits() {
    return !(K == 64 && FORM == FORM_PINGPONG && (sizeof(typename P::T) == 8 || P::COMP));
}

template <class P, int FORM>
static hipError_t launch_window_p(const WindowLaunch &a, hipStream_t st) {
    switch (a.K) {
        case 8: return launch_window_t<P, 8, FORM>(a, st);
        case 16: return launch_window_t<P, 16, FORM>(a, st);
        case 32: return launch_window_t<P, 32, FORM>(a, st);
        case 64:
            if constexpr (shape_fits<P, 64, FORM>()) return launch_window_t<P, 64, FORM>(a, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

template <class P>
static hipError_t launch_window_f(const WindowLaunch &a, hipStream_t st) {
    switch (a.form) {
        case FORM_INPLACE: return launch_window_p<P, FORM_INPLACE>(a, st);
        case FORM_PINGPONG: return launch_window_p<P, FORM_PINGPONG>(a, st);
        case FORM_ALTERNATING: return launch_window_p<P, FORM_ALTERNATING>(a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_window(const WindowLaunch &a, hipStream_t st) {
    switch (a.precision) {
        case HEAT_FP64: return launch_window_f<F64>(a, st);
        case HEAT_FP32: return launch_window_f<F32>(a, st);
        case HEAT_FP32C: return launch_window_f<F32C>(a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sum_partials(const double *partial, int64_t n, double *d_out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partial, n, d_out);
    return hipGetLastError();
}

int64_t step_chunk_cells(int precision) {
    return 64 * STEP_U * (precision == HEAT_FP64 ? F64::VEC : F32::VEC);
}

hipError_t launch_step(int precision, const void *src, void *dst, int64_t N, double r, int wpg,
                       hipStream_t st) {
    const int64_t CH = step_chunk_cells(precision);
    const int64_t chunks = (N + CH - 1) / CH;
    const int64_t blocks = (chunks + wpg - 1) / wpg;
    const int vec_ok = aligned16(src) && aligned16(dst);
    if (precision == HEAT_FP64)
        hipLaunchKernelGGL(k_step<F64>, dim3((unsigned)blocks), dim3(64 * wpg), 0, st,
                           reinterpret_cast<const double *>(src), reinterpret_cast<double *>(dst), N,
                           r, chunks, vec_ok);
    else if (precision == HEAT_FP32)
        hipLaunchKernelGGL(k_step<F32>, dim3((unsigned)blocks), dim3(64 * wpg), 0, st,
                           reinterpret_cast<const float *>(src), reinterpret_cast<float *>(dst), N,
                           r, chunks, vec_ok);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_sum(int precision, const void *u, int64_t N, double *partial, double *d_out,
                      hipStream_t st) {
    const int vec_ok = aligned16(u);
    if (precision == HEAT_FP64)
        hipLaunchKernelGGL(k_sum_partial<double>, dim3(SUM_BLOCKS), dim3(256), 0, st,
                           reinterpret_cast<const double *>(u), N, partial, vec_ok);
    else
        hipLaunchKernelGGL(k_sum_partial<float>, dim3(SUM_BLOCKS), dim3(256), 0, st,
                           reinterpret_cast<const float *>(u), N, partial, vec_ok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, st, partial, (int64_t)SUM_BLOCKS, d_out);
    return hipGetLastError();
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st) {
    const int64_t nvec = (int64_t)(bytes / 16);
    const int64_t chunks = (nvec + 64 * STEP_U - 1) / (64 * STEP_U);
    const int64_t blocks = (chunks + 3) / 4;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const uint4 *>(src), reinterpret_cast<uint4 *>(dst), nvec);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

template <class P, int K>
static hipError_t launch_batch_t(const BatchPlanDev &plan, int grid, int wpg, hipStream_t st) {
    hipLaunchKernelGGL((k_batch<P, K>), dim3(grid), dim3(64 * wpg), 0, st, plan);
    return hipGetLastError();
}

template <class P, int K>
static hipError_t launch_batch_round_t(const BatchRing *rings, const int64_t *tile_prefix, int k,
                                       int active, int64_t items, int wpg, hipStream_t st) {
    const int64_t blocks = (items + wpg - 1) / wpg;
    hipLaunchKernelGGL((k_batch_round<P, K, FORM_ALTERNATING>), dim3((unsigned)blocks),
                       dim3(64 * wpg), 0, st, rings, tile_prefix, k, active, items);
    return hipGetLastError();
}

hipError_t launch_batch_round(int precision, int K, const BatchRing *rings,
                              const int64_t *tile_prefix, int k, int active, int64_t items, int wpg,
                              hipStream_t st) {
    if (items <= 0) return hipSuccess;
    if (precision == HEAT_FP64 && K == 32)
        return launch_batch_round_t<F64, 32>(rings, tile_prefix, k, active, items, wpg, st);
    if (precision == HEAT_FP32 && K == 32)
        return launch_batch_round_t<F32, 32>(rings, tile_prefix, k, active, items, wpg, st);
    if (precision == HEAT_FP32C && K == 32)
        return launch_batch_round_t<F32C, 32>(rings, tile_prefix, k, active, items, wpg, st);
    return hipErrorInvalidValue;
}

hipError_t launch_batch(int precision, int K, const BatchPlanDev &plan, int grid, int wpg,
                        hipStream_t st) {
    if (precision == HEAT_FP64 && K == 32) return launch_batch_t<F64, 32>(plan, grid, wpg, st);
    if (precision == HEAT_FP32 && K == 32) return launch_batch_t<F32, 32>(plan, grid, wpg, st);
    if (precision == HEAT_FP32C && K == 32) return launch_batch_t<F32C, 32>(plan, grid, wpg, st);
    return hipErrorInvalidValue;
}

template <class P, int K>
static int occupancy_blocks(int wpg) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch<P, K>, 64 * wpg, 0) != hipSuccess)
        return 0;
    return nb;
}

int batch_grid_size(int precision, int K, int wpg, int *grid) {
    int dev = 0, cus = 0;
    HEAT_HIP(hipGetDevice(&dev));
    HEAT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int nb = 0;
    if (precision == HEAT_FP64 && K == 32) nb = occupancy_blocks<F64, 32>(wpg);
    else if (precision == HEAT_FP32 && K == 32) nb = occupancy_blocks<F32, 32>(wpg);
    else if (precision == HEAT_FP32C && K == 32) nb = occupancy_blocks<F32C, 32>(wpg);
    if (nb < 1) nb = 1;
    *grid = nb * cus;
    return HEAT_OK;
}

}  // namespace heat
