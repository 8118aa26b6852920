// resident.h -- the resident temporal-blocking kernel: one launch advances a
// ring through all nt steps with every tile's window kept in registers, and
// neighbouring tiles swap their edge cells through memory every T steps.
//
// This is the paper's segment algorithm (Section 2, last paragraph: each
// segment computes its cells and exchanges ghost cells with its two
// neighbours every step) with the segment a workgroup's tile and the ghost
// zone H cells deep, exchanged every T <= H steps: between exchanges a tile
// advances on its own, its windows' outer H cells going stale at one cell
// per step (the trapezoid of the round kernel, without reloading the window
// every round).
//
// Edge exchange.  After every T steps each tile writes the first H and the
// last H cells it owns into its slots of parity e & 1 in an exchange area (e =
// the number of exchanges so far, counting this one), every value as 64-bit
// words of 32 value bits beside the 32-bit tag epoch_base + e, and then
// reads its outer halo -- the H cells left of its output and the H cells
// right of it -- from its neighbours' slots, polling each word until its tag
// reads e.  A 64-bit store and load are single-copy atomic, so a word with
// the right tag holds that epoch's bits: no counter, fence or wait for the
// stores' completion stands between a tile's edges and its neighbours'
// reads.  The two parities alternate, so a slot is written again only two
// exchanges later, when every reader has moved on: a tile writes parity e & 1
// at exchange e + 2 only after it has read its neighbours' exchange e + 1,
// which they wrote after their reads of exchange e.  At the end every tile
// writes its output back into the ring.  Its neighbours loaded their
// windows from the ring before their first exchange; a run that makes no
// exchange (nt <= T) orders them by epoch counters instead: every tile
// raises its counter once loaded and waits for its neighbours' before it
// stores.
//
// Tags and counters are not cleared between launches: a launch counts on
// from epoch_base, which every tag and counter of the previous launch ended
// at or below.
//
// Every tile must be resident at once (the waits are across workgroups):
// the launcher refuses grids larger than the occupancy allows, and a wait
// longer than spin_limit polls sets status[0] (a pinned host word the host
// reads once the launch is done) and every wavefront leaves, so
// a grid that cannot be resident (another launch holding the CUs) ends with
// an error instead of hanging.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "heat_device.h"
#include "heat_internal.h"
#include "window.h"

namespace heat {

// Poll an epoch counter until it reaches `need`.  The counters only order
// a tile's final stores after its neighbours' window loads, whose values
// were in registers before the neighbours raised them: relaxed polls do.
__device__ __forceinline__ bool resident_wait(const ResidentArgs &a, int64_t tile,
                                              uint32_t need) {
    int64_t spins = 0;
    while (true) {
        const uint32_t v =
            __hip_atomic_load(a.flags + tile, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (v >= need) return true;
        if (++spins > a.spin_limit) {
            __hip_atomic_store(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            return false;
        }
        if ((spins & 63) == 0 &&
            __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0)
            return false;
        __builtin_amdgcn_s_sleep(2);
    }
}

// Wait for every tile whose output lies within H cells of tile t's on the
// ring (the tiles its halo reads, and the tiles whose halos read it).  Only
// the last tile can be shorter than W (>= H for every other), so the walk
// reaches two tiles away at most when that one is shorter than H.
__device__ __forceinline__ bool resident_wait_neighbours(const ResidentArgs &a, int64_t t,
                                                         uint32_t need) {
    if (a.tiles == 1) return true;
    const int64_t last_len = a.N - (a.tiles - 1) * a.W;
    int64_t acc = 0, q = t;
    for (int64_t g = 0; g + 1 < a.tiles && acc < a.H; ++g) {
        q = q == 0 ? a.tiles - 1 : q - 1;
        if (!resident_wait(a, q, need)) return false;
        acc += q == a.tiles - 1 ? last_len : a.W;
    }
    acc = 0;
    q = t;
    for (int64_t g = 0; g + 1 < a.tiles && acc < a.H; ++g) {
        q = q + 1 == a.tiles ? 0 : q + 1;
        if (!resident_wait(a, q, need)) return false;
        acc += q == a.tiles - 1 ? last_len : a.W;
    }
    return true;
}

// An edge cell in the exchange area: one 64-bit word per 32 bits of the
// value, its high half the epoch tag.
template <class T>
struct EdgeWord;
template <>
struct EdgeWord<double> {
    static constexpr int WORDS = 2;
    __device__ static void put(uint64_t *s, double x, uint32_t tag) {
        const uint64_t bits = (uint64_t)__double_as_longlong(x);
        const uint64_t t = (uint64_t)tag << 32;
        __hip_atomic_store(s, (bits & 0xffffffffu) | t, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(s + 1, (bits >> 32) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static bool get(const uint64_t *s, uint32_t tag, double &x) {
        const uint64_t lo = __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint64_t hi = __hip_atomic_load(s + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(lo >> 32) != tag || (uint32_t)(hi >> 32) != tag) return false;
        x = __longlong_as_double((long long)((lo & 0xffffffffu) | (hi << 32)));
        return true;
    }
};
template <>
struct EdgeWord<float> {
    static constexpr int WORDS = 1;
    __device__ static void put(uint64_t *s, float x, uint32_t tag) {
        __hip_atomic_store(s, (uint64_t)__float_as_uint(x) | (uint64_t)tag << 32,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static bool get(const uint64_t *s, uint32_t tag, float &x) {
        const uint64_t w = __hip_atomic_load(s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((uint32_t)(w >> 32) != tag) return false;
        x = __uint_as_float((uint32_t)w);
        return true;
    }
};

// Slot (cells from the start of a parity) that halo cell i of tile t is
// read from.  i < H: the cell H - i left of the tile's output, among the
// last H owned cells (side 1) of the tile it falls in; i >= H: the cell
// i - H right of its end, among the first H (side 0).  Tile q's slots are
// [q * 2H, q * 2H + H) for side 0 and the next H for side 1; side 1 slot j
// holds owned cell L - H + j of a tile of L cells.  Only the last tile can
// be shorter than H, so the walks visit two tiles at most.
__device__ __forceinline__ int64_t edge_source(const ResidentArgs &a, int64_t t, int i,
                                               int64_t last_len) {
    const int H = a.H;
    int64_t q = t;
    if (i < H) {
        int64_t d = H - i;
        for (int64_t g = 0; g < a.tiles; ++g) {
            q = q == 0 ? a.tiles - 1 : q - 1;
            const int64_t L = q == a.tiles - 1 ? last_len : a.W;
            if (d <= L) break;
            d -= L;
        }
        return q * 2 * H + H + (H - d);
    }
    int64_t d = i - H;
    for (int64_t g = 0; g < a.tiles; ++g) {
        q = q + 1 == a.tiles ? 0 : q + 1;
        const int64_t L = q == a.tiles - 1 ? last_len : a.W;
        if (d < L) break;
        d -= L;
    }
    return q * 2 * H + d;
}

// The LDS copy of a tile holds what passes through it: whole K-cell runs of
// the lanes that hold edge or halo cells (one predicate per lane, not per
// cell), in tile coordinates c = H + output position.  Runs that meet the
// first 2H coordinates lie in [0, 2H + K) (region A); runs that meet
// [wl, wl + 2H) lie above b_lo = (wl - K) rounded down to 4 cells (region B,
// 16-byte accesses), which follows region A when the two are disjoint; a
// short tile's copy is indexed by tile coordinate, which then stays under the
// same bound.  Cells of the copy: resident_tile_cells.
template <class P, int K>
__device__ __forceinline__ void tile_lds_put(typename P::T *dst, const typename P::T (&v)[K]) {
    using T = typename P::T;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = P::VEC;
    VT *p = reinterpret_cast<VT *>(dst);
#pragma unroll
    for (int j = 0; j < K / VEC; ++j) {
        VT x;
#pragma unroll
        for (int k = 0; k < VEC; ++k) x[k] = v[j * VEC + k];
        p[j] = x;
    }
}
template <class P, int K>
__device__ __forceinline__ void tile_lds_get(const typename P::T *src, typename P::T (&v)[K]) {
    using T = typename P::T;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = P::VEC;
    const VT *p = reinterpret_cast<const VT *>(src);
#pragma unroll
    for (int j = 0; j < K / VEC; ++j) {
        const VT x = p[j];
#pragma unroll
        for (int k = 0; k < VEC; ++k) v[j * VEC + k] = x[k];
    }
}
__host__ __device__ constexpr int64_t resident_tile_cells(int64_t W, int H, int K) {
    return W + 2 * H < 4 * (int64_t)H + 3 * K + 4 ? W + 2 * H : 4 * (int64_t)H + 3 * K + 4;
}
// Cells of a launch's LDS tile copy: the two edge regions, or the whole span
__host__ __device__ constexpr int64_t resident_lds_cells(int64_t W, int H, int K, bool edges) {
    return edges ? resident_tile_cells(W, H, K) : W + 2 * H;
}
// LDS index of tile coordinate c in a tile of wl output cells (of W at most)
__device__ __forceinline__ int tile_lds_at(int c, int64_t W, int H, int K, int wl, bool edges) {
    const int a_end = 2 * H + K, b_lo = (wl - K) & ~3;
    const bool split = edges && resident_tile_cells(W, H, K) < W + 2 * H && b_lo >= a_end;
    return split && c >= a_end ? c - b_lo + a_end : c;
}
__device__ __forceinline__ bool runs_meet(int a0, int a1, int b0, int b1) {
    return a0 < b1 && b0 < a1;
}

// LDS bytes of a resident workgroup: the waves' edge exchange (XD), then the
// tile copy (resident_tile_cells, 16-byte aligned).
template <class P>
constexpr int resident_lds_bytes(int K, int G, int XD, int tile_cells) {
    return (XD ? (exchange_lds_bytes<P>(K, G, XD) + 15) / 16 * 16 : 0) +
           tile_cells * (int)sizeof(typename P::T);
}

// One workgroup per tile; G = blockDim.x / 64 waves share it (XD = 4 or 2:
// LDS edge exchange every S = K/XD steps, as in window_tile; XD = 0: G = 1).
template <class P, int K, int FORM, int XD>
__global__ void __launch_bounds__(512) k_resident(ResidentArgs a) {
    using T = typename P::T;
    extern __shared__ __align__(16) unsigned char heat_xlds[];
    __shared__ int abort_flag;
    constexpr int WIN = 64 * K;
    constexpr bool XCHG = XD != 0;
    constexpr int S = exchange_depth<K, XD>();
    const int lane = threadIdx.x & 63;
    const int G = blockDim.x >> 6;
    const int w = threadIdx.x >> 6;
    const int64_t tile = xcd_remap(blockIdx.x, gridDim.x);
    if (tile >= a.tiles) return;
    const int H = a.H;
    const int64_t N = a.N, W = a.W, b = tile * W;
    const int64_t wlen = (N - b) < W ? (N - b) : W;
    const int64_t off = XCHG ? (int64_t)w * (WIN - 2 * S) : 0;
    const int64_t g0 = b - H + off;
    const int lo = (XCHG && w > 0) ? S : H;
    const int hi = (XCHG && w + 1 < G) ? WIN - S : WIN - H;
    const bool fast = a.vec_ok && b - H >= 0 && b + W + H <= N && wlen == W;
    const T r = (T)a.r;
    const T rl = P::LOW ? (T)(a.r - (double)r) : T(0);
    T *const ring0 = reinterpret_cast<T *>(a.u);
    if (threadIdx.x == 0) abort_flag = 0;

    T v[K], e[K];
    window_load<P, K>(ring0, N, g0, fast, lane, v);
    if constexpr (P::COMP) {
#pragma unroll
        for (int j = 0; j < K; ++j) e[j] = T(0);
    }
    if (a.part_in) {
        const double s = tile_sum<K>(v, lane, lo, hi, off, H, wlen);
        if (lane == 0) a.part_in[tile * G + w] = s;
    }
    T *xu = reinterpret_cast<T *>(heat_xlds);
    T *xe = xu + 2 * G * 2 * S;
    T *tl = reinterpret_cast<T *>(
        heat_xlds + (XCHG ? (exchange_lds_bytes<P>(K, G, XD) + 15) / 16 * 16 : 0));
    const int c0 = (int)off + lane * K;   // tile coordinate of this lane's first cell
    const int wl = (int)wlen;
    // lanes holding edge cells (tile coordinates [H, 2H), [wl, wl + H)) or
    // halo cells ([0, H), [wl + H, wl + 2H))
    const bool io_lane = runs_meet(c0, c0 + K, 0, 2 * H) || runs_meet(c0, c0 + K, wl, wl + 2 * H);
    const bool halo_lane =
        runs_meet(c0, c0 + K, 0, H) || runs_meet(c0, c0 + K, wl + H, wl + 2 * H);
    const int nthr = blockDim.x;
    const bool edges = a.lds_edges != 0;
    constexpr int WORDS = EdgeWord<T>::WORDS;
    const int64_t last_len = N - (a.tiles - 1) * W;
    int xbuf = 0;
    uint32_t epoch = 0;
    int64_t done = 0;
    while (done < a.nt) {
        const int steps = (int)((a.nt - done) < a.T ? (a.nt - done) : a.T);
        if constexpr (XCHG) {
            // chunks of S steps; the waves swap edges after every chunk but
            // the run's last (here also after a round's last, since the
            // windows carry on into the next round)
            int s = 0;
            for (; steps - s > S; s += S) {
                advance<P, K, FORM>(v, e, S, r, rl);
                exchange_part<K, XD>(v, xu, xbuf, G, w, lane);
                if constexpr (P::COMP) exchange_part<K, XD>(e, xe, xbuf, G, w, lane);
                __syncthreads();
                exchange_take<K, XD>(v, xu, xbuf, G, w, lane);
                if constexpr (P::COMP) exchange_take<K, XD>(e, xe, xbuf, G, w, lane);
                xbuf ^= 1;
            }
            advance<P, K, FORM>(v, e, steps - s, r, rl);
        } else {
            advance<P, K, FORM>(v, e, steps, r, rl);
        }
        done += steps;
        if constexpr (P::COMP) {
            // the round ends: u := fl32(u + e), e := 0, as at every round end
#pragma unroll
            for (int j = 0; j < K; ++j) {
                v[j] = v[j] + e[j];
                e[j] = T(0);
            }
        }
        if (done >= a.nt) break;
        ++epoch;
        if constexpr (XCHG) {
            // the waves' overlaps, stale by the last chunk's steps
            exchange_part<K, XD>(v, xu, xbuf, G, w, lane);
            __syncthreads();
            exchange_take<K, XD>(v, xu, xbuf, G, w, lane);
            xbuf ^= 1;
        }
        // publish the first and the last H owned cells through the tile copy,
        // then read the outer halo (output positions [-H, 0) and [wl, wl + H),
        // tile coordinates [0, H) and [wl + H, wl + 2H)) from the neighbours'
        // slots of this parity
        const uint32_t tag = a.epoch_base + epoch;
        uint64_t *const area = a.xa + (int64_t)(epoch & 1) * a.tiles * 2 * H * WORDS;
        if (io_lane) tile_lds_put<P, K>(tl + tile_lds_at(c0, W, H, K, wl, edges), v);
        __syncthreads();
        for (int i = threadIdx.x; i < 2 * H; i += nthr) {
            const int p = i < H ? i : wl - 2 * H + i;
            if (p >= 0 && p < wl)
                EdgeWord<T>::put(area + (tile * 2 * H + i) * WORDS,
                                 tl[tile_lds_at(H + p, W, H, K, wl, edges)], tag);
        }
        for (int i = threadIdx.x; i < 2 * H; i += nthr) {
            const uint64_t *src = area + edge_source(a, tile, i, last_len) * WORDS;
            T x = T(0);
            int64_t spins = 0;
            while (!EdgeWord<T>::get(src, tag, x)) {
                if (++spins > a.spin_limit) {
                    __hip_atomic_store(a.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
                    abort_flag = 1;
                    break;
                }
                if ((spins & 63) == 0 &&
                    __hip_atomic_load(a.status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0) {
                    abort_flag = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            tl[tile_lds_at(i < H ? i : wl + i, W, H, K, wl, edges)] = x;
        }
        __syncthreads();
        if (abort_flag) return;
        if (halo_lane) tile_lds_get<P, K>(tl + tile_lds_at(c0, W, H, K, wl, edges), v);
    }
    if (a.part_out) {
        const double s = tile_sum<K>(v, lane, lo, hi, off, H, wlen);
        if (lane == 0) a.part_out[tile * G + w] = s;
    }
    if (epoch == 0) {
        // no exchange: a neighbour may still be loading its window from the
        // cells this tile is about to store
        if (threadIdx.x == 0) {
            __hip_atomic_store(a.flags + tile, a.epoch_base + 1, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            if (!resident_wait_neighbours(a, tile, a.epoch_base + 1)) abort_flag = 1;
        }
        __syncthreads();
        if (abort_flag) return;
    }
    window_store<P, K>(ring0, g0, lo, hi, off, H, wlen, fast, lane, v);
}

template <class P, int K, int FORM, int XD>
constexpr bool resident_fits() {
    return !(K == 64 && FORM == FORM_PINGPONG && (sizeof(typename P::T) == 8 || P::COMP)) &&
           !(XD && K / XD < 4);
}

// Workgroups of this instantiation one CU can hold at once.
template <class P, int K, int FORM, int XD>
int resident_blocks_per_cu(int G, int tile_cells) {
    if constexpr (!resident_fits<P, K, FORM, XD>()) {
        return 0;
    } else {
        int n = 0;
        const size_t lds = (size_t)resident_lds_bytes<P>(K, G, XD, tile_cells);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_resident<P, K, FORM, XD>, 64 * G,
                                                         lds) != hipSuccess)
            return 0;
        return n;
    }
}

template <class P, int K, int FORM, int XD>
hipError_t launch_resident_t(const ResidentArgs &a, int G, hipStream_t st) {
    if constexpr (!resident_fits<P, K, FORM, XD>()) {
        return hipErrorInvalidValue;
    } else {
        const unsigned lds = (unsigned)resident_lds_bytes<P>(
            K, G, XD, (int)resident_lds_cells(a.W, a.H, K, a.lds_edges != 0));
        hipLaunchKernelGGL((k_resident<P, K, FORM, XD>), dim3((unsigned)a.tiles), dim3(64 * G),
                           lds, st, a);
        return hipGetLastError();
    }
}

// Dispatch on (K, form) over the forms in FORMS (bit f set: form f built);
// with `blocks` set, return the occupancy in *blocks instead of launching.
template <class P, int XD, int FORMS>
hipError_t resident_dispatch(const ResidentArgs &a, int K, int form, int G, hipStream_t st,
                             int *blocks) {
#define HEAT_RESIDENT_CASE(KK, FF)                                                   \
    if constexpr ((FORMS >> FF) & 1) {                                               \
        if (K == KK && form == FF) {                                                 \
            if (blocks) {                                                            \
                *blocks = resident_blocks_per_cu<P, KK, FF, XD>(                     \
                    G, (int)resident_lds_cells(a.W, a.H, KK, a.lds_edges != 0));     \
                return hipSuccess;                                                   \
            }                                                                        \
            return launch_resident_t<P, KK, FF, XD>(a, G, st);                       \
        }                                                                            \
    }
    HEAT_RESIDENT_CASE(8, FORM_INPLACE)
    HEAT_RESIDENT_CASE(8, FORM_PINGPONG)
    HEAT_RESIDENT_CASE(8, FORM_ALTERNATING)
    HEAT_RESIDENT_CASE(16, FORM_INPLACE)
    HEAT_RESIDENT_CASE(16, FORM_PINGPONG)
    HEAT_RESIDENT_CASE(16, FORM_ALTERNATING)
    HEAT_RESIDENT_CASE(32, FORM_INPLACE)
    HEAT_RESIDENT_CASE(32, FORM_PINGPONG)
    HEAT_RESIDENT_CASE(32, FORM_ALTERNATING)
    HEAT_RESIDENT_CASE(64, FORM_INPLACE)
    HEAT_RESIDENT_CASE(64, FORM_PINGPONG)
    HEAT_RESIDENT_CASE(64, FORM_ALTERNATING)
#undef HEAT_RESIDENT_CASE
    return hipErrorInvalidValue;
}

template <class P, int FORMS>
hipError_t resident_any_xd(const ResidentArgs &a, int K, int form, int G, int xd, hipStream_t st,
                           int *blocks) {
    switch (xd) {
        case 0: return resident_dispatch<P, 0, FORMS>(a, K, form, G, st, blocks);
        case 4: return resident_dispatch<P, 4, FORMS>(a, K, form, G, st, blocks);
        case 2: return resident_dispatch<P, 2, FORMS>(a, K, form, G, st, blocks);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace heat
