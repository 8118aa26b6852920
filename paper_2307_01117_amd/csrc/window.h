// window.h -- the temporal-blocking window of one wavefront: load, T steps in
// registers, store, with the optional fused per-tile sums.  Shared by the
// plain round kernel (kernels.hip) and the batch kernels (batch_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "heat_device.h"

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

// Store the cells this wave owns: window positions [lo, hi) whose tile
// position off + pos lies in the output [H, H + wlen).  Fast path (whole
// window inside the ring, full tile): lo, hi are multiples of 4, so a 16-byte
// group never straddles the ownership boundaries.
template <class P, int K>
__device__ __forceinline__ void window_store(typename P::T *__restrict__ dst, int64_t g0, int lo,
                                             int hi, int64_t off, int H, int64_t wlen, bool fast,
                                             int lane, const typename P::T (&v)[K]) {
    using T = typename P::T;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = P::VEC;
    if (fast) {
        VT *p = reinterpret_cast<VT *>(dst + g0 + (int64_t)lane * K);
#pragma unroll
        for (int j = 0; j < K / VEC; ++j) {
            const int pos = lane * K + j * VEC;
            if (pos >= lo && pos < hi) {
                VT x;
#pragma unroll
                for (int k = 0; k < VEC; ++k) x[k] = v[j * VEC + k];
                p[j] = x;
            }
        }
    } else {
        // g0 = b - H + off, so ring cell of window position pos is
        // b + (off + pos - H), inside [b, b + wlen) when owned and valid
        const int64_t b = g0 + H - off;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const int pos = lane * K + j;
            const int64_t pg = off + pos;
            if (pos >= lo && pos < hi && pg >= H && pg < H + wlen) dst[b + (pg - H)] = v[j];
        }
    }
}

// binary64 sum of the cells this wave owns (window positions [lo, hi)) that
// lie in the tile's output, lane by lane in index order, then a fixed
// butterfly over the wave; lane 0's value is returned.
template <int K, class T>
__device__ __forceinline__ double tile_sum(const T (&v)[K], int lane, int lo, int hi, int64_t off,
                                           int H, int64_t wlen) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const int pos = lane * K + j;
        const int64_t pg = off + pos;
        if (pos >= lo && pos < hi && pg >= H && pg < H + wlen) s += (double)v[j];
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    return s;
}

// Register forms of the T-step loop.
enum RegForm { FORM_INPLACE = 1, FORM_PINGPONG = 2, FORM_ALTERNATING = 3 };

// n steps of the window in the chosen register form (the state is back in v
// and e afterwards).
template <class P, int K, int FORM>
__device__ __forceinline__ void advance(typename P::T (&v)[K], typename P::T (&e)[K], int n,
                                        typename P::T r, typename P::T rl) {
    using T = typename P::T;
    if constexpr (P::COMP) {
        if constexpr (FORM == FORM_PINGPONG) {
            T v2[K], e2[K];
            int s = 0;
            for (; s + 2 <= n; s += 2) {
                window_step_comp_pp<K, P::LOW>(v, e, v2, e2, r, rl);
                window_step_comp_pp<K, P::LOW>(v2, e2, v, e, r, rl);
            }
            if (s < n) window_step_comp<K, P::LOW>(v, e, r, rl);
        } else if constexpr (FORM == FORM_ALTERNATING) {
            int s = 0;
            for (; s + 2 <= n; s += 2) {
                window_step_comp<K, P::LOW>(v, e, r, rl);
                window_step_comp_bwd<K, P::LOW>(v, e, r, rl);
            }
            if (s < n) window_step_comp<K, P::LOW>(v, e, r, rl);
        } else {
            for (int s = 0; s < n; ++s) window_step_comp<K, P::LOW>(v, e, r, rl);
        }
    } else {
        if constexpr (FORM == FORM_PINGPONG) {
            T v2[K];
            int s = 0;
            for (; s + 2 <= n; s += 2) {
                window_step_pp<K>(v, v2, r);
                window_step_pp<K>(v2, v, r);
            }
            if (s < n) window_step<K>(v, r);
        } else if constexpr (FORM == FORM_ALTERNATING) {
            int s = 0;
            for (; s + 2 <= n; s += 2) {
                window_step<K>(v, r);
                window_step_bwd<K>(v, r);
            }
            if (s < n) window_step<K>(v, r);
        } else {
            for (int s = 0; s < n; ++s) window_step<K>(v, r);
        }
    }
}

// ----------------------------------------------------- cooperating waves
//
// The G waves of a workgroup can share one tile: wave w's window starts
// w*(64K - 2S) cells right of wave 0's, so neighbouring windows overlap by 2S
// cells, with the exchange depth S = K/XD (XD = 4 or 2).  Inside the group,
// each wave's edge cells go stale at one cell per step from each side; every
// S steps the waves swap S edge cells through LDS, which makes every window
// exact again except at the group's two outer edges (the halo H, as for a
// lone wave).  This is the ghost-zone exchange between segments, one level
// down: each wave is a segment, and the exchange is deep (S cells every S
// steps) instead of one cell every step.  Only the tile's outer halo is
// recomputed redundantly, plus 2S cells per pair of neighbouring waves: the
// deeper exchange (XD = 2) halves the number of exchanges for twice that
// overlap.
//
// LDS layout (per workgroup): two buffers (alternated, so one barrier per
// exchange suffices) x G waves x 2 edges x S cells, for u and, in the
// compensated form, e.  Edge 0 of wave w holds its cells [S, 2S) (what wave
// w-1 needs at its right end), edge 1 its cells [64K - 2S, 64K - S) (what
// wave w+1 needs at its left end); both live in one lane (S <= K/2).
template <int K, int XD>
constexpr int exchange_depth() { return XD ? K / XD : 0; }
static_assert(exchange_depth<16, 4>() % 2 == 0 && exchange_depth<8, 2>() % 2 == 0,
              "exchange chunks must be whole step pairs");

template <class P>
constexpr int exchange_lds_bytes(int K, int G, int XD) {
    return 2 * G * 2 * (K / XD) * (int)sizeof(typename P::T) * (P::COMP ? 2 : 1);
}

template <int K, int XD, class T>
__device__ __forceinline__ void exchange_part(T (&v)[K], T *x, int buf, int G, int w, int lane) {
    constexpr int S = exchange_depth<K, XD>();
    T *mine = x + (size_t)(buf * G + w) * 2 * S;
    if (lane == 0 && w > 0) {
#pragma unroll
        for (int j = 0; j < S; ++j) mine[j] = v[S + j];
    }
    if (lane == 63 && w + 1 < G) {
#pragma unroll
        for (int j = 0; j < S; ++j) mine[S + j] = v[K - 2 * S + j];
    }
}

// Lane 0 and lane 63 read their neighbours' edges straight into the state
// registers (the loads run with only that lane enabled).
template <int K, int XD, class T>
__device__ __forceinline__ void exchange_take(T (&v)[K], const T *x, int buf, int G, int w,
                                              int lane) {
    constexpr int S = exchange_depth<K, XD>();
    if (lane == 0 && w > 0) {
        const T *src = x + (size_t)(buf * G + w - 1) * 2 * S + S;   // left wave's edge 1
#pragma unroll
        for (int j = 0; j < S; ++j) v[j] = src[j];
    }
    if (lane == 63 && w + 1 < G) {
        const T *src = x + (size_t)(buf * G + w + 1) * 2 * S;       // right wave's edge 0
#pragma unroll
        for (int j = 0; j < S; ++j) v[K - S + j] = src[j];
    }
}

// Process one tile: output cells [b, b + min(W, N - b)).  Lone wave
// (XD = 0): G = 1, w = 0, W = 64K - 2H.  Cooperating waves (XD = 4 or 2):
// wave w of G, xlds = the workgroup's exchange area (see above),
// W = G*64K - (G-1)*2S - 2H, S = K/XD.  part_in / part_out (may be NULL): per-wave
// binary64 sums of the state before and after the round, written at index
// `part` -- the conservation checksum fused into the first and last rounds
// (no extra pass over HBM).
template <class P, int K, int FORM, int XD = 0>
__device__ __forceinline__ void window_tile(const typename P::T *__restrict__ src,
                                            typename P::T *__restrict__ dst, int64_t N, int H,
                                            int steps, double r64, int64_t b, int64_t W,
                                            bool vec_ok, int lane, double *part_in = nullptr,
                                            double *part_out = nullptr, int64_t part = 0,
                                            int G = 1, int w = 0,
                                            typename P::T *xlds = nullptr) {
    using T = typename P::T;
    constexpr int WIN = 64 * K;
    constexpr bool XCHG = XD != 0;
    constexpr int S = exchange_depth<K, XD>();
    // the coefficient in the storage type; the compensated form also carries
    // the rest of the binary64 coefficient, rl = fl32(r64 - r) (unused when
    // P::LOW is false: the launcher takes that form only when rl is +0)
    const T r = (T)r64;
    const T rl = P::LOW ? (T)(r64 - (double)r) : T(0);
    // this wave's window in tile coordinates: [off, off + WIN)
    const int64_t off = XCHG ? (int64_t)w * (WIN - 2 * S) : 0;
    const int64_t g0 = b - H + off;
    const int64_t wlen = (N - b) < W ? (N - b) : W;
    // cells this wave owns: its window minus the halo (outer edges) or minus
    // S (edges shared with a neighbour wave)
    const int lo = (XCHG && w > 0) ? S : H;
    const int hi = (XCHG && w + 1 < G) ? WIN - S : WIN - H;
    // whole tile span [b - H, b + W + H) inside the ring, full tile
    const bool fast = vec_ok && b - H >= 0 && b + W + H <= N && wlen == W;
    T v[K];
    window_load<P, K>(src, N, g0, fast, lane, v);
    if (part_in) {
        const double s = tile_sum<K>(v, lane, lo, hi, off, H, wlen);
        if (lane == 0) part_in[part] = s;
    }
    if constexpr (!XCHG) {
        // The lone wave's loops are written out here rather than through
        // advance(): with the binary64 in-place form the compiler's register
        // assignment depends on this shape (rotating K registers per step
        // instead of copying the array), and so does the occupancy.
        if constexpr (P::COMP) {
            T e[K];
#pragma unroll
            for (int j = 0; j < K; ++j) e[j] = T(0);
            if constexpr (FORM == FORM_PINGPONG) {
                T v2[K], e2[K];
                int s = 0;
                for (; s + 2 <= steps; s += 2) {
                    window_step_comp_pp<K, P::LOW>(v, e, v2, e2, r, rl);
                    window_step_comp_pp<K, P::LOW>(v2, e2, v, e, r, rl);
                }
                if (s < steps) window_step_comp<K, P::LOW>(v, e, r, rl);
            } else if constexpr (FORM == FORM_ALTERNATING) {
                int s = 0;
                for (; s + 2 <= steps; s += 2) {
                    window_step_comp<K, P::LOW>(v, e, r, rl);
                    window_step_comp_bwd<K, P::LOW>(v, e, r, rl);
                }
                if (s < steps) window_step_comp<K, P::LOW>(v, e, r, rl);
            } else {
                for (int s = 0; s < steps; ++s) window_step_comp<K, P::LOW>(v, e, r, rl);
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
    } else {
        // chunks of S steps (S even), each followed by an exchange, then the
        // last chunk of 1..S steps: an odd step count only ever ends the
        // round and there is a single final call, so the loop keeps one
        // register assignment
        T e[K];
        if constexpr (P::COMP) {
#pragma unroll
            for (int j = 0; j < K; ++j) e[j] = T(0);
        }
        T *xu = xlds;
        T *xe = xlds + 2 * G * 2 * S;
        int s = 0, buf = 0;
        for (; steps - s > S; s += S) {
            advance<P, K, FORM>(v, e, S, r, rl);
            exchange_part<K, XD>(v, xu, buf, G, w, lane);
            if constexpr (P::COMP) exchange_part<K, XD>(e, xe, buf, G, w, lane);
            __syncthreads();
            exchange_take<K, XD>(v, xu, buf, G, w, lane);
            if constexpr (P::COMP) exchange_take<K, XD>(e, xe, buf, G, w, lane);
            buf ^= 1;
        }
        advance<P, K, FORM>(v, e, steps - s, r, rl);
        if constexpr (P::COMP) {
#pragma unroll
            for (int j = 0; j < K; ++j) v[j] = v[j] + e[j];   // fold: u := fl32(u + e)
        }
    }
    if (part_out) {
        const double s = tile_sum<K>(v, lane, lo, hi, off, H, wlen);
        if (lane == 0) part_out[part] = s;
    }
    window_store<P, K>(dst, g0, lo, hi, off, H, wlen, fast, lane, v);
}

}  // namespace heat
