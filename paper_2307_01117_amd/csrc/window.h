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

}  // namespace heat
