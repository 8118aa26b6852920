// heat_device.h -- device-side building blocks shared by the HIP kernels of
// the heat-stencil library (gfx950, wave64).  Included only by .hip files.
//
// The update is the explicit-Euler step of the paper's Eq. (heat:discrete) on
// a periodic ring (Section 2): new = c + r * ((l - 2c) + q) in binary64, and
// the binary32 / compensated binary32 forms documented in heat.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace heat {

// ------------------------------------------------------------ precisions

struct F64 {
    using T = double;
    static constexpr int VEC = 2;        // cells per 16-byte access
    static constexpr bool COMP = false;
    static constexpr bool LOW = false;
};
struct F32 {
    using T = float;
    static constexpr int VEC = 4;
    static constexpr bool COMP = false;
    static constexpr bool LOW = false;
};
struct F32C {
    using T = float;
    static constexpr int VEC = 4;
    static constexpr bool COMP = true;   // carries the compensation term e
    static constexpr bool LOW = true;    // and the coefficient's low part rl
};
// The compensated form for a coefficient that is a binary32 number (rl = 0):
// the same update without the low-part term, bit for bit (see comp_update).
struct F32C0 {
    using T = float;
    static constexpr int VEC = 4;
    static constexpr bool COMP = true;
    static constexpr bool LOW = false;
};

// 16-byte groups as the compiler's own vector types (what the nontemporal
// load/store builtins accept).
typedef double v2f64 __attribute__((ext_vector_type(2)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef unsigned int v4u32 __attribute__((ext_vector_type(4)));

template <class T> struct Vec16;
template <> struct Vec16<double> { using type = v2f64; };
template <> struct Vec16<float> { using type = v4f32; };

// Streaming accesses for data touched once per launch: the nontemporal hint
// keeps the sweep from evicting useful lines (measured +13 % on a plain copy).
template <class VT>
__device__ __forceinline__ VT load_stream(const VT *p) {
    return __builtin_nontemporal_load(p);
}
template <class VT>
__device__ __forceinline__ void store_stream(VT v, VT *p) {
    __builtin_nontemporal_store(v, p);
}

// ------------------------------------------------------ cross-lane moves
//
// DPP row/wave controls of the GFX9 family: wave_ror:1 rotates the wave right
// by one lane (lane i receives lane i-1, lane 0 receives lane 63), wave_rol:1
// rotates left (lane i receives lane i+1, lane 63 receives lane 0).  They are
// ordinary VALU moves: no LDS traffic, no waitcnt.
constexpr int DPP_WAVE_ROL1 = 0x134;
constexpr int DPP_WAVE_ROR1 = 0x13C;

__device__ __forceinline__ int dpp_from_prev_i(int x) {
    return __builtin_amdgcn_mov_dpp(x, DPP_WAVE_ROR1, 0xF, 0xF, false);
}
__device__ __forceinline__ int dpp_from_next_i(int x) {
    return __builtin_amdgcn_mov_dpp(x, DPP_WAVE_ROL1, 0xF, 0xF, false);
}
__device__ __forceinline__ float from_prev(float x) {
    return __int_as_float(dpp_from_prev_i(__float_as_int(x)));
}
__device__ __forceinline__ float from_next(float x) {
    return __int_as_float(dpp_from_next_i(__float_as_int(x)));
}
__device__ __forceinline__ double from_prev(double x) {
    int lo = dpp_from_prev_i(__double2loint(x));
    int hi = dpp_from_prev_i(__double2hiint(x));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double from_next(double x) {
    int lo = dpp_from_next_i(__double2loint(x));
    int hi = dpp_from_next_i(__double2hiint(x));
    return __hiloint2double(hi, lo);
}

// ------------------------------------------------------------ the update
//
// binary64: l - 2c is computed as fma(-2, c, l).  2c is exact, so the single
// rounding of the fused form equals the rounding of l - (2c): the result is
// bit-identical to evaluating ((l - 2c) + q) step by step.  The final
// c + r * lap is NOT fused (the library is built with -ffp-contract=off).
__device__ __forceinline__ double cell_update(double l, double c, double q, double r) {
    return c + r * (__builtin_fma(-2.0, c, l) + q);
}
// binary32: the second difference as the difference of the two one-sided
// differences, (q - c) - (c - l) (flux form).  Both are exact when neighbours
// are within a factor 2.  A sweep over consecutive cells forms each one-sided
// difference once: the right difference of cell j is the left difference of
// cell j + 1 (see the window steps below).
__device__ __forceinline__ float cell_update(float l, float c, float q, float r) {
    return c + r * ((q - c) - (c - l));
}
__device__ __forceinline__ float flux_update(float c, float dl, float dr, float r) {
    return c + r * (dr - dl);
}

// One step on K consecutive cells held by each lane (lane L holds cells
// [L*K, L*K + K) of the wave's window).  The end cells exchange neighbours
// with the adjacent lanes; lanes 0 and 63 receive wrapped values, which only
// corrupt the window's outer cells (the trapezoid shrinks by one per step).
template <int K, class T>
__device__ __forceinline__ void window_step(T (&v)[K], T r) {
    if constexpr (sizeof(T) == 4 && K >= 16) {
        // binary32: two interleaved sweeps, chain a over [0, M) and chain b
        // over [M, K), M = K/2 + 1, each carrying its last right difference
        // as the next cell's left difference.  The difference across the
        // chain boundary is formed once, before either chain writes.
        constexpr int M = K / 2 + 1;
        constexpr int NB = K - M;
        T dla = v[0] - from_prev(v[K - 1]);
        const T right = from_next(v[0]);
        T dlb = v[M] - v[M - 1];
        const T dra_last = dlb;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const T ca = v[j];
            const T dra = (j + 1 < M) ? v[j + 1] - ca : dra_last;
            v[j] = flux_update(ca, dla, dra, r);
            dla = dra;
            if (j < NB) {
                const T cb = v[M + j];
                const T qb = (M + j + 1 < K) ? v[M + j + 1] : right;
                const T drb = qb - cb;
                v[M + j] = flux_update(cb, dlb, drb, r);
                dlb = drb;
            }
        }
    } else if constexpr (sizeof(T) == 4) {
        T dl = v[0] - from_prev(v[K - 1]);
        const T right = from_next(v[0]);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const T c = v[j];
            const T dr = ((j + 1 < K) ? v[j + 1] : right) - c;
            v[j] = flux_update(c, dl, dr, r);
            dl = dr;
        }
    } else {
        T prev = from_prev(v[K - 1]);
        const T right = from_next(v[0]);
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const T c = v[j];
            const T q = (j + 1 < K) ? v[j + 1] : right;
            v[j] = cell_update(prev, c, q, r);
            prev = c;
        }
    }
}

// Ping-pong form of the same step: reads a[], writes b[].  Two of them in a
// row return the state to a[] with no register copies (the binary64 in-place
// form keeps the old left value past the write of each cell, which makes the
// compiler rotate the whole array through the registers once per step; the
// binary32 flux form carries a difference instead and needs no copies).
// Costs K more registers.
template <int K, class T>
__device__ __forceinline__ void window_step_pp(const T (&a)[K], T (&b)[K], T r) {
    const T left = from_prev(a[K - 1]);
    const T right = from_next(a[0]);
    if constexpr (sizeof(T) == 4) {
        T dl = a[0] - left;
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const T dr = ((j + 1 < K) ? a[j + 1] : right) - a[j];
            b[j] = flux_update(a[j], dl, dr, r);
            dl = dr;
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const T l = j == 0 ? left : a[j - 1];
            const T q = (j + 1 < K) ? a[j + 1] : right;
            b[j] = cell_update(l, a[j], q, r);
        }
    }
}

// Backward in-place step: the same update swept from the last cell to the
// first.  A binary64 forward step frees the register of cell j-1 when it
// writes cell j, a backward one frees cell j+1's: alternating them leaves
// every value where it started after two steps, so the loop needs no register
// copies and only K + 1 registers (the alternating register form).
template <int K, class T>
__device__ __forceinline__ void window_step_bwd(T (&v)[K], T r) {
    if constexpr (sizeof(T) == 4 && K >= 16) {
        // chain a: cells K-1 .. M (NB cells); chain b: cells M-1 .. 0 (M
        // cells), M = K/2 + 1, as in the forward sweep; each carries its last
        // left difference as the next cell's right difference
        constexpr int M = K / 2 + 1;
        constexpr int NB = K - M;
        const T left = from_prev(v[K - 1]);
        T dra = from_next(v[0]) - v[K - 1];
        T drb = v[M] - v[M - 1];
        const T dla_last = drb;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j < NB) {
                const int ia = K - 1 - j;
                const T ca = v[ia];
                const T dla = ia > M ? ca - v[ia - 1] : dla_last;
                v[ia] = flux_update(ca, dla, dra, r);
                dra = dla;
            }
            const int ib = M - 1 - j;
            const T cb = v[ib];
            const T dlb = cb - (ib > 0 ? v[ib - 1] : left);
            v[ib] = flux_update(cb, dlb, drb, r);
            drb = dlb;
        }
    } else if constexpr (sizeof(T) == 4) {
        const T left = from_prev(v[K - 1]);
        T dr = from_next(v[0]) - v[K - 1];
#pragma unroll
        for (int j = K - 1; j >= 0; --j) {
            const T c = v[j];
            const T dl = c - (j > 0 ? v[j - 1] : left);
            v[j] = flux_update(c, dl, dr, r);
            dr = dl;
        }
    } else {
        const T left = from_prev(v[K - 1]);
        T next = from_next(v[0]);
#pragma unroll
        for (int j = K - 1; j >= 0; --j) {
            const T c = v[j];
            const T l = j > 0 ? v[j - 1] : left;
            v[j] = cell_update(l, c, next, r);
            next = c;
        }
    }
}

// Compensated binary32 step of the pair (u, e).  The coefficient is the pair
// r + rl (r = fl32 of the binary64 coefficient, rl = fl32 of the rest).  The
// Laplacian of u + e is the difference of the pair's two one-sided fluxes,
// sr - sl, each flux (u[i+1] - u[i]) + (e[i+1] - e[i]) formed once per sweep
// (the right flux of cell j is the left flux of cell j + 1).  u takes the
// increment in one fused rounding, t = fma(r, L, c); the rounding error of t
// is c + r*L - t, which one more fma gives to within a rounding of its own
// (c - t is exact whenever t and c lie within a factor 2 of each other), and
// it gathers in e with the coefficient's low part times L:
//     t = fma(r, L, c);  res = fma(r, L, c - t);
//     e' = fma(rl, L, res) + e;  u' = t.
// LOW = false drops the fma with rl for a binary32 coefficient (rl = +0).
// The bits are the same: fma(+0, L, res) is res except that res = -0 may
// become +0, and then both give e' = e, because e is never -0 (it starts a
// round at +0, and a binary32 sum is -0 only when both terms are).
__device__ __forceinline__ float pair_flux(float uq, float uc, float eq, float ec) {
    return (uq - uc) + (eq - ec);
}
template <bool LOW>
__device__ __forceinline__ void comp_update(float &u, float &e, float sl, float sr, float r,
                                            float rl) {
    const float c = u;
    const float L = sr - sl;
    const float t = __builtin_fmaf(r, L, c);
    const float res = __builtin_fmaf(r, L, c - t);
    const float lo = LOW ? __builtin_fmaf(rl, L, res) : res;
    e = lo + e;
    u = t;
}

// The compensated sweeps below run, from 16 cells per lane on, as two
// interleaved chains over [0, M) and [M, K), M = K/2 + 1, like the binary32
// sweeps: each chain carries its own flux, the flux across the chain
// boundary is formed before either chain writes, and the two chains'
// independent operations sit next to each other in the instruction stream
// (the update of every cell is the same as in one sweep, so are the bits).
template <int K, bool LOW>
__device__ __forceinline__ void window_step_comp(float (&u)[K], float (&e)[K], float r,
                                                 float rl) {
    float sl = pair_flux(u[0], from_prev(u[K - 1]), e[0], from_prev(e[K - 1]));
    const float ru = from_next(u[0]);
    const float re = from_next(e[0]);
    if constexpr (K >= 16) {
        constexpr int M = K / 2 + 1;
        constexpr int NB = K - M;
        float slb = pair_flux(u[M], u[M - 1], e[M], e[M - 1]);
        const float sr_last = slb;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const float sr = (j + 1 < M) ? pair_flux(u[j + 1], u[j], e[j + 1], e[j]) : sr_last;
            comp_update<LOW>(u[j], e[j], sl, sr, r, rl);
            sl = sr;
            if (j < NB) {
                const int b = M + j;
                const float srb = pair_flux((b + 1 < K) ? u[b + 1] : ru, u[b],
                                            (b + 1 < K) ? e[b + 1] : re, e[b]);
                comp_update<LOW>(u[b], e[b], slb, srb, r, rl);
                slb = srb;
            }
        }
    } else {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            const float sr = pair_flux((j + 1 < K) ? u[j + 1] : ru, u[j],
                                       (j + 1 < K) ? e[j + 1] : re, e[j]);
            comp_update<LOW>(u[j], e[j], sl, sr, r, rl);
            sl = sr;
        }
    }
}

template <int K, bool LOW>
__device__ __forceinline__ void window_step_comp_bwd(float (&u)[K], float (&e)[K], float r,
                                                     float rl) {
    const float lu = from_prev(u[K - 1]);
    const float le = from_prev(e[K - 1]);
    float sr = pair_flux(from_next(u[0]), u[K - 1], from_next(e[0]), e[K - 1]);
    if constexpr (K >= 16) {
        // chain a: cells K-1 .. M (NB cells); chain b: cells M-1 .. 0 (M
        // cells); each carries its last left flux as the next cell's right
        // flux
        constexpr int M = K / 2 + 1;
        constexpr int NB = K - M;
        float srb = pair_flux(u[M], u[M - 1], e[M], e[M - 1]);
        const float sl_last = srb;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j < NB) {
                const int a = K - 1 - j;
                const float sl = a > M ? pair_flux(u[a], u[a - 1], e[a], e[a - 1]) : sl_last;
                comp_update<LOW>(u[a], e[a], sl, sr, r, rl);
                sr = sl;
            }
            const int b = M - 1 - j;
            const float slb = pair_flux(u[b], b > 0 ? u[b - 1] : lu, e[b], b > 0 ? e[b - 1] : le);
            comp_update<LOW>(u[b], e[b], slb, srb, r, rl);
            srb = slb;
        }
    } else {
#pragma unroll
        for (int j = K - 1; j >= 0; --j) {
            const float sl = pair_flux(u[j], j > 0 ? u[j - 1] : lu, e[j], j > 0 ? e[j - 1] : le);
            comp_update<LOW>(u[j], e[j], sl, sr, r, rl);
            sr = sl;
        }
    }
}

template <int K, bool LOW>
__device__ __forceinline__ void window_step_comp_pp(const float (&u)[K], const float (&e)[K],
                                                    float (&un)[K], float (&en)[K], float r,
                                                    float rl) {
    const float ru = from_next(u[0]);
    const float re = from_next(e[0]);
    float sl = pair_flux(u[0], from_prev(u[K - 1]), e[0], from_prev(e[K - 1]));
    // from 16 cells per lane, a second chain over [K/2, K) interleaved with
    // the first (the inputs are never overwritten, so no boundary care)
    constexpr int NA = K >= 16 ? K / 2 : K;
    float slb = 0.f;
    if constexpr (K >= 16) slb = pair_flux(u[NA], u[NA - 1], e[NA], e[NA - 1]);
#pragma unroll
    for (int j = 0; j < NA; ++j) {
        const float sr = pair_flux((j + 1 < K) ? u[j + 1] : ru, u[j], (j + 1 < K) ? e[j + 1] : re,
                                   e[j]);
        float a = u[j], b = e[j];
        comp_update<LOW>(a, b, sl, sr, r, rl);
        un[j] = a;
        en[j] = b;
        sl = sr;
        if constexpr (K >= 16) {
            const int i = NA + j;
            const float srb = pair_flux((i + 1 < K) ? u[i + 1] : ru, u[i],
                                        (i + 1 < K) ? e[i + 1] : re, e[i]);
            float c = u[i], d = e[i];
            comp_update<LOW>(c, d, slb, srb, r, rl);
            un[i] = c;
            en[i] = d;
            slb = srb;
        }
    }
}

// ------------------------------------------------------------ indexing

// Map a workgroup id so that consecutive logical ids stay on one XCD.
// Workgroups are dispatched round-robin over the 8 XCDs, so hardware id b
// runs on XCD b % 8; logical ids [x*q + min(x, rem), ...) go to XCD x.
__device__ __forceinline__ int64_t xcd_remap(int64_t b, int64_t grid) {
    const int64_t q = grid >> 3, rem = grid & 7;
    const int64_t x = b & 7, k = b >> 3;
    return x * q + (x < rem ? x : rem) + k;
}

__device__ __forceinline__ int64_t wrap_index(int64_t i, int64_t N) {
    int64_t m = i % N;
    return m < 0 ? m + N : m;
}

}  // namespace heat
