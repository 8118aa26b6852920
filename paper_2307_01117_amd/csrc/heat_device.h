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
};
struct F32 {
    using T = float;
    static constexpr int VEC = 4;
    static constexpr bool COMP = false;
};
struct F32C {
    using T = float;
    static constexpr int VEC = 4;
    static constexpr bool COMP = true;   // carries the compensation term e
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
// binary32: both differences are exact when neighbours are within a factor 2.
__device__ __forceinline__ float cell_update(float l, float c, float q, float r) {
    return c + r * ((l - c) + (q - c));
}

// One step on K consecutive cells held by each lane (lane L holds cells
// [L*K, L*K + K) of the wave's window).  The end cells exchange neighbours
// with the adjacent lanes; lanes 0 and 63 receive wrapped values, which only
// corrupt the window's outer cells (the trapezoid shrinks by one per step).
template <int K, class T>
__device__ __forceinline__ void window_step(T (&v)[K], T r) {
    if constexpr (sizeof(T) == 4 && K >= 16) {
        // binary32: two interleaved sweeps, chain a over [0, M) and chain b
        // over [M, K), M = K/2 + 1.  Same per-cell arithmetic (bit-identical);
        // measured on MI355X 2 % faster for the in-place form, whose issue
        // rate is set by how often two VALU instructions pair in a cycle.
        constexpr int M = K / 2 + 1;
        constexpr int NB = K - M;
        T pa = from_prev(v[K - 1]);
        const T right = from_next(v[0]);
        T pb = v[M - 1];
        const T ra = v[M];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const T ca = v[j];
            const T qa = (j + 1 < M) ? v[j + 1] : ra;
            v[j] = cell_update(pa, ca, qa, r);
            pa = ca;
            if (j < NB) {
                const T cb = v[M + j];
                const T qb = (M + j + 1 < K) ? v[M + j + 1] : right;
                v[M + j] = cell_update(pb, cb, qb, r);
                pb = cb;
            }
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
// row return the state to a[] with no register copies (the in-place form
// makes the compiler rotate the whole array through the registers once per
// step).  Costs K more registers.
template <int K, class T>
__device__ __forceinline__ void window_step_pp(const T (&a)[K], T (&b)[K], T r) {
    const T left = from_prev(a[K - 1]);
    const T right = from_next(a[0]);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const T l = j == 0 ? left : a[j - 1];
        const T q = (j + 1 < K) ? a[j + 1] : right;
        b[j] = cell_update(l, a[j], q, r);
    }
}

// Backward in-place step: the same update swept from the last cell to the
// first.  A forward step frees the register of cell j-1 when it writes cell
// j, a backward one frees cell j+1's: alternating them leaves every value
// where it started after two steps, so the loop needs no register copies and
// only K + 1 registers (the alternating register form).
template <int K, class T>
__device__ __forceinline__ void window_step_bwd(T (&v)[K], T r) {
    if constexpr (sizeof(T) == 4 && K >= 16) {
        // chain a: cells K-1 .. M (NB cells); chain b: cells M-1 .. 0 (M
        // cells), M = K/2 + 1, as in the forward sweep
        constexpr int M = K / 2 + 1;
        constexpr int NB = K - M;
        const T left = from_prev(v[K - 1]);
        T na = from_next(v[0]);
        T nb = v[M];
        const T lb = v[M - 1];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j < NB) {
                const int ia = K - 1 - j;
                const T ca = v[ia];
                const T la = ia > M ? v[ia - 1] : lb;
                v[ia] = cell_update(la, ca, na, r);
                na = ca;
            }
            const int ib = M - 1 - j;
            const T cb = v[ib];
            const T l2 = ib > 0 ? v[ib - 1] : left;
            v[ib] = cell_update(l2, cb, nb, r);
            nb = cb;
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

// Compensated binary32 step of the pair (u, e): the Laplacian of u + e is
// formed from the exact-ish differences of both parts, then added to u with
// Fast2Sum so that the rounding error of the addition is kept in e.
template <int K>
__device__ __forceinline__ void window_step_comp(float (&u)[K], float (&e)[K], float r) {
    float pu = from_prev(u[K - 1]);
    float pe = from_prev(e[K - 1]);
    const float ru = from_next(u[0]);
    const float re = from_next(e[0]);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float c = u[j], ec = e[j];
        const float q = (j + 1 < K) ? u[j + 1] : ru;
        const float eq = (j + 1 < K) ? e[j + 1] : re;
        const float d = r * (((pu - c) + (q - c)) + ((pe - ec) + (eq - ec)));
        const float y = d + ec;
        const float t = c + y;
        e[j] = y - (t - c);
        u[j] = t;
        pu = c;
        pe = ec;
    }
}

template <int K>
__device__ __forceinline__ void window_step_comp_bwd(float (&u)[K], float (&e)[K], float r) {
    const float lu = from_prev(u[K - 1]);
    const float le = from_prev(e[K - 1]);
    float nu = from_next(u[0]);
    float ne = from_next(e[0]);
#pragma unroll
    for (int j = K - 1; j >= 0; --j) {
        const float c = u[j], ec = e[j];
        const float l = j > 0 ? u[j - 1] : lu;
        const float el = j > 0 ? e[j - 1] : le;
        const float d = r * (((l - c) + (nu - c)) + ((el - ec) + (ne - ec)));
        const float y = d + ec;
        const float t = c + y;
        e[j] = y - (t - c);
        u[j] = t;
        nu = c;
        ne = ec;
    }
}

template <int K>
__device__ __forceinline__ void window_step_comp_pp(const float (&u)[K], const float (&e)[K],
                                                    float (&un)[K], float (&en)[K], float r) {
    const float lu = from_prev(u[K - 1]);
    const float le = from_prev(e[K - 1]);
    const float ru = from_next(u[0]);
    const float re = from_next(e[0]);
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const float c = u[j], ec = e[j];
        const float l = j == 0 ? lu : u[j - 1];
        const float el = j == 0 ? le : e[j - 1];
        const float q = (j + 1 < K) ? u[j + 1] : ru;
        const float eq = (j + 1 < K) ? e[j + 1] : re;
        const float d = r * (((l - c) + (q - c)) + ((el - ec) + (eq - ec)));
        const float y = d + ec;
        const float t = c + y;
        en[j] = y - (t - c);
        un[j] = t;
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
