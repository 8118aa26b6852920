// round.h -- the round kernel of the temporal-blocked stencil and its
// launcher, as templates: kernels.hip instantiates the lone-wave variant,
// kernels_xchg.hip the variant whose waves share a tile through LDS (kept
// apart so that the two compile in parallel and each kernel holds one loop
// structure, which keeps its register count at what the window needs) for
// binary64.  kernels_f32.hip and kernels_f32c.hip instantiate both variants
// of the plain and the compensated binary32 forms, which are built with
// their own instruction scheduler; no other file may instantiate them (see
// launch_window_any).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "heat_device.h"
#include "heat_internal.h"
#include "window.h"

namespace heat {

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// One round over all tiles, mapped XCD-contiguously.  XD = 0: one wavefront
// per tile (part = tile).  XD = 4 or 2: the workgroup's waves share one tile
// and swap K/XD edge cells through the launch's dynamic LDS area.
template <class P, int K, int FORM, int XD>
__global__ void __launch_bounds__(512)
k_window(const typename P::T *__restrict__ src, typename P::T *__restrict__ dst, int64_t N,
         int32_t H, int32_t steps, double r, int64_t tiles, int64_t W, int32_t vec_ok,
         double *part_in, double *part_out) {
    extern __shared__ __align__(16) unsigned char heat_xlds[];
    const int lane = threadIdx.x & 63;
    const int wpg = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int64_t blk = xcd_remap(blockIdx.x, gridDim.x);
    const int64_t part = blk * wpg + wave;
    const int64_t tile = XD ? blk : part;
    if (tile >= tiles) return;
    window_tile<P, K, FORM, XD>(src, dst, N, H, steps, r, tile * W, W,
                                  vec_ok != 0, lane, part_in, part_out, part, wpg, wave,
                                  reinterpret_cast<typename P::T *>(heat_xlds));
}

// Shapes that cannot hold their state in registers (they would spill), and
// shapes whose exchange depth K/XD would be below 4 cells.
template <class P, int K, int FORM, int XD>
constexpr bool shape_fits() {
    return !(K == 64 && FORM == FORM_PINGPONG && (sizeof(typename P::T) == 8 || P::COMP)) &&
           !(XD && K / XD < 4);
}

template <class P, int K, int FORM, int XD>
hipError_t launch_window_t(const WindowLaunch &a, hipStream_t st) {
    using T = typename P::T;
    if constexpr (!shape_fits<P, K, FORM, XD>()) {
        return hipErrorInvalidValue;
    } else {
        const int64_t W = window_tile_cells(K, a.H, a.wpg, XD);
        const int64_t tiles = (a.N + W - 1) / W;
        const int64_t blocks = XD ? tiles : (tiles + a.wpg - 1) / a.wpg;
        const int vec_ok = aligned16(a.src) && aligned16(a.dst);
        const unsigned lds = XD ? (unsigned)exchange_lds_bytes<P>(K, a.wpg, XD) : 0u;
        hipLaunchKernelGGL((k_window<P, K, FORM, XD>), dim3((unsigned)blocks), dim3(64 * a.wpg),
                           lds, st, reinterpret_cast<const T *>(a.src),
                           reinterpret_cast<T *>(a.dst), a.N, a.H, a.steps, a.r, tiles, W, vec_ok,
                           a.part_in, a.part_out);
        return hipGetLastError();
    }
}

template <class P, int FORM, int XD>
hipError_t launch_window_k(const WindowLaunch &a, hipStream_t st) {
    switch (a.K) {
        case 8: return launch_window_t<P, 8, FORM, XD>(a, st);
        case 16: return launch_window_t<P, 16, FORM, XD>(a, st);
        case 32: return launch_window_t<P, 32, FORM, XD>(a, st);
        case 64: return launch_window_t<P, 64, FORM, XD>(a, st);
        default: return hipErrorInvalidValue;
    }
}

template <class P, int XD>
hipError_t launch_window_f(const WindowLaunch &a, hipStream_t st) {
    switch (a.form) {
        case FORM_INPLACE: return launch_window_k<P, FORM_INPLACE, XD>(a, st);
        case FORM_PINGPONG: return launch_window_k<P, FORM_PINGPONG, XD>(a, st);
        case FORM_ALTERNATING: return launch_window_k<P, FORM_ALTERNATING, XD>(a, st);
        default: return hipErrorInvalidValue;
    }
}

// The binary32 forms' kernels live in kernels_f32.hip and kernels_f32c.hip
// alone: a second instantiation elsewhere, compiled with another scheduler,
// would leave it to the linker which of the two copies a launch runs.
template <int XD>
hipError_t launch_window_any(const WindowLaunch &a, hipStream_t st) {
    switch (a.precision) {
        case HEAT_FP64: return launch_window_f<F64, XD>(a, st);
        case HEAT_FP32: return launch_window_fp32(a, st);
        case HEAT_FP32C: return launch_window_fp32c(a, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace heat
