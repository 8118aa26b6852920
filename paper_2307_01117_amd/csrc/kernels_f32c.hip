// kernels_f32c.hip -- every kernel of the compensated binary32 form: the
// round kernels of the plain path, lone and exchanging waves (round.h), and
// the batching form's class (batch_kernels.h).  This file alone is built
// with LLVM's max-ilp instruction scheduler (see build.py): the compensated
// update is a chain of dependent operations per cell, and interleaving the
// chains of neighbouring cells pairs more VALU instructions than the default
// occupancy-first schedule (measured on MI355X with an earlier ten-operation
// update: 5,430 against 4,790 GCUP/s for the best shape of each on a
// 1e8-cell ring).  The instruction order does not change any result.
#include "batch_kernels.h"
#include "resident.h"
#include "round.h"

namespace heat {

// The coefficient's low part as the kernels derive it, rl = fl32(r - fl32(r)),
// is zero: r is a binary32 number (or within 2^-150 of one).
static bool low_part_zero(double r) {
    const float rh = (float)r;
    return (float)(r - (double)rh) == 0.0f;
}

// Window kernels for both coefficient classes: the general form, and the
// form without the low-part term for a binary32 coefficient (one operation
// fewer per cell update, the same bits).
template <class P>
static hipError_t launch_window_comp(const WindowLaunch &a, hipStream_t st) {
    switch (a.xd) {
        case 0: return launch_window_f<P, 0>(a, st);
        case 4: return launch_window_f<P, 4>(a, st);
        case 2: return launch_window_f<P, 2>(a, st);
        default: return hipErrorInvalidValue;
    }
}

// The lighter kernel's 32-cell lone waves, in place or ping-pong, run the
// ping-pong sweep held to 3 waves per SIMD.  Its state (u, e and their
// second copies: 4 x 32 registers) takes 171 VGPRs unconstrained, so 2
// waves per SIMD; with the cap 168 and 3 waves, and then it outruns the
// in-place sweep (140 VGPRs, 3 waves) at every ring length and group size
// measured on MI355X: 1e5 to 1e8 cells, 1 to 8 waves per group, +2.5 % to
// +9.5 % (1e8 cells: 6,906 against 6,458 GCUP/s).  Under the cap the
// compiler keeps one 64-bit per-lane value in scratch memory across the
// step loop (8 bytes written and read once per lane and launch: 6 % over
// the round's algorithmic HBM bytes, on a kernel bound by its arithmetic);
// a build without the spill (the kernel alone in its file, 168 VGPRs, no
// scratch) ran 5 % slower: the register it frees serves the step loop.
// The general form's kernel (with the low-part term) ran slower under the
// same cap and keeps its own.  The sweep order changes no bit of the result.
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(3)))
k_window_c0_lone32(const float *__restrict__ src, float *__restrict__ dst, int64_t N, int32_t H,
                   int32_t steps, double r, int64_t tiles, int64_t W, int32_t vec_ok,
                   double *part_in, double *part_out) {
    const int lane = threadIdx.x & 63;
    const int wpg = blockDim.x >> 6;
    const int wave = threadIdx.x >> 6;
    const int64_t part = xcd_remap(blockIdx.x, gridDim.x) * wpg + wave;
    if (part >= tiles) return;
    window_tile<F32C0, 32, FORM_PINGPONG, 0>(src, dst, N, H, steps, r, part * W, W, vec_ok != 0,
                                             lane, part_in, part_out, part, wpg, wave);
}

static hipError_t launch_window_c0_lone32(const WindowLaunch &a, hipStream_t st) {
    const int64_t W = window_tile_cells(32, a.H, a.wpg, 0);
    const int64_t tiles = (a.N + W - 1) / W;
    const int64_t blocks = (tiles + a.wpg - 1) / a.wpg;
    const int vec_ok = aligned16(a.src) && aligned16(a.dst);
    hipLaunchKernelGGL(k_window_c0_lone32, dim3((unsigned)blocks), dim3(64 * a.wpg), 0, st,
                       reinterpret_cast<const float *>(a.src), reinterpret_cast<float *>(a.dst), a.N,
                       a.H, a.steps, a.r, tiles, W, vec_ok, a.part_in, a.part_out);
    return hipGetLastError();
}

hipError_t launch_window_fp32c(const WindowLaunch &a, hipStream_t st) {
    if (a.precision != HEAT_FP32C) return hipErrorInvalidValue;
    if (!low_part_zero(a.r)) return launch_window_comp<F32C>(a, st);
    if (a.xd == 0 && a.K == 32 && (a.form == FORM_INPLACE || a.form == FORM_PINGPONG))
        return launch_window_c0_lone32(a, st);
    return launch_window_comp<F32C0>(a, st);
}

// The resident kernel in the in-place form, for both coefficient classes.
hipError_t launch_resident_fp32c(const ResidentArgs &a, int K, int form, int G, int xd,
                                 hipStream_t st, int *blocks_per_cu) {
    return low_part_zero(a.r)
               ? resident_any_xd<F32C0, 1 << FORM_INPLACE>(a, K, form, G, xd, st, blocks_per_cu)
               : resident_any_xd<F32C, 1 << FORM_INPLACE>(a, K, form, G, xd, st, blocks_per_cu);
}

// The batch classes: 32-cell lanes swept in place (under this file's
// scheduler the fastest form at 32 cells per lane), one wave per tile, or
// for long rings tiles of 4 waves that swap edges through LDS (the plain
// path's tuned compensated shape).
constexpr int BATCH_FP32C_FORM = FORM_INPLACE;

hipError_t launch_batch_round_fp32c(int K, int G, const BatchRing *rings,
                                    const int64_t *tile_prefix, int k, int active, int64_t items,
                                    int wpg, hipStream_t st) {
    if (K != 32) return hipErrorInvalidValue;
    if (G == 4)
        return launch_batch_round_x<F32C, 32, BATCH_FP32C_FORM>(rings, tile_prefix, k, active,
                                                                items, G, st);
    if (G != 1) return hipErrorInvalidValue;
    return launch_batch_round_t<F32C, 32, BATCH_FP32C_FORM>(rings, tile_prefix, k, active, items,
                                                            wpg, st);
}

hipError_t launch_batch_fp32c(int K, const BatchPlanDev &plan, int grid, int wpg,
                              hipStream_t st) {
    if (K != 32) return hipErrorInvalidValue;
    return launch_batch_t<F32C, 32>(plan, grid, wpg, st);
}

int batch_occupancy_fp32c(int K, int wpg) {
    return K == 32 ? occupancy_blocks<F32C, 32>(wpg) : 0;
}

}  // namespace heat
