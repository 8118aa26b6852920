// kernels_f32.hip -- every kernel of the plain binary32 form except the
// one-step sweep: the round kernels of the plain path, lone and exchanging
// waves (round.h), and the batching form's classes (batch_kernels.h).  This
// file is built with LLVM's max-ilp instruction scheduler (see build.py),
// which interleaves the four-operation chains of neighbouring cells so that
// more VALU instructions pair (measured on MI355X for the best shape of each
// size: +1 % to +4 % from 1e5 to 1e8 cells).  The instruction order does
// not change any result.
#include "batch_kernels.h"
#include "resident.h"
#include "round.h"

namespace heat {

hipError_t launch_window_fp32(const WindowLaunch &a, hipStream_t st) {
    if (a.precision != HEAT_FP32) return hipErrorInvalidValue;
    switch (a.xd) {
        case 0: return launch_window_f<F32, 0>(a, st);
        case 4: return launch_window_f<F32, 4>(a, st);
        case 2: return launch_window_f<F32, 2>(a, st);
        default: return hipErrorInvalidValue;
    }
}

// The batch classes: in-place sweeps, 32-cell lanes, or 64-cell lanes for
// rings of at least 65,536 cells, one wave per tile or (the longest rings)
// tiles of 4 waves that swap edges through LDS.
hipError_t launch_batch_round_fp32(int K, int G, const BatchRing *rings,
                                   const int64_t *tile_prefix, int k, int active, int64_t items,
                                   int wpg, hipStream_t st) {
    if (G == 4 && K == 64)
        return launch_batch_round_x<F32, 64, FORM_INPLACE>(rings, tile_prefix, k, active, items,
                                                           G, st);
    if (G != 1) return hipErrorInvalidValue;
    if (K == 64)
        return launch_batch_round_t<F32, 64, FORM_INPLACE>(rings, tile_prefix, k, active, items,
                                                           wpg, st);
    if (K == 32)
        return launch_batch_round_t<F32, 32, FORM_INPLACE>(rings, tile_prefix, k, active, items,
                                                           wpg, st);
    return hipErrorInvalidValue;
}

hipError_t launch_batch_fp32(int K, const BatchPlanDev &plan, int grid, int wpg, hipStream_t st) {
    if (K != 32) return hipErrorInvalidValue;
    return launch_batch_t<F32, 32>(plan, grid, wpg, st);
}

// The resident kernel in the in-place form (the binary32 forms' best).
hipError_t launch_resident_fp32(const ResidentArgs &a, int K, int form, int G, int xd,
                                hipStream_t st, int *blocks_per_cu) {
    return resident_any_xd<F32, 1 << FORM_INPLACE>(a, K, form, G, xd, st, blocks_per_cu);
}

int batch_occupancy_fp32(int K, int wpg) {
    return K == 32 ? occupancy_blocks<F32, 32>(wpg) : 0;
}

}  // namespace heat
