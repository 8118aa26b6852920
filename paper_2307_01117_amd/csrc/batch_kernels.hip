// batch_kernels.hip -- the batching form's launchers and its binary64
// kernel classes (batch_kernels.h); the binary32 forms' classes are in
// kernels_f32.hip and kernels_f32c.hip.
#include "batch_kernels.h"

namespace heat {

// Kernel classes of the batch (the fastest register form of each, measured).
hipError_t launch_batch_round(int precision, int K, int G, const BatchRing *rings,
                              const int64_t *tile_prefix, int k, int active, int64_t items, int wpg,
                              hipStream_t st) {
    if (items <= 0) return hipSuccess;
    if (G > 1) {
        if (G > 4) return hipErrorInvalidValue;
        if (precision == HEAT_FP64 && K == 64)
            return launch_batch_round_x<F64, 64, FORM_ALTERNATING>(rings, tile_prefix, k, active,
                                                                   items, G, st);
        if (precision == HEAT_FP32)
            return launch_batch_round_fp32(K, G, rings, tile_prefix, k, active, items, wpg, st);
        if (precision == HEAT_FP32C)
            return launch_batch_round_fp32c(K, G, rings, tile_prefix, k, active, items, wpg, st);
        return hipErrorInvalidValue;
    }
    if (precision == HEAT_FP64 && K == 64)
        return launch_batch_round_t<F64, 64, FORM_ALTERNATING>(rings, tile_prefix, k, active, items,
                                                               wpg, st);
    if (precision == HEAT_FP64 && K == 32)
        return launch_batch_round_t<F64, 32, FORM_ALTERNATING>(rings, tile_prefix, k, active, items,
                                                               wpg, st);
    if (precision == HEAT_FP32)
        return launch_batch_round_fp32(K, 1, rings, tile_prefix, k, active, items, wpg, st);
    if (precision == HEAT_FP32C)
        return launch_batch_round_fp32c(K, 1, rings, tile_prefix, k, active, items, wpg, st);
    return hipErrorInvalidValue;
}

hipError_t launch_batch(int precision, int K, const BatchPlanDev &plan, int grid, int wpg,
                        hipStream_t st) {
    if (precision == HEAT_FP64 && K == 32) return launch_batch_t<F64, 32>(plan, grid, wpg, st);
    if (precision == HEAT_FP32) return launch_batch_fp32(K, plan, grid, wpg, st);
    if (precision == HEAT_FP32C) return launch_batch_fp32c(K, plan, grid, wpg, st);
    return hipErrorInvalidValue;
}

int batch_grid_size(int precision, int K, int wpg, int *grid) {
    int dev = 0, cus = 0;
    HEAT_HIP(hipGetDevice(&dev));
    HEAT_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    int nb = 0;
    if (precision == HEAT_FP64 && K == 32) nb = occupancy_blocks<F64, 32>(wpg);
    else if (precision == HEAT_FP32) nb = batch_occupancy_fp32(K, wpg);
    else if (precision == HEAT_FP32C) nb = batch_occupancy_fp32c(K, wpg);
    if (nb < 1) nb = 1;
    *grid = nb * cus;
    return HEAT_OK;
}

}  // namespace heat
