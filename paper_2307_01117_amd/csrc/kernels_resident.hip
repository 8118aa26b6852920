// kernels_resident.hip -- the resident kernel's binary64 instantiations (every
// register form) and the precision dispatch; the binary32 forms' live in
// kernels_f32.hip and kernels_f32c.hip, built with their own scheduler.
#include "resident.h"

namespace heat {

hipError_t launch_resident(int precision, const ResidentArgs &a, int K, int form, int G, int xd,
                           hipStream_t st, int *blocks_per_cu) {
    switch (precision) {
        case HEAT_FP64:
            return resident_any_xd<F64, (1 << FORM_INPLACE) | (1 << FORM_PINGPONG) |
                                            (1 << FORM_ALTERNATING)>(a, K, form, G, xd, st,
                                                                     blocks_per_cu);
        case HEAT_FP32: return launch_resident_fp32(a, K, form, G, xd, st, blocks_per_cu);
        case HEAT_FP32C: return launch_resident_fp32c(a, K, form, G, xd, st, blocks_per_cu);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace heat
