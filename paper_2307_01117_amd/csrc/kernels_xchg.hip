// kernels_xchg.hip -- the binary64 round kernel whose workgroup waves share
// one tile and swap K/4 edge cells through LDS every K/4 steps (window.h,
// round.h); the deeper exchange (K/2) is in kernels_xchg2.hip.
#include "round.h"

namespace heat {

hipError_t launch_window_xchg(const WindowLaunch &a, hipStream_t st) {
    return launch_window_any<4>(a, st);
}

}  // namespace heat
