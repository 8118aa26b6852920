// kernels_xchg2.hip -- the binary64 round kernel whose workgroup waves share
// one tile and swap K/2 edge cells through LDS every K/2 steps (window.h,
// round.h): half as many exchanges as kernels_xchg.hip for twice the overlap
// between neighbouring waves, and a depth of 4 cells already at 8 cells per
// lane.  Its own translation unit, so that it compiles in parallel.
#include "round.h"

namespace heat {

hipError_t launch_window_xchg2(const WindowLaunch &a, hipStream_t st) {
    return launch_window_any<2>(a, st);
}

}  // namespace heat
