// kernels_xchg.hip -- the round kernel whose workgroup waves share one tile
// and swap edge cells through LDS every K/4 steps (window.h, round.h).
#include "round.h"

namespace heat {

hipError_t launch_window_xchg(const WindowLaunch &a, hipStream_t st) {
    return launch_window_any<true>(a, st);
}

}  // namespace heat
