// heat_internal.h -- host-side internals shared by the library's .hip files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>

#include <string>

#include "heat.h"

namespace heat {

// ----------------------------------------------------------- errors

// Record a thread-local message for heat_last_error() and return `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
// HIP error -> HEAT_EDEVICE with the call site in the message.
int fail_hip(hipError_t e, const char *what);

#define HEAT_HIP(call)                                             \
    do {                                                           \
        hipError_t _e = (call);                                    \
        if (_e != hipSuccess) return ::heat::fail_hip(_e, #call);  \
    } while (0)

// One piece of a host <-> device copy (runtime.hip, stage_copies).
struct StageSeg {
    void *dev;
    void *host;
    size_t bytes;
};
// Blocking copy of a list of segments between pageable host memory and the
// device: waits for `st` first (the device side may be stream-ordered
// memory or the result of work on it); totals of 64 MiB or more go through
// the pinned multi-lane staging, smaller ones through plain copies on `st`.
int stage_copies(bool to_device, const StageSeg *segs, size_t count, hipStream_t st);

inline size_t storage_bytes(int precision) { return precision == HEAT_FP64 ? 8 : 4; }

// A launch's grid counts work-items in 32 bits: one wavefront per tile must
// stay below this many threads.
constexpr int64_t MAX_GRID_THREADS = (int64_t(1) << 32) - 256;

// ----------------------------------------------------------- planning

struct Plan {
    int kernel = HEAT_KERNEL_TB;
    int K = 16;          // cells per lane (TB)
    int T = 32;          // steps per round
    int H = 32;          // halo cells per side of a window (multiple of 4, >= T)
    int wpg = 4;         // wavefronts per workgroup
    int form = 3;        // TB register form: 1 in-place, 2 ping-pong, 3 alternating
    int xd = 0;          // TB: 0 = a tile per wave; 4 or 2 = the workgroup's waves share a
                         // tile and swap K/xd edge cells through LDS every K/xd steps
    int64_t W = 0;       // output cells per tile (TB) / cells per chunk (STEP)
    int64_t tiles = 0;   // tiles (TB) or chunks (STEP) per launch
    int64_t parts = 0;   // per-wave partial sums of a fused checksum (TB)
    int64_t rounds = 0;  // launches
};

// Fill `p` for a problem; returns HEAT_OK or HEAT_EINVAL (message set).
int make_plan(int64_t N, int64_t nt, int precision, const heat_config *cfg, Plan *p);

// Steps per round the planner uses by default for (N, precision).  For the
// compensated form this fixes where the state is folded to binary32, so it
// is a pure function of (N, precision) -- never of timing or of a batch mix.
int default_steps_per_round(int64_t N, int precision);
int default_cells_per_lane(int64_t N, int precision);
// Steps per round used for a run of nt steps with target round length T: a
// result-neutral even split near T for binary64 and plain binary32; T itself
// (or nt, if shorter) for the compensated form, whose round length is part
// of its result.
int64_t balanced_steps_per_round(int64_t nt, int64_t T, int precision);
// Halo depth H >= steps for a window of 64*K cells (line-aligned when possible).
int halo_cells(int64_t steps, int precision, int K);
int default_register_form(int64_t N, int precision);
// Launch shape from the tuning table for a ring of length N.
void tuned_shape(int64_t N, int precision, int *K, int *T, int *wpg, int *form, int *exchange);
// Resident shapes the tuning table keeps per quarter decade (the planner
// picks one per call), and the points of a quarter decade the tuner
// measures them at: its two ends and their geometric middle.
constexpr int RESIDENT_SHAPES = 6;
constexpr int RESIDENT_POINTS = 3;
struct ResidentChoice {
    heat_config c;                   // kernel = RESIDENT, the tuned T
    double min_nt[RESIDENT_POINTS];  // at each point, the run length from which it is
                                     // faster (0: it does not gain there)
    double gain[RESIDENT_POINTS];    // gain over the round kernel at full SIMD load at
                                     // each point (0: cannot run there; all 0: not recorded)
};
// The resident shapes recorded for N's quarter decade; returns how many.
int tuned_resident(int64_t N, int precision, ResidentChoice (&out)[RESIDENT_SHAPES]);
// Changes whenever the tuning table may have changed.
uint64_t tune_generation();
// The measuring points of N's quarter decade.
void resident_points(int64_t N, int64_t (&pts)[RESIDENT_POINTS]);
// A quantity recorded at the points (a shape's gain at full load, or its
// shortest winning run) at N: linear in log N between the points, constant
// beyond them; a point where it is 0 (not measured) is skipped.
inline double resident_interp(const double (&g)[RESIDENT_POINTS],
                              const int64_t (&pts)[RESIDENT_POINTS], int64_t N) {
    double xs[RESIDENT_POINTS], ys[RESIDENT_POINTS];
    int n = 0;
    for (int k = 0; k < RESIDENT_POINTS; ++k) {
        const double x = std::log((double)pts[k]);
        if (g[k] > 0.0 && (n == 0 || x > xs[n - 1])) {
            xs[n] = x;
            ys[n++] = g[k];
        }
    }
    if (n == 0) return 0.0;
    const double x = std::log((double)N);
    if (x <= xs[0]) return ys[0];
    for (int i = 1; i < n; ++i)
        if (x <= xs[i]) return ys[i - 1] + (ys[i] - ys[i - 1]) * (x - xs[i - 1]) / (xs[i] - xs[i - 1]);
    return ys[n - 1];
}

// Gain the resident kernel must show over the round kernel on a long run.
constexpr double RESIDENT_TUNE_MARGIN = 1.03;

// A resident shape fitted to N: for binary64 and binary32 (whose results do
// not depend on T) the exchange interval, from the tuned T down to half of
// it, whose tiles put the fewest waves on the busiest SIMD (a CU takes
// ceil(tiles / CUs) workgroups, whose waves share its 4 SIMDs, and every
// tile waits for the slowest); the longest on a tie.  *fitted: that shape;
// *eff: its load efficiency, the mean number of waves per SIMD over the
// busiest SIMD's, in (0, 1].  HEAT_EINVAL if no interval lets every tile be
// resident at once.
int resident_fit(int64_t N, int64_t nt, int precision, const heat_config &c,
                 heat_config *fitted, double *eff);

// ----------------------------------------------------------- kernels

// One round of the temporal-blocked window kernel: every tile loads 64*K
// cells per wave starting H cells left of its output, advances `steps`
// (<= H) steps in registers and writes its W output cells (window_tile_cells).
struct WindowLaunch {
    int precision = HEAT_FP64;
    int K = 32;
    int form = 3;                 // register form: 1 in-place, 2 ping-pong, 3 alternating
    const void *src = nullptr;
    void *dst = nullptr;
    int64_t N = 0;
    int H = 0;
    int steps = 0;
    double r = 0.0;
    int wpg = 2;
    int xd = 0;                   // 0: a tile per wave; 4 or 2: the wpg waves of a workgroup
                                  // share one tile, exchange depth K/xd
    double *part_in = nullptr;    // per-wave sums of the input (first round), or NULL
    double *part_out = nullptr;   // per-wave sums of the output (last round), or NULL
};
hipError_t launch_window(const WindowLaunch &a, hipStream_t st);
hipError_t launch_window_lone(const WindowLaunch &a, hipStream_t st);   // kernels.hip
hipError_t launch_window_xchg(const WindowLaunch &a, hipStream_t st);   // kernels_xchg.hip
hipError_t launch_window_xchg2(const WindowLaunch &a, hipStream_t st);  // kernels_xchg2.hip
// binary32, lone or exchanging waves as a.xd says                    // kernels_f32.hip
hipError_t launch_window_fp32(const WindowLaunch &a, hipStream_t st);
// compensated binary32, lone or exchanging waves as a.xd says         // kernels_f32c.hip
hipError_t launch_window_fp32c(const WindowLaunch &a, hipStream_t st);
// Output cells of one tile: 64K - 2H for a lone wave (xd = 0); for wpg
// cooperating waves, wpg windows of 64K cells overlapping by 2*(K/xd), minus 2H.
int64_t window_tile_cells(int K, int H, int wpg, int xd);
// Reduce `arrays` consecutive arrays of n partial sums each (partial[a*n, a*n + n))
// into d_out[a], one workgroup per array, in one launch.
hipError_t launch_sum_partials(const double *partial, int64_t n, int arrays, double *d_out,
                               hipStream_t st);

// One step of the coalesced sweep (binary64 or binary32).
hipError_t launch_step(int precision, const void *src, void *dst, int64_t N, double r, int wpg,
                       hipStream_t st);

// Cells per wave chunk of the step kernel.
int64_t step_chunk_cells(int precision);

// Deterministic binary64 sum: `partial` needs SUM_BLOCKS doubles (fewer are
// used for rings under 16.8 M cells: one slice per 4,096 cells), result in
// d_out[0].
constexpr int SUM_BLOCKS = 4096;
hipError_t launch_sum(int precision, const void *u, int64_t N, double *partial, double *d_out,
                      hipStream_t st);

// binary64 <-> binary32 state conversions, relative to `shift` (0 = none):
// dst = fl32(src - shift) and dst = shift + src.
hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t st,
                             double shift = 0.0);
hipError_t launch_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t st,
                             double shift = 0.0);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st);
// Streaming 16-byte copy (bandwidth probe), same launch shape as k_step.
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st);

// ----------------------------------------------------------- resident

// One launch of the resident kernel (resident.h): every tile's window stays
// in registers for all nt steps; tiles swap edges through buf[] every T steps.
struct ResidentArgs {
    void *u;                 // state in and out, N cells
    int64_t N;
    int64_t W;               // output cells per tile
    int64_t tiles;
    int64_t nt;
    int32_t H;               // halo cells per side (>= T)
    int32_t T;               // steps between edge exchanges
    double r;
    uint64_t *xa;            // exchange area, resident_area_words(); every tag <= epoch_base
    uint32_t *flags;         // [tiles] epoch counters, all <= epoch_base at launch
    uint32_t epoch_base;     // this launch's epochs are epoch_base + 1, 2, ...
    uint32_t *status;        // [1] pinned host word: zero at launch; nonzero once a wait timed out
    int64_t spin_limit;
    double *part_in;         // per-wave sums of the input, or NULL
    double *part_out;        // per-wave sums of the output, or NULL
    int32_t vec_ok;          // u 16-byte aligned
    int32_t lds_edges;       // 1: the LDS tile copy holds the two edge regions only
                             // (resident_tile_cells); 0: the whole tile span W + 2H
};
// 64-bit words of a resident launch's exchange area: two parities, per tile
// its first and its last H owned cells, each cell one word per 32 bits of its
// storage type (32 bits of the value beside a 32-bit epoch tag).
inline int64_t resident_area_words(int64_t tiles, int H, int cell_bytes) {
    return 2 * tiles * 2 * (int64_t)H * (cell_bytes / 4);
}
// Launch (or, with blocks_per_cu set, report how many workgroups of that
// shape one CU holds) for a precision, cells per lane, register form,
// waves per group and exchange depth (0, 4 or 2).  kernels_resident.hip
// dispatches; the binary32 forms' instantiations live in kernels_f32.hip /
// kernels_f32c.hip (in-place form only).
hipError_t launch_resident(int precision, const ResidentArgs &a, int K, int form, int G, int xd,
                           hipStream_t st, int *blocks_per_cu);
hipError_t launch_resident_fp32(const ResidentArgs &a, int K, int form, int G, int xd,
                                hipStream_t st, int *blocks_per_cu);
hipError_t launch_resident_fp32c(const ResidentArgs &a, int K, int form, int G, int xd,
                                 hipStream_t st, int *blocks_per_cu);

// ----------------------------------------------------------- batching

struct BatchRing {          // one ring of a fused launch (device table entry)
    void *buf[2];           // state at even / odd rounds
    int64_t N;
    int64_t W;              // output cells per tile
    int64_t tiles;
    int64_t flag_base;      // first epoch counter of this ring
    double r;
    int32_t H;              // halo (>= steps of any round)
    int32_t T;              // steps per full round
    int32_t rounds;         // rounds (the last one may be shorter)
    int32_t copy_round;     // 1 if an extra copy-back round follows (odd rounds)
    int64_t nt;
    int32_t vec_ok;         // both buffers 16-byte aligned
    int32_t round0;         // rounds already done before this launch sequence
    int32_t K;              // cells per lane of the kernel class that runs it
    int32_t G;              // waves sharing one tile (1: a wave per tile; >1: LDS exchange)
};

struct BatchPlanDev {       // device pointers of one fused launch
    const BatchRing *rings; // sorted by total rounds (incl. copy), descending
    const int64_t *tile_prefix;   // [nrings+1]
    const int64_t *round_start;   // [max_rounds+1] first item of each round
    const int32_t *active;        // [max_rounds] rings still running in round k
    uint32_t *flags;              // epoch counter per (ring, tile)
    unsigned long long *work;     // [0] next unclaimed work item
    uint32_t *status;             // [0] nonzero once a dependency wait timed out
    int64_t total_items;
    int32_t max_rounds;
    int32_t chunk;
    int64_t spin_limit;
};

hipError_t launch_batch(int precision, int K, const BatchPlanDev &plan, int grid, int wpg,
                        hipStream_t st);
// One round of every active ring (rings[0, active) in the sorted table).
// G = 1: one wave per tile, wpg waves per workgroup; G > 1: one workgroup of
// G waves per tile (LDS edge exchange; wpg ignored).
hipError_t launch_batch_round(int precision, int K, int G, const BatchRing *rings,
                              const int64_t *tile_prefix, int k, int active, int64_t items, int wpg,
                              hipStream_t st);
int batch_grid_size(int precision, int K, int wpg, int *grid);
// The plain binary32 form's batch classes (kernels_f32.hip).
hipError_t launch_batch_round_fp32(int K, int G, const BatchRing *rings,
                                   const int64_t *tile_prefix, int k, int active, int64_t items,
                                   int wpg, hipStream_t st);
hipError_t launch_batch_fp32(int K, const BatchPlanDev &plan, int grid, int wpg, hipStream_t st);
int batch_occupancy_fp32(int K, int wpg);
// The compensated form's batch classes (kernels_f32c.hip).
hipError_t launch_batch_round_fp32c(int K, int G, const BatchRing *rings,
                                    const int64_t *tile_prefix, int k, int active, int64_t items,
                                    int wpg, hipStream_t st);
hipError_t launch_batch_fp32c(int K, const BatchPlanDev &plan, int grid, int wpg,
                              hipStream_t st);
int batch_occupancy_fp32c(int K, int wpg);

// Shared device-side state for the batch/server runtime (stream-ordered pool).
int device_pool_setup();

}  // namespace heat
