// kernels.hip -- HIP kernels (gfx950, wave64) of the periodic 1D heat stencil
// and their host launchers.
//
// Operation: the explicit-Euler step of the paper's Eq. (heat:discrete) on a
// periodic ring (Section 2), applied nt times with a Jacobi double buffer.
// The paper's per-step ghost-zone exchange between segments (Section 2, last
// paragraph) appears here at four levels:
//   * between lanes of a wavefront: DPP rotates (no memory traffic);
//   * between the waves of a workgroup that share a tile: edge cells
//     swapped through LDS every K/4 steps (round.h, window.h);
//   * between tiles of one round: overlapping windows read from HBM;
//   * between rounds: the kernel boundary (plain form) or per-tile epoch
//     counters (fused batch form).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "heat_device.h"
#include "heat_internal.h"
#include "round.h"
#include "window.h"

namespace heat {

// ==================================================================== STEP
// One step per launch.  A wave owns a chunk of 64 vectors of 16 bytes, one
// per lane, so the load and the store are each one fully coalesced
// instruction: lane L holds cells base + L*VEC + [0, VEC).  Neighbours inside
// the chunk come from the adjacent lanes (DPP); the two cells just outside it
// are read by lanes 0 and 63.  Every cell is read once and written once, so
// both accesses are marked streaming (non-temporal): measured on MI355X this
// lifts a plain copy from about 5.8 to 6.5 TB/s.

template <class P>
__global__ void __launch_bounds__(512)
k_step(const typename P::T *__restrict__ src, typename P::T *__restrict__ dst, int64_t N, double r_in,
       int64_t chunks, int32_t vec_ok) {
    using T = typename P::T;
    using VT = typename Vec16<T>::type;
    constexpr int VEC = P::VEC;
    constexpr int64_t CH = 64 * VEC;
    const int lane = threadIdx.x & 63;
    const int wpg = blockDim.x >> 6;
    const int64_t chunk = xcd_remap(blockIdx.x, gridDim.x) * wpg + (threadIdx.x >> 6);
    if (chunk >= chunks) return;
    const T r = (T)r_in;
    const int64_t base = chunk * CH;
    if (vec_ok && base + CH <= N) {
        const VT x = load_stream(reinterpret_cast<const VT *>(src + base + lane * VEC));
        T c[VEC];
#pragma unroll
        for (int k = 0; k < VEC; ++k) c[k] = x[k];
        T edge = T(0);
        if (lane == 0) edge = src[base == 0 ? N - 1 : base - 1];
        if (lane == 63) edge = src[base + CH == N ? 0 : base + CH];
        const T prev_last = from_prev(c[VEC - 1]);
        const T next_first = from_next(c[0]);
        const T left = lane == 0 ? edge : prev_last;
        const T right = lane == 63 ? edge : next_first;
        VT y;
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const T l = k == 0 ? left : c[k - 1];
            const T q = k == VEC - 1 ? right : c[k + 1];
            y[k] = cell_update(l, c[k], q, r);
        }
        store_stream(y, reinterpret_cast<VT *>(dst + base + lane * VEC));
    } else {
#pragma unroll
        for (int k = 0; k < VEC; ++k) {
            const int64_t i = base + lane * VEC + k;
            if (i < N) {
                const T l = src[i == 0 ? N - 1 : i - 1];
                const T q = src[i == N - 1 ? 0 : i + 1];
                dst[i] = cell_update(l, src[i], q, r);
            }
        }
    }
}

// ===================================================================== SUM
// binary64 sum with a fixed shape: block b owns [b*N/G, (b+1)*N/G), each
// thread keeps a Neumaier-compensated sum of its strided elements, the block
// adds the 256 thread totals in a fixed tree, a second one-block pass does
// the same over the G partials.  Same N -> same order -> same bits.

__device__ __forceinline__ void neumaier_add(double &s, double &c, double x) {
    const double t = s + x;
    if (fabs(s) >= fabs(x))
        c += (s - t) + x;
    else
        c += (x - t) + s;
    s = t;
}

template <int BS>
__device__ __forceinline__ double block_tree_sum(double v) {
    __shared__ double red[BS];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = BS / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + w];
        __syncthreads();
    }
    return red[0];
}

// Slices start on multiples of 4 elements so the body can use 16-byte
// (binary64) or 16-byte (binary32, 4 at a time) loads when aligned.
template <class T>
__global__ void __launch_bounds__(256) k_sum_partial(const T *__restrict__ u, int64_t N,
                                                     double *__restrict__ partial, int32_t vec_ok) {
    const int64_t G = gridDim.x, b = blockIdx.x;
    const int64_t lo = ((b * N) / G) & ~int64_t(3);
    const int64_t hi = b + 1 == G ? N : (((b + 1) * N) / G) & ~int64_t(3);
    double s = 0.0, c = 0.0;
    if (vec_ok) {
        using VT = typename Vec16<T>::type;
        constexpr int VEC = 16 / sizeof(T);
        const int64_t nv = (hi - lo) / VEC;
        const VT *p = reinterpret_cast<const VT *>(u + lo);
        for (int64_t i = threadIdx.x; i < nv; i += 256) {
            VT x = p[i];
            const T *xs = reinterpret_cast<const T *>(&x);
#pragma unroll
            for (int k = 0; k < VEC; ++k) neumaier_add(s, c, (double)xs[k]);
        }
        for (int64_t i = lo + nv * VEC + threadIdx.x; i < hi; i += 256) neumaier_add(s, c, (double)u[i]);
    } else {
        for (int64_t i = lo + threadIdx.x; i < hi; i += 256) neumaier_add(s, c, (double)u[i]);
    }
    const double tot = block_tree_sum<256>(s + c);
    if (threadIdx.x == 0) partial[b] = tot;
}

// Final pass: workgroup b reduces the n partial sums partial[b*n, b*n + n)
// into out[b], so the sums before and after a run reduce in one launch.
// Thread t adds partial[t], partial[t + 1024], ... in that order (a fixed
// order for a given n); each thread keeps 16 loads in flight, so up to 16,384
// partials cost one memory latency instead of one per 2,048.
constexpr int FINAL_THREADS = 1024;
constexpr int FINAL_LOADS = 16;

__global__ void __launch_bounds__(FINAL_THREADS) k_sum_final(const double *__restrict__ partial,
                                                             int64_t n, double *__restrict__ out) {
    const double *p = partial + (int64_t)blockIdx.x * n;
    double s = 0.0, c = 0.0;
    for (int64_t base = threadIdx.x; base < n; base += (int64_t)FINAL_LOADS * FINAL_THREADS) {
        double x[FINAL_LOADS];
#pragma unroll
        for (int u = 0; u < FINAL_LOADS; ++u) {
            const int64_t i = base + (int64_t)u * FINAL_THREADS;
            x[u] = i < n ? p[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < FINAL_LOADS; ++u)
            if (base + (int64_t)u * FINAL_THREADS < n) neumaier_add(s, c, x[u]);
    }
    const double tot = block_tree_sum<FINAL_THREADS>(s + c);
    if (threadIdx.x == 0) out[blockIdx.x] = tot;
}

// ================================================================= CONVERT

// Stage-in and stage-out of the binary32 forms, optionally relative to a
// shift s: v = fl32(u - s) (binary64 difference, then round to nearest
// even) and u = s + v (binary64).  s = 0 takes the plain conversions, which
// keep the sign of zero.

__global__ void k_f64_to_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n,
                             double s) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = s != 0.0 ? (float)(a[i] - s) : (float)a[i];
}

__global__ void k_f32_to_f64(const float *__restrict__ a, double *__restrict__ b, int64_t n,
                             double s) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b[i] = s != 0.0 ? s + (double)a[i] : (double)a[i];   // widening is exact
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ==================================================================== COPY
// Bandwidth probe: every lane moves one 16-byte vector, coalesced and
// streaming, exactly like the fast path of k_step without the arithmetic.

__global__ void __launch_bounds__(256) k_copy(const v4u32 *__restrict__ src, v4u32 *__restrict__ dst,
                                              int64_t nvec) {
    const int64_t i = (xcd_remap(blockIdx.x, gridDim.x) * (int64_t)(blockDim.x >> 6) +
                       (threadIdx.x >> 6)) * 64 + (threadIdx.x & 63);
    if (i < nvec) store_stream(load_stream(src + i), dst + i);
}

// ================================================================ LAUNCHERS


int64_t window_tile_cells(int K, int H, int wpg, int xd) {
    const int64_t win = 64 * (int64_t)K;
    if (!xd) return win - 2 * (int64_t)H;
    return wpg * win - (wpg - 1) * 2 * (int64_t)(K / xd) - 2 * (int64_t)H;
}

hipError_t launch_window(const WindowLaunch &a, hipStream_t st) {
    switch (a.xd) {
        case 0: return launch_window_lone(a, st);
        case 4: return launch_window_xchg(a, st);
        case 2: return launch_window_xchg2(a, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_window_lone(const WindowLaunch &a, hipStream_t st) {
    return launch_window_any<0>(a, st);
}

hipError_t launch_sum_partials(const double *partial, int64_t n, int arrays, double *d_out,
                               hipStream_t st) {
    hipLaunchKernelGGL(k_sum_final, dim3((unsigned)arrays), dim3(FINAL_THREADS), 0, st, partial, n,
                       d_out);
    return hipGetLastError();
}

int64_t step_chunk_cells(int precision) {
    return 64 * (precision == HEAT_FP64 ? F64::VEC : F32::VEC);
}

hipError_t launch_step(int precision, const void *src, void *dst, int64_t N, double r, int wpg,
                       hipStream_t st) {
    const int64_t CH = step_chunk_cells(precision);
    const int64_t chunks = (N + CH - 1) / CH;
    const int64_t blocks = (chunks + wpg - 1) / wpg;
    const int vec_ok = aligned16(src) && aligned16(dst);
    if (precision == HEAT_FP64)
        hipLaunchKernelGGL(k_step<F64>, dim3((unsigned)blocks), dim3(64 * wpg), 0, st,
                           reinterpret_cast<const double *>(src), reinterpret_cast<double *>(dst), N,
                           r, chunks, vec_ok);
    else if (precision == HEAT_FP32)
        hipLaunchKernelGGL(k_step<F32>, dim3((unsigned)blocks), dim3(64 * wpg), 0, st,
                           reinterpret_cast<const float *>(src), reinterpret_cast<float *>(dst), N,
                           r, chunks, vec_ok);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// Workgroups of the first pass: one per 4,096 cells, at most SUM_BLOCKS.  A
// fixed shape for a given N, so the sum is deterministic; a short ring (the
// requests of the serving mix) no longer launches thousands of empty slices.
static unsigned sum_blocks(int64_t N) {
    const int64_t b = (N + 4095) / 4096;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(SUM_BLOCKS, b));
}

hipError_t launch_sum(int precision, const void *u, int64_t N, double *partial, double *d_out,
                      hipStream_t st) {
    const int vec_ok = aligned16(u);
    const unsigned G = sum_blocks(N);
    if (precision == HEAT_FP64)
        hipLaunchKernelGGL(k_sum_partial<double>, dim3(G), dim3(256), 0, st,
                           reinterpret_cast<const double *>(u), N, partial, vec_ok);
    else
        hipLaunchKernelGGL(k_sum_partial<float>, dim3(G), dim3(256), 0, st,
                           reinterpret_cast<const float *>(u), N, partial, vec_ok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(FINAL_THREADS), 0, st, partial, (int64_t)G,
                       d_out);
    return hipGetLastError();
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 65536) b = 65536;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t st, double shift) {
    hipLaunchKernelGGL(k_f64_to_f32, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n, shift);
    return hipGetLastError();
}

hipError_t launch_f32_to_f64(const float *src, double *dst, int64_t n, hipStream_t st, double shift) {
    hipLaunchKernelGGL(k_f32_to_f64, dim3(grid_for(n)), dim3(256), 0, st, src, dst, n, shift);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t st) {
    const int64_t nvec = (int64_t)(bytes / 16);
    const int64_t chunks = (nvec + 63) / 64;
    const int64_t blocks = (chunks + 3) / 4;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, st,
                       reinterpret_cast<const v4u32 *>(src), reinterpret_cast<v4u32 *>(dst), nvec);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

}  // namespace heat
