// tune.hip -- the planner's tuning table and the autotuner that fills it.
//
// The table maps (precision, ring-length bucket) to the temporal-blocking
// launch shape: cells per lane K, target steps per round T, wavefronts per
// workgroup, register form and whether the waves of a workgroup share one
// tile through LDS edge exchanges.  None of these change a binary64 or binary32
// result (the update of every cell is the same whatever the tiling), and the
// compensated form's round length is fixed outside the table, so tuning is
// always result-neutral.  The autotuner times every candidate shape with HIP
// events on a synthetic ring of the requested length and keeps the fastest.
//
// A second table holds the batching form's kernel class per (precision,
// bucket): cells per lane K, waves per tile G and the target round length,
// picked by the batch autotuner, which times every built class on a
// synthetic batch of rings of one length.  A third holds, per quarter decade
// of N where it won, the resident kernel's shape and the shortest run it is
// faster on.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "heat_batch.h"
#include "heat_internal.h"

namespace heat {

namespace {

constexpr int NBUCKETS = 10;   // [10^b, 10^(b+1)) for b = 0..8, and >= 1e9
constexpr int NQUART = 40;     // resident entries: [10^(q/4), 10^((q+1)/4)), and >= 10^9.75

struct TuneEntry {
    int K, T, wpg, form;   // form: 1 in-place, 2 ping-pong, 3 alternating
    int xchg;              // heat_exchange: 1 lone waves, 2 LDS exchange
};

struct BatchEntry {
    int K = 0, G = 0, T = 0;   // K = 0: not tuned (the batching form's own rule)
};

// The resident kernel's shape for a bucket, and the shortest run it is
// measured faster on (K = 0: the round kernel always).
struct ResidentEntry {
    int K = 0, T = 0, G = 0, form = 0, xchg = 0;
    int64_t min_nt = 0;
};

struct TuneTable {
    std::mutex mu;
    TuneEntry e[3][NBUCKETS];
    BatchEntry b[3][NBUCKETS];
    ResidentEntry rs[3][NQUART];
    bool env_loaded = false;
    TuneTable() {
        for (int p = 0; p < 3; ++p)
            for (int b = 0; b < NBUCKETS; ++b)
                // defaults from a sweep on MI355X at N = 1e8 (see default_* in runtime.hip)
                e[p][b] = TuneEntry{32, p == HEAT_FP32C ? 64 : 96, 2, 3, HEAT_EXCHANGE_NONE};
    }
};

TuneTable &table() {
    static TuneTable t;
    return t;
}

int bucket_of(int64_t N) {
    int b = 0;
    for (int64_t x = 10; b < NBUCKETS - 1 && N >= x; x *= 10) ++b;
    return b;
}

// Quarter-decade bucket: the largest q with N >= ceil(10^(q/4)).
const int64_t QUARTER_EDGE[NQUART] = {
        1,         2,          4,          6,          10,         18,         32,
        57,        100,        178,        317,        563,        1000,       1779,
        3163,      5624,       10000,      17783,      31623,      56235,      100000,
        177828,    316228,     562342,     1000000,    1778280,    3162278,    5623414,
        10000000,  17782795,   31622777,   56234133,   100000000,  177827942,  316227767,
        562341326, 1000000000, 1778279411, 3162277661LL, 5623413252LL};

int quarter_bucket_of(int64_t N) {
    int q = 0;
    while (q + 1 < NQUART && N >= QUARTER_EDGE[q + 1]) ++q;
    return q;
}

// First ring length of quarter decade q (q = NQUART: one past the last).
int64_t quarter_edge(int q) {
    return q < NQUART ? QUARTER_EDGE[q] : QUARTER_EDGE[NQUART - 1] * 2;
}

int load_file(const char *path) {
    FILE *f = std::fopen(path, "r");
    if (!f) return fail(HEAT_EINVAL, "cannot open tuning table %s", path);
    TuneTable &t = table();
    char line[256];
    int n = 0, rc = HEAT_OK;
    while (std::fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        if (line[0] == 'r') {
            // resident shape: "r precision quarter_bucket K T G form exchange min_nt"
            int p, b, K, T, G, form, xchg;
            long long mn;
            const int got = std::sscanf(line + 1, "%d %d %d %d %d %d %d %lld", &p, &b, &K, &T, &G,
                                        &form, &xchg, &mn);
            // "r precision quarter_bucket 0 0 0 0 0 0": no resident shape for it
            if (got == 8 && p >= 0 && p <= 2 && b >= 0 && b < NQUART && K == 0 && T == 0 &&
                G == 0 && form == 0 && xchg == 0 && mn == 0) {
                std::lock_guard<std::mutex> lk(t.mu);
                t.rs[p][b] = ResidentEntry{};
                ++n;
                continue;
            }
            if (got != 8 || p < 0 || p > 2 || b < 0 || b >= NQUART ||
                (K != 8 && K != 16 && K != 32 && K != 64) || T < 1 || (T % 4) || 3 * T > 64 * K ||
                G < 1 || G > 8 || form < 1 || form > 3 || (p != HEAT_FP64 && form != 1) ||
                xchg < HEAT_EXCHANGE_NONE || xchg > HEAT_EXCHANGE_LDS_DEEP ||
                (xchg == HEAT_EXCHANGE_NONE && G != 1) ||
                (xchg == HEAT_EXCHANGE_LDS && (G < 2 || K < 16)) ||
                (xchg == HEAT_EXCHANGE_LDS_DEEP && (G < 2 || K < 8)) || mn < 1) {
                rc = fail(HEAT_EINVAL, "bad tuning table line: %s", line);
                break;
            }
            std::lock_guard<std::mutex> lk(t.mu);
            t.rs[p][b] = ResidentEntry{K, T, G, form, xchg, (int64_t)mn};
            ++n;
            continue;
        }
        if (line[0] == 'b') {
            // batch class: "b precision bucket K G T" ("... 0 0 0": the rule)
            int p, b, K, G, T;
            const int got = std::sscanf(line + 1, "%d %d %d %d %d", &p, &b, &K, &G, &T);
            const bool rule = got == 5 && K == 0 && G == 0 && T == 0;
            if (got != 5 || p < 0 || p > 2 || b < 0 || b >= NBUCKETS ||
                (!rule && (!batch_class_exists(p, K, G) || T < 1 || (T % 4) || 3 * T > 64 * K))) {
                rc = fail(HEAT_EINVAL, "bad tuning table line: %s", line);
                break;
            }
            std::lock_guard<std::mutex> lk(t.mu);
            t.b[p][b] = BatchEntry{K, G, T};
            ++n;
            continue;
        }
        int p, b, K, T, wpg, form, xchg = HEAT_EXCHANGE_NONE;
        const int got = std::sscanf(line, "%d %d %d %d %d %d %d", &p, &b, &K, &T, &wpg, &form, &xchg);
        if ((got != 6 && got != 7) || p < 0 || p > 2 || b < 0 || b >= NBUCKETS ||
            (K != 8 && K != 16 && K != 32 && K != 64) || T < 1 || (T % 4) || 3 * T > 64 * K ||
            wpg < 1 || wpg > 8 ||
            (K == 64 && form == 2 && p != HEAT_FP32) || form < 1 || form > 3 ||
            xchg < HEAT_EXCHANGE_NONE || xchg > HEAT_EXCHANGE_LDS_DEEP ||
            (xchg == HEAT_EXCHANGE_LDS && (wpg < 2 || K < 16)) ||
            (xchg == HEAT_EXCHANGE_LDS_DEEP && (wpg < 2 || K < 8))) {
            rc = fail(HEAT_EINVAL, "bad tuning table line: %s", line);
            break;
        }
        std::lock_guard<std::mutex> lk(t.mu);
        t.e[p][b] = TuneEntry{K, T, wpg, form, xchg};
        ++n;
    }
    std::fclose(f);
    return rc;
}

void load_env_once() {
    TuneTable &t = table();
    {
        std::lock_guard<std::mutex> lk(t.mu);
        if (t.env_loaded) return;
        t.env_loaded = true;
    }
    const char *path = std::getenv("HEAT_TUNE_TABLE");
    if (path && *path) (void)load_file(path);
}

}  // namespace

bool tuned_batch_class(int64_t N, int precision, int *K, int *G, int *T) {
    if (precision < 0 || precision > 2) return false;
    load_env_once();
    TuneTable &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    const BatchEntry &e = t.b[precision][bucket_of(N)];
    if (e.K == 0) return false;
    *K = e.K;
    *G = e.G;
    *T = e.T;
    return true;
}

bool tuned_resident(int64_t N, int precision, heat_config *c, int64_t *min_nt) {
    if (precision < 0 || precision > 2) return false;
    load_env_once();
    TuneTable &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    const ResidentEntry &e = t.rs[precision][quarter_bucket_of(N)];
    if (e.K == 0) return false;
    *c = heat_config{HEAT_KERNEL_RESIDENT, e.K, e.T, e.G, e.form, e.xchg};
    *min_nt = e.min_nt;
    return true;
}

void tuned_shape(int64_t N, int precision, int *K, int *T, int *wpg, int *form, int *exchange) {
    load_env_once();
    TuneTable &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    const TuneEntry &e = t.e[precision][bucket_of(N)];
    *K = e.K;
    *T = e.T;
    *wpg = e.wpg;
    *form = e.form;
    *exchange = e.xchg;
}

}  // namespace heat

using namespace heat;

// Deterministic synthetic fill (values in [0, 1)); speed does not depend on them.
__global__ void k_tune_fill(double *a, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        uint64_t x = (uint64_t)i * 0x9E3779B97F4A7C15ull;
        x ^= x >> 29;
        a[i] = (double)(x >> 11) * 0x1.0p-53;
    }
}

extern "C" {

int heat_tune_load(const char *path) {
    if (!path) return fail(HEAT_EINVAL, "path is NULL");
    return load_file(path);
}

int heat_tune_save(const char *path) {
    if (!path) return fail(HEAT_EINVAL, "path is NULL");
    FILE *f = std::fopen(path, "w");
    if (!f) return fail(HEAT_EINVAL, "cannot write %s", path);
    TuneTable &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    std::fprintf(f, "# precision bucket(log10 N) cells_per_lane steps_per_round waves_per_group "
                    "register_form exchange\n");
    for (int p = 0; p < 3; ++p)
        for (int b = 0; b < NBUCKETS; ++b)
            std::fprintf(f, "%d %d %d %d %d %d %d\n", p, b, t.e[p][b].K, t.e[p][b].T, t.e[p][b].wpg,
                         t.e[p][b].form, t.e[p][b].xchg);
    bool any = false;
    for (int p = 0; p < 3; ++p)
        for (int b = 0; b < NBUCKETS; ++b) {
            const BatchEntry &e = t.b[p][b];
            if (!e.K) continue;
            if (!any)
                std::fprintf(f, "# batch class: b precision bucket(log10 N) cells_per_lane "
                                "waves_per_tile steps_per_round\n");
            any = true;
            std::fprintf(f, "b %d %d %d %d %d\n", p, b, e.K, e.G, e.T);
        }
    any = false;
    for (int p = 0; p < 3; ++p)
        for (int b = 0; b < NQUART; ++b) {
            const ResidentEntry &e = t.rs[p][b];
            if (!e.K) continue;
            if (!any)
                std::fprintf(f, "# resident kernel: r precision quarter_bucket(4 log10 N) cells_per_lane "
                                "steps_per_round waves_per_group register_form exchange "
                                "min_steps\n");
            any = true;
            std::fprintf(f, "r %d %d %d %d %d %d %d %lld\n", p, b, e.K, e.T, e.G, e.form, e.xchg,
                         (long long)e.min_nt);
        }
    std::fclose(f);
    return HEAT_OK;
}

// Gain a tuned batch class must show over the rule on the synthetic batch.
constexpr double BATCH_TUNE_MARGIN = 1.03;
// Gain the resident kernel must show over the round kernel on a long run.
constexpr double RESIDENT_TUNE_MARGIN = 1.03;

int heat_autotune_batch(int32_t precision, int64_t N, int32_t install, int32_t *K_out,
                        int32_t *G_out, int32_t *T_out, double *best_gcups) {
    if (precision != HEAT_FP64 && precision != HEAT_FP32 && precision != HEAT_FP32C)
        return fail(HEAT_EINVAL, "unknown precision %d", precision);
    if (N < 1 || N >= 100000000) return fail(HEAT_EINVAL, "N out of range (1 to 99,999,999)");
    int rc = device_pool_setup();
    if (rc) return rc;
    // Rings whose lengths spread log-uniformly over N's decade [10^b,
    // 10^(b+1)) (ring i of n: 10^(b + (i + 1/2)/n) cells), as many as hold
    // about 3e7 cells (at most 4,096).  One length at the decade's low edge
    // would favour tiles that happen to fit it (measured: tuned on rings of
    // exactly 1e5 cells, the classes lost 8 % on the uneven 4,096-ring batch).
    int b = 0;
    for (int64_t x = 10; b < NBUCKETS - 1 && N >= x; x *= 10) ++b;
    const double lo = (double)b;
    std::vector<int64_t> lens;
    {
        const double mean = (std::pow(10.0, lo + 1) - std::pow(10.0, lo)) / std::log(10.0);
        const int64_t n = std::max<int64_t>(1, std::min<int64_t>(4096, (int64_t)(3e7 / mean)));
        for (int64_t i = 0; i < n; ++i) {
            const int64_t len = std::max<int64_t>(1, (int64_t)std::pow(10.0, lo + (i + 0.5) / n));
            lens.push_back(len);
        }
    }
    const int64_t count = (int64_t)lens.size();
    // Step counts spread over [100, 7,680] (ring i: the golden-ratio sequence
    // frac(i * 0.618...) scaled): a batch's rings run different numbers of
    // rounds, and one common count, or a short one, hides the halo work of
    // deep rounds (measured: tuned over 640 steps the classes picked 640-step
    // rounds that lost 8 % on the uneven 4,096-ring batch).
    std::vector<int64_t> nts((size_t)count);
    int64_t cups_nt = 0;
    for (int64_t i = 0; i < count; ++i) {
        const double f = std::fmod((double)i * 0.6180339887498949, 1.0);
        nts[(size_t)i] = 100 + (int64_t)(f * (7680 - 100));
        cups_nt += lens[(size_t)i] * nts[(size_t)i];
    }
    hipStream_t st = nullptr;
    HEAT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    const size_t es = storage_bytes(precision);
    void *a = nullptr, *w = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (a) (void)hipFreeAsync(a, st);
        if (w) (void)hipFreeAsync(w, st);
        (void)hipStreamSynchronize(st);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(st);
    };
    // the rings' states and scratch, each ring 256-byte aligned
    std::vector<size_t> off((size_t)count + 1, 0);
    for (int64_t i = 0; i < count; ++i)
        off[(size_t)i + 1] = off[(size_t)i] +
                             (((size_t)lens[(size_t)i] * std::max<size_t>(es, 8) + 255) & ~size_t(255));
    hipError_t e = hipMallocAsync(&a, off[(size_t)count], st);
    if (e == hipSuccess) e = hipMallocAsync(&w, off[(size_t)count], st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return fail_hip(e, "batch autotune setup");
    }
    hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, st, (double *)w,
                       (int64_t)(off[(size_t)count] / 8));
    std::vector<heat_ring> rings((size_t)count);
    for (int64_t i = 0; i < count; ++i) {
        char *u = (char *)a + off[(size_t)i], *s2 = (char *)w + off[(size_t)i];
        const int64_t len = lens[(size_t)i];
        if (precision == HEAT_FP64)
            e = hipMemcpyAsync(u, s2, (size_t)len * 8, hipMemcpyDeviceToDevice, st);
        else
            e = launch_f64_to_f32((const double *)s2, (float *)u, len, st);
        if (e != hipSuccess) break;
        rings[(size_t)i] = heat_ring{len, nts[(size_t)i], 0.25, precision, 1, u, s2};
    }
    if (e != hipSuccess) {
        cleanup();
        return fail_hip(e, "batch autotune fill");
    }
    // candidates: the rule (K = 0) first, then every built class at every
    // round length its window allows
    struct Cand {
        int K, G, T;
    };
    std::vector<Cand> cands{{0, 0, 0}};
    const int Ts_all[] = {64, 96, 128, 160, 192, 256, 320, 480, 640};
    for (int K : {32, 64})
        for (int G : {1, 4})
            for (int T : Ts_all) {
                if (!batch_class_exists(precision, K, G)) continue;
                if (precision == HEAT_FP32C && T != default_steps_per_round(N, precision)) continue;
                if (3 * T > 64 * K) continue;
                cands.push_back({K, G, T});
            }
    double best = -1.0, rule = -1.0;
    int bK = 0, bG = 0, bT = 0;
    for (const Cand &cd : cands) {
                const int K = cd.K, G = cd.G, T = cd.T;
                // one untimed pass, then one timed pass
                rc = batch_run_class(rings.data(), (int32_t)count, st, K, G, T);
                if (!rc) e = hipEventRecord(e0, st);
                if (!rc && e == hipSuccess)
                    rc = batch_run_class(rings.data(), (int32_t)count, st, K, G, T);
                if (!rc && e == hipSuccess) e = hipEventRecord(e1, st);
                if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (rc || e != hipSuccess) {
                    cleanup();
                    return rc ? rc : fail_hip(e, "batch autotune timing");
                }
                const double g = (double)cups_nt / (ms * 1e-3) / 1e9;
                if (K == 0) rule = g;
                if (g > best) {
                    best = g;
                    bK = K;
                    bG = G;
                    bT = T;
                }
    }
    cleanup();
    // a class replaces the rule only if it is clearly faster on this batch
    // (the synthetic batch stands in for real ones only roughly)
    if (bK && best < BATCH_TUNE_MARGIN * rule) {
        bK = bG = bT = 0;
        best = rule;
    }
    if (install) {
        TuneTable &t = table();
        std::lock_guard<std::mutex> lk(t.mu);
        t.b[precision][bucket_of(N)] = BatchEntry{bK, bG, bT};
    }
    if (K_out) *K_out = bK;
    if (G_out) *G_out = bG;
    if (T_out) *T_out = bT;
    if (best_gcups) *best_gcups = best;
    return HEAT_OK;
}

int heat_autotune(int32_t precision, int64_t N, int32_t install, heat_config *best_out,
                  double *best_gcups) {
    if (precision != HEAT_FP64 && precision != HEAT_FP32 && precision != HEAT_FP32C)
        return fail(HEAT_EINVAL, "unknown precision %d", precision);
    if (N < 1 || N > (int64_t(1) << 34)) return fail(HEAT_EINVAL, "N out of range");
    int rc = device_pool_setup();
    if (rc) return rc;
    hipStream_t st = nullptr;
    HEAT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    const size_t es = storage_bytes(precision);
    void *a = nullptr, *w = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (a) (void)hipFreeAsync(a, st);
        if (w) (void)hipFreeAsync(w, st);
        (void)hipStreamSynchronize(st);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(st);
    };
    hipError_t e = hipMallocAsync(&a, (size_t)N * std::max<size_t>(es, 8), st);
    if (e == hipSuccess) e = hipMallocAsync(&w, (size_t)N * std::max<size_t>(es, 8), st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return fail_hip(e, "autotune setup");
    }
    hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, st, (double *)w, N);
    if (precision == HEAT_FP64)
        e = hipMemcpyAsync(a, w, (size_t)N * 8, hipMemcpyDeviceToDevice, st);
    else
        e = launch_f64_to_f32((const double *)w, (float *)a, N, st);
    if (e != hipSuccess) {
        cleanup();
        return fail_hip(e, "autotune fill");
    }
    const int Ts_all[] = {16, 32, 48, 64, 96, 128, 160, 192, 256, 320};
    double best = -1.0;
    heat_config bc{};
    // The coefficient the shapes are timed at.  The compensated form runs a
    // lighter kernel for a binary32 coefficient (no low-part term) with other
    // register needs, so it is timed at one that is not (0.3): a binary32
    // coefficient then runs its kernel on the general form's best shape
    // (measured on MI355X at 1e8 cells: within 0.5 % of that kernel's own
    // best, while the reverse cost the general form 11 %).
    const double r_tune = precision == HEAT_FP32C ? 0.3 : 0.25;
    for (int K : {8, 16, 32, 64})
        for (int form : {1, 2, 3})
            for (int wpg : {1, 2, 4, 8})
                for (int xchg : {HEAT_EXCHANGE_NONE, HEAT_EXCHANGE_LDS, HEAT_EXCHANGE_LDS_DEEP})
                    for (int T : Ts_all) {
                        if (precision == HEAT_FP32C && T != default_steps_per_round(N, precision))
                            continue;
                        if (3 * T > 64 * K) continue;
                        if (K == 64 && form == 2 && precision != HEAT_FP32) continue;
                        if (xchg == HEAT_EXCHANGE_LDS && (wpg < 2 || K < 16)) continue;
                        if (xchg == HEAT_EXCHANGE_LDS_DEEP && (wpg < 2 || K < 8)) continue;
                        heat_config c{HEAT_KERNEL_TB, K, T, wpg, form, xchg};
                        // whole rounds, at least 4 and at least 384 steps, so the
                        // per-launch overheads weigh as they do in real runs
                        int64_t R = std::max<int64_t>(4, (384 + T - 1) / T);
                        R += R & 1;   // even: no copy-back in the timed run
                        const int64_t nt = R * T;
                        rc = heat_solve_dev_cfg(a, w, N, 1, r_tune, T, precision, &c, st,
                                                nullptr, nullptr);
                        if (!rc) e = hipEventRecord(e0, st);
                        if (!rc && e == hipSuccess)
                            rc = heat_solve_dev_cfg(a, w, N, 1, r_tune, nt, precision, &c, st,
                                                    nullptr, nullptr);
                        if (!rc && e == hipSuccess) e = hipEventRecord(e1, st);
                        if (!rc && e == hipSuccess) e = hipEventSynchronize(e1);
                        float ms = 0.f;
                        if (!rc && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                        if (rc || e != hipSuccess) {
                            cleanup();
                            return rc ? rc : fail_hip(e, "autotune timing");
                        }
                        const double g = (double)N * (double)nt / (ms * 1e-3) / 1e9;
                        if (g > best) {
                            best = g;
                            bc = c;
                        }
                    }
    cleanup();
    if (install) {
        TuneTable &t = table();
        std::lock_guard<std::mutex> lk(t.mu);
        TuneEntry &en = t.e[precision][bucket_of(N)];
        en = TuneEntry{bc.cells_per_lane, bc.steps_per_round, bc.waves_per_group, bc.register_form,
                       bc.exchange};
        if (precision == HEAT_FP32C) en.T = default_steps_per_round(N, precision);
    }
    if (best_out) *best_out = bc;
    if (best_gcups) *best_gcups = best;
    return HEAT_OK;
}

// The resident kernel against the round kernel the planner runs (the
// table's shape), for N's quarter decade: every resident shape that can be
// resident there is timed over a long run at both ends of the quarter decade
// (its speed jumps with the tile count against the CU count, so a shape
// that fits one end may not fit the other), and the shape whose smaller gain
// over the round kernel is the largest wins; then it and the round kernel
// are timed over a short run at both ends too.  Each kernel's time is a fixed
// cost plus a cost per step, so the two lengths give, at each end, the run
// length from which the resident one is faster; the larger is recorded.  It
// is kept if its smaller gain is RESIDENT_TUNE_MARGIN.
int heat_autotune_resident(int32_t precision, int64_t N, int32_t install, heat_config *best_out,
                           int64_t *min_steps_out, double *gain_out) {
    if (precision != HEAT_FP64 && precision != HEAT_FP32 && precision != HEAT_FP32C)
        return fail(HEAT_EINVAL, "unknown precision %d", precision);
    if (N < 1 || N > (int64_t(1) << 34)) return fail(HEAT_EINVAL, "N out of range");
    int rc = device_pool_setup();
    if (rc) return rc;
    const int q = quarter_bucket_of(N);
    const int64_t ends[2] = {quarter_edge(q), std::max(quarter_edge(q), quarter_edge(q + 1) - 1)};
    hipStream_t st = nullptr;
    HEAT_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    const size_t es = storage_bytes(precision);
    void *a = nullptr, *w = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    auto cleanup = [&]() {
        if (a) (void)hipFreeAsync(a, st);
        if (w) (void)hipFreeAsync(w, st);
        (void)hipStreamSynchronize(st);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamDestroy(st);
    };
    const int64_t Nmax = ends[1];
    hipError_t e = hipMallocAsync(&a, (size_t)Nmax * std::max<size_t>(es, 8), st);
    if (e == hipSuccess) e = hipMallocAsync(&w, (size_t)Nmax * std::max<size_t>(es, 8), st);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        cleanup();
        return fail_hip(e, "autotune setup");
    }
    hipLaunchKernelGGL(k_tune_fill, dim3(1024), dim3(256), 0, st, (double *)w, Nmax);
    if (precision == HEAT_FP64)
        e = hipMemcpyAsync(a, w, (size_t)Nmax * 8, hipMemcpyDeviceToDevice, st);
    else
        e = launch_f64_to_f32((const double *)w, (float *)a, Nmax, st);
    if (e != hipSuccess) {
        cleanup();
        return fail_hip(e, "autotune fill");
    }
    // the coefficient as in heat_autotune
    const double r_tune = precision == HEAT_FP32C ? 0.3 : 0.25;
    // one untimed call (it also refuses a shape that cannot be resident),
    // then one timed
    auto time_run = [&](const heat_config &c, int64_t n, int64_t nt, double *ms_out) -> int {
        int rc2 = heat_solve_dev_cfg(a, w, n, 1, r_tune, nt, precision, &c, st, nullptr, nullptr);
        if (rc2) return rc2;
        hipError_t e2 = hipEventRecord(e0, st);
        if (e2 == hipSuccess)
            rc2 = heat_solve_dev_cfg(a, w, n, 1, r_tune, nt, precision, &c, st, nullptr, nullptr);
        if (!rc2 && e2 == hipSuccess) e2 = hipEventRecord(e1, st);
        if (!rc2 && e2 == hipSuccess) e2 = hipEventSynchronize(e1);
        float ms = 0.f;
        if (!rc2 && e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, e0, e1);
        if (!rc2 && e2 != hipSuccess) rc2 = fail_hip(e2, "autotune timing");
        *ms_out = ms;
        return rc2;
    };
    const int64_t nt_short = 128, nt_long = 1024;
    const heat_config tb{HEAT_KERNEL_TB, 0, 0, 0, 0, 0};   // what the planner runs
    double tb_l[2] = {0, 0}, tb_s[2] = {0, 0};
    for (int k = 0; k < 2 && !rc; ++k) {
        rc = time_run(tb, ends[k], nt_long, &tb_l[k]);
        if (!rc) rc = time_run(tb, ends[k], nt_short, &tb_s[k]);
    }
    if (rc) {
        cleanup();
        return rc;
    }
    const bool comp = precision == HEAT_FP32C;
    double best_score = 0.0;
    double best_l[2] = {0, 0};
    heat_config rc_best{};
    struct GX { int G, x; };
    for (int K : {8, 16, 32})
        for (GX gx : {GX{1, HEAT_EXCHANGE_NONE}, GX{2, HEAT_EXCHANGE_LDS_DEEP},
                      GX{4, HEAT_EXCHANGE_LDS}, GX{4, HEAT_EXCHANGE_LDS_DEEP},
                      GX{8, HEAT_EXCHANGE_LDS_DEEP}})
            for (int form : {1, 3})
                for (int T : {32, 48, 64, 96, 128}) {
                    if (comp && T != default_steps_per_round(N, precision)) continue;
                    if (precision != HEAT_FP64 && form != 1) continue;
                    if (3 * T > 64 * K) continue;
                    if (gx.x == HEAT_EXCHANGE_LDS && K < 16) continue;
                    heat_config c{HEAT_KERNEL_RESIDENT, K, T, gx.G, form, gx.x};
                    double ms[2] = {0, 0};
                    bool fits = true;
                    for (int k = 0; k < 2 && fits; ++k) {
                        rc = time_run(c, ends[k], nt_long, &ms[k]);
                        if (rc == HEAT_EINVAL) fits = false;   // not resident at this size
                        else if (rc) {
                            cleanup();
                            return rc;
                        }
                    }
                    if (!fits || ms[0] <= 0.0 || ms[1] <= 0.0) continue;
                    const double score = std::min(tb_l[0] / ms[0], tb_l[1] / ms[1]);
                    if (score > best_score) {
                        best_score = score;
                        rc_best = c;
                        best_l[0] = ms[0];
                        best_l[1] = ms[1];
                    }
                }
    rc = HEAT_OK;
    ResidentEntry found;
    if (best_score >= RESIDENT_TUNE_MARGIN) {
        double cross = 1.0;
        for (int k = 0; k < 2 && !rc; ++k) {
            double rs_s = 0.0;
            rc = time_run(rc_best, ends[k], nt_short, &rs_s);
            if (rc) break;
            // t = a + b * nt for each kernel; the resident one is faster from
            // nt* = (a_res - a_tb) / (b_tb - b_res) on
            const double span = (double)(nt_long - nt_short);
            const double b_tb = (tb_l[k] - tb_s[k]) / span, b_rs = (best_l[k] - rs_s) / span;
            const double a_tb = tb_s[k] - b_tb * nt_short, a_rs = rs_s - b_rs * nt_short;
            const double c = b_rs < b_tb ? (a_rs - a_tb) / (b_tb - b_rs) : (double)nt_short;
            cross = std::max(cross, std::min(c, (double)nt_long));
        }
        if (rc) {
            cleanup();
            return rc;
        }
        found = ResidentEntry{rc_best.cells_per_lane, rc_best.steps_per_round,
                              rc_best.waves_per_group, rc_best.register_form, rc_best.exchange,
                              (int64_t)std::ceil(cross)};
    }
    cleanup();
    if (install) {
        TuneTable &t = table();
        std::lock_guard<std::mutex> lk(t.mu);
        t.rs[precision][q] = found;
    }
    if (best_out) *best_out = best_score > 0.0 ? rc_best : heat_config{};
    if (min_steps_out) *min_steps_out = found.min_nt;
    if (gain_out) *gain_out = best_score;
    return HEAT_OK;
}

}  // extern "C"
