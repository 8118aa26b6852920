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
#include <atomic>
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
    int64_t min_nt[RESIDENT_POINTS] = {0, 0, 0};   // shortest winning run per point
                                                   // (0: it does not gain there)
    int gain_milli[RESIDENT_POINTS] = {0, 0, 0};   // gain at full SIMD load per point,
                                                   // thousandths (0: cannot run there)
};
struct ResidentSet {
    ResidentEntry s[RESIDENT_SHAPES];
    int n = 0;
};

struct TuneTable {
    std::mutex mu;
    TuneEntry e[3][NBUCKETS];
    BatchEntry b[3][NBUCKETS];
    ResidentSet rs[3][NQUART];
    bool env_loaded = false;
    TuneTable() {
        for (int p = 0; p < 3; ++p)
            for (int b = 0; b < NBUCKETS; ++b)
                // defaults from a sweep on MI355X at N = 1e8 (see default_* in runtime.hip)
                e[p][b] = TuneEntry{32, p == HEAT_FP32C ? 64 : 96, 2, 3, HEAT_EXCHANGE_NONE};
    }
};

// Bumped whenever the table may have changed (a file loaded, an autotuner
// installed), so callers can cache what they derived from it.
std::atomic<uint64_t> g_generation{0};

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
    // a file's r-lines replace the quarter decades they name
    bool named[3][NQUART] = {};
    while (std::fgets(line, sizeof line, f)) {
        if (!std::strchr(line, '\n') && !std::feof(f)) {
            // longer than the buffer: a comment's rest is skipped, anything
            // else is refused
            int ch;
            while ((ch = std::fgetc(f)) != EOF && ch != '\n') {
            }
            if (line[0] != '#') {
                rc = fail(HEAT_EINVAL, "tuning table line too long: %.40s...", line);
                break;
            }
            continue;
        }
        if (line[0] == '#' || line[0] == '\n') continue;
        if (line[0] == 'r') {
            // resident shape: "r precision quarter_bucket K T G form exchange
            // min_nt" (one shortest winning run for the whole quarter decade)
            // or "... min_nt at each point, gain_milli at each point"
            int p, b, K, T, G, form, xchg, gm[RESIDENT_POINTS] = {0, 0, 0};
            long long m3[RESIDENT_POINTS] = {0, 0, 0};
            int got = std::sscanf(line + 1, "%d %d %d %d %d %d %d %lld %lld %lld %d %d %d", &p,
                                  &b, &K, &T, &G, &form, &xchg, &m3[0], &m3[1], &m3[2], &gm[0],
                                  &gm[1], &gm[2]);
            long long mn = m3[0];
            if (got == 8) {
                m3[1] = m3[2] = mn;
            } else if (got == 13) {
                // every number >= 0, a shortest run recorded at some point
                bool ok = gm[0] >= 0 && gm[1] >= 0 && gm[2] >= 0;
                mn = 0;
                for (long long m : m3) {
                    ok = ok && m >= 0;
                    mn = std::max(mn, m);
                }
                got = ok ? 8 : -1;
            } else {
                got = -1;
            }
            // "r precision quarter_bucket 0 0 0 0 0 0": no resident shape for it
            if (got == 8 && p >= 0 && p <= 2 && b >= 0 && b < NQUART && K == 0 && T == 0 &&
                G == 0 && form == 0 && xchg == 0 && mn == 0) {
                std::lock_guard<std::mutex> lk(t.mu);
                t.rs[p][b] = ResidentSet{};
                named[p][b] = true;
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
            ResidentSet &set = t.rs[p][b];
            if (!named[p][b]) set = ResidentSet{};
            named[p][b] = true;
            if (set.n == RESIDENT_SHAPES) {
                rc = fail(HEAT_EINVAL, "more than %d resident shapes for one quarter decade: %s",
                          RESIDENT_SHAPES, line);
                break;
            }
            set.s[set.n++] = ResidentEntry{K, T, G, form, xchg,
                                           {(int64_t)m3[0], (int64_t)m3[1], (int64_t)m3[2]},
                                           {gm[0], gm[1], gm[2]}};
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
    g_generation.fetch_add(1);
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

int tuned_resident(int64_t N, int precision, ResidentChoice (&out)[RESIDENT_SHAPES]) {
    if (precision < 0 || precision > 2) return 0;
    load_env_once();
    TuneTable &t = table();
    std::lock_guard<std::mutex> lk(t.mu);
    const ResidentSet &set = t.rs[precision][quarter_bucket_of(N)];
    for (int i = 0; i < set.n; ++i) {
        const ResidentEntry &e = set.s[i];
        out[i] = ResidentChoice{heat_config{HEAT_KERNEL_RESIDENT, e.K, e.T, e.G, e.form, e.xchg},
                                {(double)e.min_nt[0], (double)e.min_nt[1], (double)e.min_nt[2]},
                                {e.gain_milli[0] / 1000.0, e.gain_milli[1] / 1000.0,
                                 e.gain_milli[2] / 1000.0}};
    }
    return set.n;
}

uint64_t tune_generation() {
    load_env_once();
    return g_generation.load();
}

void resident_points(int64_t N, int64_t (&pts)[RESIDENT_POINTS]) {
    const int q = quarter_bucket_of(N);
    const int64_t lo = quarter_edge(q), hi = std::max(lo, quarter_edge(q + 1) - 1);
    pts[0] = lo;
    pts[1] = (int64_t)std::llround(std::sqrt((double)lo * (double)hi));
    pts[2] = hi;
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
        for (int b = 0; b < NQUART; ++b)
            for (int i = 0; i < t.rs[p][b].n; ++i) {
                const ResidentEntry &e = t.rs[p][b].s[i];
                if (!any)
                    std::fprintf(f, "# resident kernel: r precision quarter_bucket(4 log10 N) "
                                    "cells_per_lane steps_per_round waves_per_group "
                                    "register_form exchange,\n# then at the quarter decade's "
                                    "lower end, middle and upper end its shortest winning run "
                                    "(0: none),\n# then there its gain at full load "
                                    "(thousandths)\n");
                any = true;
                std::fprintf(f, "r %d %d %d %d %d %d %d %lld %lld %lld %d %d %d\n", p, b, e.K,
                             e.T, e.G, e.form, e.xchg, (long long)e.min_nt[0],
                             (long long)e.min_nt[1], (long long)e.min_nt[2], e.gain_milli[0],
                             e.gain_milli[1], e.gain_milli[2]);
            }
    std::fclose(f);
    return HEAT_OK;
}

// Gain a tuned batch class must show over the rule on the synthetic batch.
constexpr double BATCH_TUNE_MARGIN = 1.03;

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
        g_generation.fetch_add(1);
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
        g_generation.fetch_add(1);
    }
    if (best_out) *best_out = bc;
    if (best_gcups) *best_gcups = best;
    return HEAT_OK;
}

// The resident kernel against the round kernel the planner runs (the
// table's shape), for N's quarter decade: every resident shape that can be
// resident there is timed over a long run at both ends of the quarter decade
// (its speed jumps with the tile count against the CU count, so a shape
// that fits one end may not fit the other; each time the fastest of three
// calls, the compensated form's shapes also at a binary32 coefficient, whose
// kernel differs).  Among the shapes whose smallest gain over the round
// kernel is at least RESIDENT_TUNE_MARGIN, the one whose smallest gain at full
// SIMD load (each end's gain over its load efficiency: the ends sample a
// saw-tooth of tile counts against CUs, which the planner evaluates at the
// N of each call) is the largest wins; that gain is recorded.  Then it and
// the round kernel are timed over a short run at both ends too.  Each
// kernel's time is a fixed cost plus a cost per step, so the two lengths
// give, in each case, the run length from which the resident one is faster;
// the largest is recorded.
int heat_autotune_resident(int32_t precision, int64_t N, int32_t install, heat_config *best_out,
                           int64_t *min_steps_out, double *gain_out) {
    if (precision != HEAT_FP64 && precision != HEAT_FP32 && precision != HEAT_FP32C)
        return fail(HEAT_EINVAL, "unknown precision %d", precision);
    if (N < 1 || N > (int64_t(1) << 34)) return fail(HEAT_EINVAL, "N out of range");
    int rc = device_pool_setup();
    if (rc) return rc;
    const int q = quarter_bucket_of(N);
    constexpr int NPOINT = RESIDENT_POINTS;
    int64_t pts[NPOINT];
    resident_points(N, pts);
    const int64_t hi = pts[NPOINT - 1];
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
    const int64_t Nmax = hi;
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
    // the coefficients: heat_autotune's, and for the compensated form also
    // one that is a binary32 number (its kernel then drops the coefficient's
    // low part, and with it some registers): a shape must gain with both
    const bool comp = precision == HEAT_FP32C;
    const double r_list[2] = {comp ? 0.3 : 0.25, 0.25};
    const int nr = comp ? 2 : 1;
    // one untimed call (it also refuses a shape that cannot be resident),
    // then the fastest of three timed ones; every call asks for the sums and
    // so waits for its result, as the calls the resident kernel is chosen
    // for do (the round kernel then pays the same wait)
    double s0 = 0.0, s1 = 0.0;
    auto time_run = [&](const heat_config &c, int64_t n, int64_t nt, double r,
                        double *ms_out) -> int {
        int rc2 = heat_solve_dev_cfg(a, w, n, 1, r, nt, precision, &c, st, &s0, &s1);
        if (rc2) return rc2;
        double best_ms = 0.0;
        for (int rep = 0; rep < 3; ++rep) {
            hipError_t e2 = hipEventRecord(e0, st);
            if (e2 == hipSuccess)
                rc2 = heat_solve_dev_cfg(a, w, n, 1, r, nt, precision, &c, st, &s0, &s1);
            if (!rc2 && e2 == hipSuccess) e2 = hipEventRecord(e1, st);
            if (!rc2 && e2 == hipSuccess) e2 = hipEventSynchronize(e1);
            float ms = 0.f;
            if (!rc2 && e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, e0, e1);
            if (!rc2 && e2 != hipSuccess) rc2 = fail_hip(e2, "autotune timing");
            if (rc2) return rc2;
            if (rep == 0 || ms < best_ms) best_ms = ms;
        }
        *ms_out = best_ms;
        return HEAT_OK;
    };
    const int64_t nt_short = 128, nt_long = 1024;
    const heat_config tb{HEAT_KERNEL_TB, 0, 0, 0, 0, 0};   // what the planner runs
    // [point][coefficient]
    double tb_l[NPOINT][2] = {}, tb_s[NPOINT][2] = {};
    for (int k = 0; k < NPOINT && !rc; ++k)
        for (int ri = 0; ri < nr && !rc; ++ri) {
            rc = time_run(tb, pts[k], nt_long, r_list[ri], &tb_l[k][ri]);
            if (!rc) rc = time_run(tb, pts[k], nt_short, r_list[ri], &tb_s[k][ri]);
        }
    if (rc) {
        cleanup();
        return rc;
    }
    // every shape that can run at some point: its smallest gain over the
    // coefficients at each point, over its load efficiency there
    struct Cand {
        heat_config c{};
        double full[NPOINT] = {0, 0, 0};
        double gain[NPOINT] = {0, 0, 0};
        int wins = 0;
    };
    std::vector<Cand> cands;
    struct GX { int G, x; };
    for (int K : {8, 16, 32})
        for (GX gx : {GX{1, HEAT_EXCHANGE_NONE}, GX{2, HEAT_EXCHANGE_LDS_DEEP},
                      GX{4, HEAT_EXCHANGE_LDS}, GX{4, HEAT_EXCHANGE_LDS_DEEP},
                      GX{8, HEAT_EXCHANGE_LDS_DEEP}})
            for (int form : {1, 3})
                for (int T : {16, 24, 32, 48, 64, 96, 128}) {
                    if (comp && T != default_steps_per_round(N, precision)) continue;
                    if (precision != HEAT_FP64 && form != 1) continue;
                    if (3 * T > 64 * K) continue;
                    if (gx.x == HEAT_EXCHANGE_LDS && K < 16) continue;
                    Cand cd;
                    cd.c = heat_config{HEAT_KERNEL_RESIDENT, K, T, gx.G, form, gx.x};
                    bool runs = false;
                    for (int k = 0; k < NPOINT; ++k) {
                        // run as the planner would at this length
                        heat_config fitted;
                        double eff = 0.0;
                        rc = resident_fit(pts[k], nt_long, precision, cd.c, &fitted, &eff);
                        if (rc == HEAT_EINVAL) continue;   // cannot be resident here
                        double g = 1e300;
                        for (int ri = 0; ri < nr && !rc; ++ri) {
                            double ms = 0.0;
                            rc = time_run(fitted, pts[k], nt_long, r_list[ri], &ms);
                            if (!rc) g = ms > 0.0 ? std::min(g, tb_l[k][ri] / ms) : 0.0;
                        }
                        if (rc == HEAT_EINVAL) continue;
                        if (rc) {
                            cleanup();
                            return rc;
                        }
                        if (g > 0.0 && eff > 0.0) {
                            cd.gain[k] = g;
                            cd.full[k] = g / eff;
                            runs = true;
                        }
                    }
                    rc = HEAT_OK;
                    if (runs) cands.push_back(cd);
                }
    // the model over the quarter decade: at each N of a fine grid, the shape
    // whose interpolated gain at full load times its load efficiency there is
    // the largest wins, if that is at least the margin
    constexpr int NGRID = 64;
    for (int j = 0; j < NGRID; ++j) {
        const int64_t n = (int64_t)std::llround(
            std::exp(std::log((double)pts[0]) +
                     (std::log((double)hi) - std::log((double)pts[0])) * j / (NGRID - 1)));
        double best_pred = 0.0;
        int best_i = -1;
        for (size_t i = 0; i < cands.size(); ++i) {
            heat_config fitted;
            double eff = 0.0;
            if (resident_fit(n, nt_long, precision, cands[i].c, &fitted, &eff) != HEAT_OK)
                continue;
            const double pred = resident_interp(cands[i].full, pts, n) * eff;
            if (pred > best_pred) {
                best_pred = pred;
                best_i = (int)i;
            }
        }
        if (best_i >= 0 && best_pred >= RESIDENT_TUNE_MARGIN) ++cands[best_i].wins;
    }
    // recorded: the fastest shape at each point (where it gains), then the
    // others the model picks, most often first
    std::vector<size_t> order;
    auto take = [&](size_t i) {
        if (order.size() < (size_t)RESIDENT_SHAPES &&
            std::find(order.begin(), order.end(), i) == order.end())
            order.push_back(i);
    };
    for (int k = 0; k < NPOINT; ++k) {
        int best_i = -1;
        for (size_t i = 0; i < cands.size(); ++i)
            if (cands[i].gain[k] >= RESIDENT_TUNE_MARGIN &&
                (best_i < 0 || cands[i].gain[k] > cands[best_i].gain[k]))
                best_i = (int)i;
        if (best_i >= 0) take((size_t)best_i);
    }
    std::vector<size_t> by_wins;
    for (size_t i = 0; i < cands.size(); ++i)
        if (cands[i].wins > 0) by_wins.push_back(i);
    std::stable_sort(by_wins.begin(), by_wins.end(),
                     [&](size_t a, size_t b) { return cands[a].wins > cands[b].wins; });
    for (size_t i : by_wins) take(i);
    // each recorded shape with the run length from which it is faster at the
    // points where it gains (else at its best point)
    ResidentSet found;
    int64_t min_steps = 0;
    for (size_t oi = 0; oi < order.size() && !rc; ++oi) {
        const Cand &cd = cands[order[oi]];
        ResidentEntry f{cd.c.cells_per_lane, cd.c.steps_per_round, cd.c.waves_per_group,
                        cd.c.register_form, cd.c.exchange, {0, 0, 0}, {0, 0, 0}};
        int top = 0;
        for (int k = 1; k < NPOINT; ++k)
            if (cd.gain[k] > cd.gain[top]) top = k;
        for (int k = 0; k < NPOINT && !rc; ++k) {
            f.gain_milli[k] = (int)std::lround(cd.full[k] * 1000.0);
            if (cd.gain[k] <= 0.0 || (cd.gain[k] < 1.0 && k != top)) continue;
            heat_config fitted;
            double eff = 0.0;
            if (resident_fit(pts[k], nt_long, precision, cd.c, &fitted, &eff) != HEAT_OK) continue;
            double cross = 1.0;
            for (int ri = 0; ri < nr && !rc; ++ri) {
                double rs_s = 0.0, rs_l = 0.0;
                rc = time_run(fitted, pts[k], nt_short, r_list[ri], &rs_s);
                if (!rc) rc = time_run(fitted, pts[k], nt_long, r_list[ri], &rs_l);
                if (rc) break;
                // t = a + b * nt for each kernel; the resident one is faster
                // from nt* = (a_res - a_tb) / (b_tb - b_res) on
                const double span = (double)(nt_long - nt_short);
                const double tl = tb_l[k][ri], ts = tb_s[k][ri];
                const double b_tb = (tl - ts) / span, b_rs = (rs_l - rs_s) / span;
                const double a_tb = ts - b_tb * nt_short, a_rs = rs_s - b_rs * nt_short;
                const double x = b_rs < b_tb ? (a_rs - a_tb) / (b_tb - b_rs) : (double)nt_short;
                cross = std::max(cross, std::min(x, (double)nt_long));
            }
            f.min_nt[k] = std::max<int64_t>(1, (int64_t)std::ceil(cross));
            min_steps = std::max(min_steps, f.min_nt[k]);
        }
        found.s[found.n++] = f;
    }
    cleanup();
    if (rc) return rc;
    if (install) {
        TuneTable &t = table();
        std::lock_guard<std::mutex> lk(t.mu);
        t.rs[precision][q] = found;
        g_generation.fetch_add(1);
    }
    // reported: the first recorded shape (else the fastest at the lower
    // end), and the smallest over the points of the best gain measured there
    double worst = 1e300;
    heat_config lead{};
    double lead_gain = 0.0;
    for (int k = 0; k < NPOINT; ++k) {
        double g = 0.0;
        for (const Cand &cd : cands) g = std::max(g, cd.gain[k]);
        worst = std::min(worst, g);
    }
    for (const Cand &cd : cands)
        if (cd.gain[0] > lead_gain) {
            lead_gain = cd.gain[0];
            lead = cd.c;
        }
    if (!order.empty()) lead = cands[order[0]].c;
    if (best_out) *best_out = lead;
    if (min_steps_out) *min_steps_out = found.n ? min_steps : 0;
    if (gain_out) *gain_out = cands.empty() ? 0.0 : worst;
    return HEAT_OK;
}

}  // extern "C"
