/*
 * heat.h -- C ABI of the MI355X (gfx950) periodic 1D heat-stencil library.
 *
 * Operation (paper, Section 2 "Model problem", Eq. heat:discrete with the
 * periodic boundary condition u(t, x) = u(t, L + x)): nt explicit-Euler steps
 *
 *     u_new[i] = u[i] + r * ((u[i-1] - 2 u[i]) + u[i+1]),   indices mod N,
 *
 * with r = alpha * dt / h^2 (the printed denominator "2h" is read as h^2, the
 * consistent second-order Laplacian; the caller supplies r directly).  Every
 * right-hand-side value is taken at the old time level.  The paper's parallel
 * algorithm (Section 2, last paragraph) cuts the ring into contiguous
 * segments that swap ghost cells every step; here the segments are tiles of
 * the GPU kernels, and `nparts` is validated and recorded but cannot change
 * the result (it is bit-identical for every 1 <= nparts <= N).
 *
 * Precisions:
 *   HEAT_FP64  -- binary64 storage and arithmetic in the order written above
 *                 (2 u[i] is exact; no other contraction).  Bit-identical to a
 *                 plain sequential evaluation.
 *   HEAT_FP32  -- binary32 storage and arithmetic: c + r*((q - c) - (c - l))
 *                 (the second difference as the difference of the two
 *                 one-sided differences; each is exact for neighbours within
 *                 a factor of 2).
 *   HEAT_FP32C -- binary32 storage; inside the kernels the state is the pair
 *                 (u, e) of binary32 numbers whose sum is the value, and r is
 *                 the pair rh + rl, rh = fl32(r), rl = fl32(r - rh).  With L
 *                 the Laplacian of u + e, formed as the difference of the
 *                 pair's one-sided fluxes ((q - c) + (eq - ec)) - ((c - l) +
 *                 (ec - el)), each step is t = fma(rh, L, c), res =
 *                 fma(rh, L, c - t) (the rounding error of t, taken with the
 *                 product unrounded), e' = fma(rl, L, res) + e, u' = t: the
 *                 increment's small parts gather in e (Kahan-style) instead
 *                 of being rounded away.  Steps are grouped into rounds of T
 *                 steps (T reported by heat_plan); at each round end the
 *                 state is folded to u := fl32(u + e).  Only u touches HBM.
 *
 * All functions are extern "C", thread-safe, never throw, and return one of
 * the heat_status codes.  After a negative return heat_last_error() gives a
 * thread-local message.  Pointers marked "device" must point to memory of
 * the current HIP device; "host" pointers to ordinary host memory.
 */
#ifndef HEAT_H
#define HEAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum heat_status {
    HEAT_OK = 0,
    HEAT_PENDING = 1,     /* heat_poll: request not finished yet                */
    HEAT_EINVAL = -1,     /* bad argument: NULL pointer, N < 1, nparts outside
                             [1, N], nt < 0, r not finite or outside [0, 1/2],
                             unknown precision, bad configuration             */
    HEAT_ENOMEM = -2,     /* device allocation failed, or a request's footprint
                             exceeds the server's whole HBM budget            */
    HEAT_EBUSY = -3,      /* server admission queue full: retry later         */
    HEAT_ENOENT = -4,     /* unknown or already consumed ticket               */
    HEAT_EDEVICE = -5,    /* HIP runtime error (message in heat_last_error)   */
    HEAT_ECANCELED = -6   /* request was cancelled                            */
};

enum heat_precision { HEAT_FP64 = 0, HEAT_FP32 = 1, HEAT_FP32C = 2 };

enum heat_kernel_choice {
    HEAT_KERNEL_AUTO = 0, /* planner decides (tuned table)                      */
    HEAT_KERNEL_STEP = 1, /* one step per launch: coalesced sweep, HBM bound    */
    HEAT_KERNEL_TB = 2,   /* temporal blocking: T steps per round in registers  */
    HEAT_KERNEL_RESIDENT = 3 /* temporal blocking in ONE launch: every tile (one
                               per workgroup) keeps its window in registers
                               for all nt steps and swaps its H edge cells
                               with its neighbour tiles through memory every T
                               steps, each value tagged with its exchange's
                               epoch (the segments' ghost-zone exchange of
                               Section 2, H cells deep).  Every tile must be resident at
                               once: the call fails with HEAT_EINVAL if the
                               ring needs more workgroups than the device
                               holds, and with HEAT_EDEVICE if a wait times
                               out (another launch holding the CUs).  Lone
                               waves need waves_per_group 1; the binary32
                               forms run in place (register_form 1).  The
                               call waits for its stream (to check the
                               waits).  Same results as HEAT_KERNEL_TB with
                               the same T.                                    */
};

/* How the waves of a workgroup share the work of a round (TB). */
enum heat_exchange {
    HEAT_EXCHANGE_AUTO = 0, /* planner decides (tuned table)                      */
    HEAT_EXCHANGE_NONE = 1, /* one tile per wavefront; windows overlap by the
                               halo only                                          */
    HEAT_EXCHANGE_LDS = 2,  /* one tile per workgroup: its waves hold adjacent
                               windows that overlap by 2S cells, S =
                               cells_per_lane / 4, and swap S edge cells through
                               LDS every S steps (a deep ghost-zone exchange
                               between segments, Section 2); needs
                               waves_per_group >= 2 and cells_per_lane >= 16    */
    HEAT_EXCHANGE_LDS_DEEP = 3 /* the same with S = cells_per_lane / 2: half as
                               many exchanges for twice the overlap; needs
                               waves_per_group >= 2 and cells_per_lane >= 8    */
};

/* Optional overrides for the planner; zero fields mean "choose". */
typedef struct heat_config {
    int32_t kernel;          /* heat_kernel_choice                              */
    int32_t cells_per_lane;  /* TB: cells held per lane, one of 8, 16, 32, 64   */
    int32_t steps_per_round; /* TB: T, a multiple of 4 with 2T < 64*cells - 8   */
    int32_t waves_per_group; /* wavefronts per workgroup, 1 to 8                */
    int32_t register_form;   /* TB: 1 = in-place forward sweeps (in binary64
                                the compiler rotates the K registers every
                                step; binary32 needs no copies),
                                2 = ping-pong (2K registers, no copies),
                                3 = alternating forward/backward in-place sweeps
                                (K + 1 registers, no copies).  HEAT_FP32C with
                                a binary32 coefficient, 32 cells per lane and
                                lone waves: 1 and 2 both run the ping-pong
                                sweep (measured faster there; same bits)      */
    int32_t exchange;        /* TB: heat_exchange                               */
} heat_config;

/* What the planner picked for a given problem (filled by heat_plan). */
typedef struct heat_plan_info {
    int32_t kernel;          /* HEAT_KERNEL_STEP, _TB or _RESIDENT              */
    int32_t cells_per_lane;  /* K (TB)                                          */
    int32_t steps_per_round; /* T: steps per round (1 for STEP; RESIDENT: steps
                                between edge exchanges)                        */
    int32_t waves_per_group;
    int32_t register_form;   /* 1 in-place, 2 ping-pong, 3 alternating (TB; the
                                form planned: heat_config names the one case
                                whose kernel sweeps in another)                */
    int32_t exchange_steps;  /* S: steps between LDS edge exchanges of the
                                waves of a tile (K/4 or K/2); 0 = one tile per
                                wave (TB)                                      */
    int64_t tile_cells;      /* W: output cells per tile (TB): 64*K - 2H for a
                                lone wave, G*64*K - (G-1)*2S - 2H for G waves,
                                H >= T the halo                                 */
    int64_t tiles;           /* tiles per round                                 */
    int64_t rounds;          /* launches (STEP: nt, TB: ceil(nt / T),
                                RESIDENT: 1)                                    */
} heat_plan_info;

/*
 * Plain form.  u: host array of N binary64 values, overwritten in place by
 * the state after nt steps.  FP64.  Blocking.  Copies to and from the current
 * device, allocates and frees its own device memory.  u may be pageable:
 * arrays of 64 MiB or more are copied through 8 lanes of pinned chunks (8
 * host threads; 128 MiB of pinned host memory, allocated on the first such
 * call per device and kept until the process ends); concurrent calls take
 * turns for those lanes.
 */
int heat_solve(double *u, int64_t N, int32_t nparts, double r, int64_t nt);

/*
 * Device form.  d_u: device array of N values (double* for HEAT_FP64, float*
 * for HEAT_FP32/HEAT_FP32C), aligned to its element size, advanced in place
 * (16-byte aligned arrays take the vector loads; any other alignment runs
 * every tile through the cell-by-cell path: same bits, slower).  Work is
 * queued on `hip_stream` (a hipStream_t; NULL = the legacy default stream).
 * Device scratch of the same size as d_u is taken from the stream-ordered
 * pool of the device.  If sum0_out / sum_out are not NULL they receive the
 * binary64 sums of the state before and after the run (the conservation
 * check, which holds up to rounding on a ring) and the call waits for the
 * stream; otherwise it returns as soon as the work is queued.
 */
int heat_solve_dev(void *d_u, int64_t N, int32_t nparts, double r, int64_t nt,
                   int32_t precision, void *hip_stream, double *sum0_out, double *sum_out);

/*
 * Device form that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation).  As heat_solve_dev with the planner's
 * default shape (the round kernel: a call of heat_solve_dev that waits may
 * take the resident kernel, same state bits, checksums equal up to the
 * rounding of their partial sums), except:
 *   - its scratch (the ping-pong state buffer and the checksum partials) is
 *     one static device array of HEAT_NOALLOC_SCRATCH_BYTES per device, held
 *     from the library's first use on that device until the process ends;
 *     a ring whose scratch (N * element size rounded up to 256 bytes, plus
 *     8 * max(4096, 2 * tiles) bytes when sums are asked for) does not fit
 *     is refused with HEAT_EINVAL -- for binary64 about 8.3 million cells,
 *     for the binary32 forms about 16.7 million;
 *   - d_sums_out: NULL, or a device array of 2 doubles that receives the
 *     binary64 sums of the state before and after the run, on the stream;
 *     the call never waits for the stream.
 * Every call on one device shares that device's array, and the array keeps
 * the last call's contents (every byte a call reads it has written first):
 * calls that overlap on one device -- on different streams or threads --
 * race and must be serialised by the caller.  No hipMalloc, hipFree or
 * other allocating call is made.
 */
#define HEAT_NOALLOC_SCRATCH_BYTES (64u << 20)
int heat_solve_dev_noalloc(void *d_u, int64_t N, int32_t nparts, double r, int64_t nt,
                           int32_t precision, void *hip_stream, double *d_sums_out);

/*
 * Device form with explicit configuration and scratch.  d_work: NULL, or a
 * caller-owned device array with room for N values of the storage type (not
 * overlapping d_u).  cfg: NULL or overrides.  Otherwise as heat_solve_dev.
 */
int heat_solve_dev_cfg(void *d_u, void *d_work, int64_t N, int32_t nparts, double r, int64_t nt,
                       int32_t precision, const heat_config *cfg, void *hip_stream,
                       double *sum0_out, double *sum_out);

/*
 * Planner: what heat_solve_dev_cfg would run for this problem, in a call that
 * asks for the sums.  With every heat_config field zero (or cfg NULL), calls
 * that wait for their result -- those asking for the sums, and heat_solve --
 * may take the resident kernel: the tuning table records up to six
 * resident shapes for N's quarter decade, each with its shortest winning run
 * and its gain over the round kernel at full SIMD load at three points of
 * the quarter decade (see heat_autotune_resident; both are taken linear in
 * log N between the points).  Each shape the run is long enough for is
 * fitted to N -- a CU holds ceil(tiles / CUs) workgroups
 * and every tile waits for the slowest, so for HEAT_FP64 and HEAT_FP32
 * (whose results do not depend on T) the exchange interval, from the tuned
 * T down to half of it, whose tiles put the fewest waves on the busiest SIMD
 * is taken -- and must fit the device at once; the shape whose gain at full
 * load at N times its load efficiency at N (mean over busiest waves per
 * SIMD) is the largest is taken if that is at least 1.03.  Other calls take the round kernel, with the same results.
 * No device work (it may query the device's occupancy).
 */
int heat_plan(int64_t N, int64_t nt, int32_t precision, const heat_config *cfg,
              heat_plan_info *out);

/*
 * binary64 sum of a device array (double* or float* by precision), computed
 * by a fixed-shape two-pass reduction (deterministic for a given N).  Waits
 * for `hip_stream`; result written to *sum_out (host).
 */
int heat_checksum_dev(const void *d_u, int64_t N, int32_t precision, void *hip_stream,
                      double *sum_out);

/* --------------------------------------------------------------- batching */

/*
 * One problem of a batch (host buffers).  u0 and u_out hold N binary64
 * values (u_out may equal u0).  FP32 forms round u0 to binary32 on the device
 * and widen the result back exactly.  sum0 / sum_nt: binary64 sums of the
 * state (in its storage precision) before and after; status: per-problem
 * heat_status.
 *
 * shift (FP32 forms; ignored for HEAT_FP64; must be finite): the device holds
 * the binary32 offsets v = fl32(u0 - shift) (difference taken in binary64,
 * rounded to nearest even) and the result is u = shift + v (binary64).  A
 * constant is a fixed point of the update (its Laplacian is zero), so in
 * exact arithmetic the offsets evolve exactly as the state does; stored
 * relative to a shift near the state's mean, binary32 resolves the
 * fluctuations instead of the mean (mean-shifted storage).  0 = no offset.
 * The sums then are N*shift + sum(v).
 */
typedef struct heat_problem {
    int64_t N;
    int32_t nparts;
    int32_t precision;
    double r;
    int64_t nt;
    const double *u0;
    double *u_out;
    double sum0;
    double sum_nt;
    int32_t status;
    int32_t reserved;
    double latency_s;   /* server: seconds from heat_submit to completion */
    double shift;       /* FP32 forms: state stored as binary32 offsets from it */
} heat_problem;

/*
 * Batching form (host buffers): validates every problem, copies them to the
 * device, advances all of them together (as heat_solve_batch_dev without
 * flags: one launch per round over the tiles of every still-running ring),
 * copies back.  Blocking.  Returns HEAT_OK if every problem succeeded, else the first
 * error; probs[i].status tells which.  Host arrays may be pageable; when
 * the problems' arrays add up to 64 MiB or more, the copies go through the
 * same pinned lanes as heat_solve's.
 */
int heat_solve_batch(heat_problem *probs, int32_t count);

/*
 * One ring of a device-resident batch.  d_u: device state (N values of the
 * precision's storage type, aligned to its element size), advanced in
 * place; d_work: device scratch of the same size.  The caller owns both.
 * Rings whose two arrays are both 16-byte aligned take the vector loads,
 * others the cell-by-cell path (same bits).
 */
typedef struct heat_ring {
    int64_t N;
    int64_t nt;
    double r;
    int32_t precision;
    int32_t nparts;
    void *d_u;
    void *d_work;
} heat_ring;

/* Flags of heat_solve_batch_dev. */
enum heat_batch_flags {
    HEAT_BATCH_WAIT = 1,       /* wait for completion and report kernel-side errors */
    HEAT_BATCH_PERSISTENT = 2, /* one persistent launch whose tiles synchronise through
                                  per-tile epoch counters instead of one launch per round
                                  (needs HEAT_BATCH_WAIT: a stalled wait is reported as
                                  HEAT_EDEVICE once the launch has drained) */
    HEAT_BATCH_GRAPH = 4       /* capture the per-round launches in a hipGraph and replay it
                                  (needs HEAT_BATCH_WAIT) */
};

/*
 * Device-resident batching form: every ring advances round by round.  Rings
 * fall into kernel classes by precision and length (32- or 64-cell lanes, or
 * for the longest rings tiles of 4 waves that swap edges through LDS); by
 * default each round of a class's still-running rings is one launch over the
 * flat list of their tiles (the kernel boundary is the round barrier).  Rings
 * are ordered by their number of rounds, so the running ones are a prefix of
 * their class's table.  A class may run longer rounds than heat_plan would,
 * which changes no binary64 or binary32 result, and the compensated form
 * keeps its fixed round length, so each ring's result is bit-identical to
 * solving it alone.  With HEAT_BATCH_PERSISTENT (32-cell lanes, one wave per
 * tile) all rounds of all rings run in a single launch:
 * tiles are claimed in round order from one counter and each waits for the
 * tiles within H cells of it to finish the previous round (agent-scope
 * release/acquire; a bounded wait turns a stall into HEAT_EDEVICE instead of
 * a hang).  Queued on hip_stream.
 */
int heat_solve_batch_dev(const heat_ring *rings, int32_t count, void *hip_stream, int32_t flags);

/* ---------------------------------------------------------------- serving */

typedef struct heat_server heat_server;

typedef struct heat_server_stats {
    uint64_t submitted, admitted, completed, cancelled, rejected;
    uint64_t ticks;            /* fused launches issued                       */
    uint64_t cell_updates;     /* total N * nt of completed requests          */
    size_t   hbm_budget;       /* bytes the server may hold on the device     */
    size_t   hbm_in_use;       /* bytes held now                              */
    size_t   hbm_peak;         /* high-water mark                             */
    int32_t  active;           /* requests resident on the device now         */
    int32_t  queued;           /* requests waiting for admission              */
} heat_server_stats;

/*
 * Create a continuous-batching server on the current device.  It owns one
 * device arena of hbm_budget_bytes (0 = 80 % of the free device memory), a
 * scheduler thread and its streams.  At most max_slots requests (0 = 4096)
 * are resident at once; max_queue (0 = 65536) may wait for admission.
 * Every scheduling step (tick) advances each resident request by 2 rounds;
 * the environment variable HEAT_SERVER_TICK_STEPS, read here, instead sizes
 * ticks in steps (each request advances the whole rounds that cover that
 * many steps).  Ticks never change a result.
 */
int heat_server_create(size_t hbm_budget_bytes, int32_t max_slots, int32_t max_queue,
                       heat_server **out);

/*
 * Submit a request (non-blocking).  *p, p->u0 and p->u_out must stay valid
 * and untouched until heat_poll returns something other than HEAT_PENDING
 * or heat_cancel returns.  Returns HEAT_EINVAL for a bad problem, HEAT_ENOMEM
 * if its footprint exceeds the whole budget (16 N bytes for binary64, 12 N
 * for the binary32 forms -- the state plus a binary64 staging buffer -- each
 * part rounded up to 256 bytes, plus 256), HEAT_EBUSY if the queue is full.
 * *ticket identifies the request.
 */
int heat_submit(heat_server *s, heat_problem *p, uint64_t *ticket);

/*
 * HEAT_PENDING while the request runs; HEAT_OK once p->u_out, p->sum0,
 * p->sum_nt and p->status are filled (the ticket is then consumed);
 * HEAT_ENOENT for an unknown or consumed ticket; another negative code if
 * the request failed.
 */
int heat_poll(heat_server *s, uint64_t ticket);

/* Block until the request is done (or failed); same returns as heat_poll.
 * Any thread may poll, wait on or cancel any ticket: the first call that
 * finds the request finished consumes the ticket, and a call that was
 * waiting on it meanwhile returns HEAT_ENOENT. */
int heat_wait(heat_server *s, uint64_t ticket);

/* Cancel a queued or running request; its ticket is consumed.  A request
 * already copying its result out completes first, and its status is still
 * set to HEAT_ECANCELED.  HEAT_ENOENT if another call consumed the ticket
 * while this one waited for the device to let go of the request. */
int heat_cancel(heat_server *s, uint64_t ticket);

int heat_server_get_stats(heat_server *s, heat_server_stats *out);

/* Cancel all outstanding work, stop the server's threads, free the arena.
 * No other call on this server may be running or follow. */
int heat_server_destroy(heat_server *s);

/* ---------------------------------------------------------------- tuning */

/*
 * Autotuner: times every temporal-blocking launch shape (cells per lane,
 * steps per round, wavefronts per workgroup, register form, lone or
 * LDS-exchanging waves) on a synthetic ring of N cells of the given
 * precision on the current device (HIP events over an even number of whole
 * rounds, at least 4 and at least 384 steps) and returns the fastest in
 * *best_out (host) with its rate in GCUP/s.  If `install` is nonzero the shape becomes the planner's
 * default for rings of N's decade (log10 bucket) in this process.  Shapes
 * never change binary64 or binary32 results; for HEAT_FP32C only shapes with
 * the form's fixed round length are tried, at a coefficient that is not a
 * binary32 number (r = 0.3; the others are timed at r = 1/4).  Allocates and
 * frees 2 * N * 8 bytes of device memory.  Blocking.
 */
int heat_autotune(int32_t precision, int64_t N, int32_t install, heat_config *best_out,
                  double *best_gcups);

/*
 * Resident-kernel autotuner for N's quarter decade [10^(q/4), 10^((q+1)/4)):
 * times every HEAT_KERNEL_RESIDENT shape over 1,024 steps at three points of
 * the quarter decade (its two ends and their geometric middle), each fitted
 * to the point as heat_plan fits it, against the round kernel the planner
 * runs (the tuning table's shape); coefficients as heat_autotune, HEAT_FP32C
 * also at r = 1/4 (whose kernel drops the coefficient's low part), the
 * smaller gain counting; each time the fastest of three calls that ask for
 * the sums and so wait, as the calls that take the resident kernel do.  Each shape's
 * gain at each point over its load efficiency there is its gain at full
 * load; heat_plan's model (that gain interpolated, times the load efficiency
 * at N) then picks a shape at each of 64 ring lengths spread over the
 * quarter decade, where one predicts a gain of at least 3 %.  `install`
 * records up to six shapes -- the fastest at each point where it gains at
 * least 3 %, then those the model picks most often (none clears the quarter
 * decade) -- each with its gain at full load at each point and, at each
 * point where it gains, the run length from which it is faster (from both
 * kernels' times over 128 and 1,024 steps, each taken as a fixed cost plus a
 * cost per step).
 * Calls that wait for their result then choose among them.  *best_out: the
 * first shape recorded (else the fastest at the lower end; all zero if none
 * can be resident); *min_steps_out: the largest run length recorded (0: none);
 * *gain_out: the smallest over the three points of the best gain measured
 * there, the round kernel's time over the resident time over 1,024 steps
 * (0 if some point fits no shape).  Any output may be NULL.  Allocates and
 * frees 2 * 10^((q+1)/4) * 8 bytes of device memory.  Blocking.
 */
int heat_autotune_resident(int32_t precision, int64_t N, int32_t install, heat_config *best_out,
                           int64_t *min_steps_out, double *gain_out);

/*
 * Batch autotuner: times every kernel class of the batching form (cells per
 * lane 32 or 64, one wave per tile or 4 waves sharing a tile through LDS,
 * as built for the precision) at every round length its window allows
 * (the compensated form: its fixed length only) on a synthetic batch of
 * rings whose lengths spread log-uniformly over N's decade (as many as hold
 * about 3e7 cells, at most 4,096; step counts spread over [100, 7,680];
 * one untimed and one timed pass, HIP events; 1 <= N < 1e8), beside the
 * batching form's own rule (each ring in the class its length suggests), and
 * returns the fastest class in *K_out, *G_out, *T_out with its rate in
 * GCUP/s (host pointers, any may be NULL) -- or K = G = T = 0 when no class
 * beats the rule by 3 % or more.  If `install` is nonzero, heat_solve_batch,
 * heat_solve_batch_dev and the server under load use that class (or the
 * rule) for rings of N's decade and precision in this process.  Classes
 * never change a result.
 * Allocates and frees about 2 * 3e7 * 8 bytes of device memory.  Blocking.
 */
int heat_autotune_batch(int32_t precision, int64_t N, int32_t install, int32_t *K_out,
                        int32_t *G_out, int32_t *T_out, double *best_gcups);

/*
 * Save / load the planner's tuning table as text (one line per precision and
 * decade: "precision bucket K T waves form exchange"; a line of six columns
 * loads as lone waves, exchange HEAT_EXCHANGE_NONE; batch classes picked by
 * heat_autotune_batch as lines "b precision bucket K G T", where K = G = T = 0
 * stands for the batching form's own rule).  A malformed line makes
 * heat_tune_load return HEAT_EINVAL and keeps the lines read before it.  The library also loads the
 * file named by the environment variable HEAT_TUNE_TABLE at first use.
 */
int heat_tune_save(const char *path);
int heat_tune_load(const char *path);

/* ------------------------------------------------------------------ misc */

/* Thread-local text for the last negative return on this thread. */
const char *heat_last_error(void);

/*
 * Plain streaming copy of `bytes` bytes (a multiple of 16, both pointers
 * 16-byte aligned) between two device buffers on hip_stream, with the same
 * launch shape as the one-step kernel.  It measures the HBM bandwidth a
 * read-once/write-once kernel reaches on this device, the ceiling the
 * one-step sweep is measured against.  Asynchronous.
 */
int heat_copy_dev(const void *d_src, void *d_dst, size_t bytes, void *hip_stream);

/* Library version string: "heat-mi355x <version> (gfx950) src <sha256>", the
 * last field the sha256 of the sources the library was built from (every
 * file of csrc/, this header and the build script), or "unknown" for a
 * build that did not supply it. */
const char *heat_version(void);

/*
 * Device facts the planner uses (host out-pointers, any may be NULL):
 * compute units, LDS bytes per workgroup, wavefront size, clock in kHz,
 * and total / free device memory in bytes.
 */
int heat_device_info(int32_t *cus, int32_t *lds_bytes, int32_t *wave_size, int32_t *clock_khz,
                     size_t *mem_total, size_t *mem_free);

#ifdef __cplusplus
}
#endif

#endif /* HEAT_H */
