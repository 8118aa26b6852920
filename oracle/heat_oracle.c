/*
 * heat_oracle.c -- CPU oracle for the periodic 1D heat stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline legs of the benchmark load it; the GPU
 * library never includes, links or calls it, and it shares no code with it.
 *
 * What it computes (paper, Section 2 "Model problem"):
 *   - Eq. (heat:discrete): one explicit-Euler step of the heat equation with a
 *     second-order central difference,
 *         u(t+dt, x_i) = u(t, x_i) + dt*alpha*(u_{i-1} - 2 u_i + u_{i+1}) / h^2,
 *     written here with r = alpha*dt/h^2.  The printed denominator is garbled
 *     (it reads "2h"); the consistent second-order Laplacian divides by h^2,
 *     and the caller passes r directly, so the reading only fixes what r means.
 *   - the periodic boundary condition u(t, x) = u(t, L + x): index i-1 of
 *     cell 0 is cell N-1, and index i+1 of cell N-1 is cell 0;
 *   - every right-hand-side value is taken at time t (Jacobi update: the
 *     new array is written from the old one, never in place);
 *   - the parallel algorithm of Section 2 (last paragraph): the grid is cut
 *     into contiguous segments, each one updated on its own after its ghost
 *     cells have been received from the two neighbouring segments.
 *
 * Arithmetic: IEEE binary64, round to nearest even, evaluated exactly in the
 * order written (build with -ffp-contract=off, no -ffast-math):
 *         new = c + r * ((l - 2.0 * c) + q)
 * 2.0*c is exact, so (l - 2.0*c) + q is the left-to-right reading of the
 * paper's numerator.
 *
 * The FP32 forms are not in the paper (it computes in binary64); they are the
 * reduced-precision forms of the same update that the GPU library offers.
 * Their second difference is written as the difference of the two one-sided
 * differences (the flux form of the numerator of Eq. (heat:discrete)):
 *   - plain FP32:  new = c + r * ((q - c) - (c - l))   (all in binary32)
 *   - compensated FP32: the state is the unevaluated sum u + e of two binary32
 *     numbers, and the coefficient is the unevaluated sum rh + rl of two
 *     binary32 numbers, rh = fl32(r), rl = fl32(r - rh) (the difference taken
 *     in binary64, where it is exact), so r is carried to about 2^-48
 *     relative instead of 2^-25.  The Laplacian of u + e is the difference
 *     of the pair's one-sided fluxes (flux form again).  One step is
 *         L   = ((q - c) + (eq - ec)) - ((c - l) + (ec - el))
 *         t   = fma(rh, L, c)
 *         res = fma(rh, L, c - t)   (the rounding error of t, c + rh*L - t,
 *                                    rounded once; c - t is exact when t
 *                                    and c are within a factor 2)
 *         e'  = fma(rl, L, res) + ec
 *         u'  = t
 *     where fma is the binary32 fused multiply-add (one rounding).  So
 *     u' + e' = (u + e) + (rh + rl) * L up to the roundings of L and of the
 *     small terms: the increment's small parts -- the coefficient's low part
 *     and the rounding of c + rh*L -- gather in e instead of being rounded
 *     away.  Steps are grouped into rounds of T steps; at the end of every
 *     round (and at the end of the run) u := fl32(u + e), e := 0.
 *
 * heat_oracle_solve_threads runs the segments as the paper's CPU codes do,
 * one thread each; heat_oracle_solve_threads_simd is the same with the
 * segment sweep vectorised (heat_cpu_simd.c, bit-identical).
 *
 * Error behaviour: no argument checks beyond what is needed not to crash
 * (N < 1 or nt < 0 do nothing); r is NOT range-checked, so unstable r can be
 * exercised as a negative control.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* One Jacobi step over the whole ring (Eq. heat:discrete + periodic BC). */
static void step_ring_f64(const double *a, double *b, int64_t N, double r)
{
    for (int64_t i = 0; i < N; ++i) {
        double l = a[(i - 1 + N) % N];
        double c = a[i];
        double q = a[(i + 1) % N];
        b[i] = c + r * ((l - 2.0 * c) + q);
    }
}

/* Unpartitioned solver: nt steps of Eq. (heat:discrete) on the ring. */
void heat_oracle_solve(const double *u0, double *out, int64_t N, double r, int64_t nt)
{
    if (N < 1) return;
    double *a = (double *)malloc((size_t)N * sizeof(double));
    double *b = (double *)malloc((size_t)N * sizeof(double));
    memcpy(a, u0, (size_t)N * sizeof(double));
    for (int64_t n = 0; n < nt; ++n) {
        step_ring_f64(a, b, N, r);
        double *t = a; a = b; b = t;
    }
    memcpy(out, a, (size_t)N * sizeof(double));
    free(a);
    free(b);
}

/*
 * Partitioned solver (Section 2, last paragraph): nparts contiguous segments,
 * segment p = [floor(p*N/P), floor((p+1)*N/P)).  Each segment keeps its own
 * array with one ghost cell on each side.  Every step first exchanges ghost
 * zones (segment p receives the last cell of p-1 and the first cell of p+1,
 * both taken mod P), then every segment applies the update to its own cells.
 * The result must equal the unpartitioned solver exactly.
 */
void heat_oracle_solve_parts(const double *u0, double *out, int64_t N, int64_t nparts,
                             double r, int64_t nt)
{
    if (N < 1 || nparts < 1 || nparts > N) return;
    int64_t P = nparts;
    int64_t *start = (int64_t *)malloc((size_t)(P + 1) * sizeof(int64_t));
    for (int64_t p = 0; p <= P; ++p) start[p] = (p * N) / P;
    double **seg = (double **)malloc((size_t)P * sizeof(double *));
    double **nxt = (double **)malloc((size_t)P * sizeof(double *));
    for (int64_t p = 0; p < P; ++p) {
        int64_t len = start[p + 1] - start[p];
        seg[p] = (double *)malloc((size_t)(len + 2) * sizeof(double));
        nxt[p] = (double *)malloc((size_t)(len + 2) * sizeof(double));
        memcpy(seg[p] + 1, u0 + start[p], (size_t)len * sizeof(double));
    }
    for (int64_t n = 0; n < nt; ++n) {
        /* ghost exchange: every value comes from the state at step n */
        for (int64_t p = 0; p < P; ++p) {
            int64_t pl = (p - 1 + P) % P, pr = (p + 1) % P;
            int64_t len_l = start[pl + 1] - start[pl];
            seg[p][0] = seg[pl][len_l];          /* last interior cell of p-1 */
            int64_t len = start[p + 1] - start[p];
            seg[p][len + 1] = seg[pr][1];        /* first interior cell of p+1 */
        }
        /* local sweeps */
        for (int64_t p = 0; p < P; ++p) {
            int64_t len = start[p + 1] - start[p];
            const double *a = seg[p];
            double *b = nxt[p];
            for (int64_t j = 1; j <= len; ++j) {
                double l = a[j - 1], c = a[j], q = a[j + 1];
                b[j] = c + r * ((l - 2.0 * c) + q);
            }
        }
        double **t = seg; seg = nxt; nxt = t;
    }
    for (int64_t p = 0; p < P; ++p) {
        int64_t len = start[p + 1] - start[p];
        memcpy(out + start[p], seg[p] + 1, (size_t)len * sizeof(double));
        free(seg[p]);
        free(nxt[p]);
    }
    free(seg);
    free(nxt);
    free(start);
}

/*
 * Threaded partitioned solver: the parallel algorithm of Section 2 as the
 * paper runs it on a CPU.  One thread per segment applies the update to its
 * own segment, step after step; ghost cells travel between neighbouring
 * segments through single-producer single-consumer queues (a mutex and a
 * condition variable guard each queue, as in the paper's hand-written C++17
 * queue).  Segment p pushes its last cell to p+1 (which uses it as its left
 * ghost) and its first cell to p-1 (its right ghost), then pops its own two
 * ghosts.  Every queue is FIFO, so a ghost popped at step n is the
 * neighbour's value at step n however far the threads drift apart, and the
 * result equals heat_oracle_solve exactly.
 *
 * Each thread allocates and fills its own segment (first touch on its own
 * NUMA node).  A start gate holds every thread until all have allocated, so
 * a failed allocation or thread creation aborts them all before any queue is
 * used.  Returns 0, -1 for bad arguments (N < 1, nparts outside
 * [1, min(N, 4096)], nt < 0), -2 if memory or a thread could not be had.
 */
#define GHOST_QUEUE_CAP 4

typedef struct {
    pthread_mutex_t m;
    pthread_cond_t cv;
    double slot[GHOST_QUEUE_CAP];
    int64_t pushed, popped;
} ghost_queue;

static void ghost_push(ghost_queue *q, double v)
{
    pthread_mutex_lock(&q->m);
    while (q->pushed - q->popped == GHOST_QUEUE_CAP) pthread_cond_wait(&q->cv, &q->m);
    q->slot[q->pushed % GHOST_QUEUE_CAP] = v;
    q->pushed++;
    pthread_cond_broadcast(&q->cv);
    pthread_mutex_unlock(&q->m);
}

static double ghost_pop(ghost_queue *q)
{
    pthread_mutex_lock(&q->m);
    while (q->pushed == q->popped) pthread_cond_wait(&q->cv, &q->m);
    double v = q->slot[q->popped % GHOST_QUEUE_CAP];
    q->popped++;
    pthread_cond_broadcast(&q->cv);
    pthread_mutex_unlock(&q->m);
    return v;
}

typedef struct {
    pthread_mutex_t m;
    pthread_cond_t cv;
    int64_t ready;  /* threads that finished allocating (successfully or not) */
    int failed;     /* some thread could not allocate, or a thread was not created */
    int state;      /* 0 wait, 1 run, -1 abort */
} start_gate;

/* One step of a segment: b[1..len] from a[0..len+1] (a[0], a[len+1] are the
 * ghost cells).  The scalar sweep is written below; heat_cpu_simd.c holds the
 * same sweep vectorised (bit-identical, see there). */
typedef void (*segment_sweep)(const double *a, double *b, int64_t len, double r);

static void sweep_scalar(const double *a, double *b, int64_t len, double r)
{
    for (int64_t j = 1; j <= len; ++j) {
        double l = a[j - 1], c = a[j], q = a[j + 1];
        b[j] = c + r * ((l - 2.0 * c) + q);
    }
}

void heat_cpu_sweep_simd(const double *a, double *b, int64_t len, double r);

typedef struct {
    const double *u0;
    double *out;
    int64_t start, len, nt;
    double r;
    segment_sweep sweep;
    ghost_queue *from_left, *from_right;  /* my ghosts arrive here */
    ghost_queue *to_right, *to_left;      /* my edge cells leave here */
    start_gate *gate;
} segment_task;

static void *segment_worker(void *arg)
{
    segment_task *t = (segment_task *)arg;
    int64_t len = t->len;
    double *a = (double *)malloc((size_t)(len + 2) * sizeof(double));
    double *b = (double *)malloc((size_t)(len + 2) * sizeof(double));
    if (a) memcpy(a + 1, t->u0 + t->start, (size_t)len * sizeof(double));

    start_gate *g = t->gate;
    pthread_mutex_lock(&g->m);
    if (!a || !b) g->failed = 1;
    g->ready++;
    pthread_cond_broadcast(&g->cv);
    while (g->state == 0) pthread_cond_wait(&g->cv, &g->m);
    int run = g->state == 1;
    pthread_mutex_unlock(&g->m);

    if (run) {
        double r = t->r;
        for (int64_t n = 0; n < t->nt; ++n) {
            ghost_push(t->to_right, a[len]);
            ghost_push(t->to_left, a[1]);
            a[0] = ghost_pop(t->from_left);
            a[len + 1] = ghost_pop(t->from_right);
            t->sweep(a, b, len, r);
            double *s = a; a = b; b = s;
        }
        memcpy(t->out + t->start, a + 1, (size_t)len * sizeof(double));
    }
    free(a);
    free(b);
    return NULL;
}

static int solve_threads_with(const double *u0, double *out, int64_t N, int64_t nparts,
                              double r, int64_t nt, segment_sweep sweep)
{
    if (N < 1 || nparts < 1 || nparts > N || nparts > 4096 || nt < 0) return -1;
    int64_t P = nparts;
    ghost_queue *from_left = (ghost_queue *)calloc((size_t)P, sizeof(ghost_queue));
    ghost_queue *from_right = (ghost_queue *)calloc((size_t)P, sizeof(ghost_queue));
    segment_task *task = (segment_task *)calloc((size_t)P, sizeof(segment_task));
    pthread_t *tid = (pthread_t *)calloc((size_t)P, sizeof(pthread_t));
    if (!from_left || !from_right || !task || !tid) {
        free(from_left); free(from_right); free(task); free(tid);
        return -2;
    }
    start_gate gate;
    pthread_mutex_init(&gate.m, NULL);
    pthread_cond_init(&gate.cv, NULL);
    gate.ready = 0;
    gate.failed = 0;
    gate.state = 0;
    for (int64_t p = 0; p < P; ++p) {
        pthread_mutex_init(&from_left[p].m, NULL);
        pthread_cond_init(&from_left[p].cv, NULL);
        pthread_mutex_init(&from_right[p].m, NULL);
        pthread_cond_init(&from_right[p].cv, NULL);
    }
    for (int64_t p = 0; p < P; ++p) {
        segment_task *t = &task[p];
        t->u0 = u0;
        t->out = out;
        t->start = (p * N) / P;
        t->len = ((p + 1) * N) / P - t->start;
        t->nt = nt;
        t->r = r;
        t->sweep = sweep;
        t->from_left = &from_left[p];
        t->from_right = &from_right[p];
        t->to_right = &from_left[(p + 1) % P];
        t->to_left = &from_right[(p - 1 + P) % P];
        t->gate = &gate;
    }
    int64_t created = 0;
    while (created < P && pthread_create(&tid[created], NULL, segment_worker, &task[created]) == 0)
        ++created;

    pthread_mutex_lock(&gate.m);
    if (created < P) gate.failed = 1;
    while (gate.ready < created) pthread_cond_wait(&gate.cv, &gate.m);
    int ok = !gate.failed;
    gate.state = ok ? 1 : -1;
    pthread_cond_broadcast(&gate.cv);
    pthread_mutex_unlock(&gate.m);
    for (int64_t p = 0; p < created; ++p) pthread_join(tid[p], NULL);

    for (int64_t p = 0; p < P; ++p) {
        pthread_mutex_destroy(&from_left[p].m);
        pthread_cond_destroy(&from_left[p].cv);
        pthread_mutex_destroy(&from_right[p].m);
        pthread_cond_destroy(&from_right[p].cv);
    }
    pthread_mutex_destroy(&gate.m);
    pthread_cond_destroy(&gate.cv);
    free(from_left); free(from_right); free(task); free(tid);
    return ok ? 0 : -2;
}

int heat_oracle_solve_threads(const double *u0, double *out, int64_t N, int64_t nparts,
                              double r, int64_t nt)
{
    return solve_threads_with(u0, out, N, nparts, r, nt, sweep_scalar);
}

/* The same method with the vectorised segment sweep (heat_cpu_simd.c). */
int heat_oracle_solve_threads_simd(const double *u0, double *out, int64_t N, int64_t nparts,
                                   double r, int64_t nt)
{
    return solve_threads_with(u0, out, N, nparts, r, nt, heat_cpu_sweep_simd);
}

/*
 * Light cone of one cell: w holds the 2*nt+1 initial values centred on the
 * cell (taken around the ring, so they may repeat when N <= 2*nt).  After s
 * steps only the cells [s, 2*nt - s] of the window are still exact; each is
 * computed with the very same operations as in the full ring, so the centre
 * after nt steps is bit-identical to that cell of heat_oracle_solve.
 */
double heat_oracle_cone(const double *w, int64_t nt, double r)
{
    int64_t len = 2 * nt + 1;
    double *a = (double *)malloc((size_t)len * sizeof(double));
    double *b = (double *)malloc((size_t)len * sizeof(double));
    memcpy(a, w, (size_t)len * sizeof(double));
    for (int64_t s = 1; s <= nt; ++s) {
        for (int64_t j = s; j <= len - 1 - s; ++j) {
            double l = a[j - 1], c = a[j], q = a[j + 1];
            b[j] = c + r * ((l - 2.0 * c) + q);
        }
        double *t = a; a = b; b = t;
    }
    double v = a[nt];
    free(a);
    free(b);
    return v;
}

/* ---------------------------------------------------------------- FP32 */

void heat_oracle_solve_f32(const float *u0, float *out, int64_t N, float r, int64_t nt)
{
    if (N < 1) return;
    float *a = (float *)malloc((size_t)N * sizeof(float));
    float *b = (float *)malloc((size_t)N * sizeof(float));
    memcpy(a, u0, (size_t)N * sizeof(float));
    for (int64_t n = 0; n < nt; ++n) {
        for (int64_t i = 0; i < N; ++i) {
            float l = a[(i - 1 + N) % N];
            float c = a[i];
            float q = a[(i + 1) % N];
            b[i] = c + r * ((q - c) - (c - l));
        }
        float *t = a; a = b; b = t;
    }
    memcpy(out, a, (size_t)N * sizeof(float));
    free(a);
    free(b);
}

float heat_oracle_cone_f32(const float *w, int64_t nt, float r)
{
    int64_t len = 2 * nt + 1;
    float *a = (float *)malloc((size_t)len * sizeof(float));
    float *b = (float *)malloc((size_t)len * sizeof(float));
    memcpy(a, w, (size_t)len * sizeof(float));
    for (int64_t s = 1; s <= nt; ++s) {
        for (int64_t j = s; j <= len - 1 - s; ++j) {
            float l = a[j - 1], c = a[j], q = a[j + 1];
            b[j] = c + r * ((q - c) - (c - l));
        }
        float *t = a; a = b; b = t;
    }
    float v = a[nt];
    free(a);
    free(b);
    return v;
}

/* ------------------------------------------------------ compensated FP32 */

/* The coefficient as two binary32 numbers: rh = fl32(r), rl = fl32(r - rh). */
static void split_r(double r, float *rh, float *rl)
{
    *rh = (float)r;
    *rl = (float)(r - (double)*rh);
}

/* One compensated step of a cell: updates (*un, *en) from its values and
 * its neighbours' (u and e at the old time level). */
static void comp_cell(float l, float c, float q, float el, float ec, float eq, float rh,
                      float rl, float *un, float *en)
{
    float L = ((q - c) + (eq - ec)) - ((c - l) + (ec - el));
    float t = fmaf(rh, L, c);
    float res = fmaf(rh, L, c - t);
    *en = fmaf(rl, L, res) + ec;
    *un = t;
}

/* One compensated step of the pair (u, e) on the ring. */
static void step_ring_f32c(const float *u, const float *e, float *un, float *en,
                           int64_t N, float rh, float rl)
{
    for (int64_t i = 0; i < N; ++i) {
        int64_t il = (i - 1 + N) % N, iq = (i + 1) % N;
        comp_cell(u[il], u[i], u[iq], e[il], e[i], e[iq], rh, rl, &un[i], &en[i]);
    }
}

/*
 * Compensated FP32 over nt steps in rounds of T steps (T >= 1; the last round
 * may be shorter).  At every round end u := fl32(u + e) and e := 0.  If
 * e_out is not NULL the run stops short of the final fold: out receives u and
 * e_out receives e of the last round, so that the unrounded pair can be
 * inspected.
 */
void heat_oracle_solve_f32c(const float *u0, float *out, float *e_out, int64_t N, double r,
                            int64_t nt, int64_t T)
{
    if (N < 1) return;
    if (T < 1) T = 1;
    float rh, rl;
    split_r(r, &rh, &rl);
    float *u = (float *)malloc((size_t)N * sizeof(float));
    float *e = (float *)calloc((size_t)N, sizeof(float));
    float *un = (float *)malloc((size_t)N * sizeof(float));
    float *en = (float *)malloc((size_t)N * sizeof(float));
    memcpy(u, u0, (size_t)N * sizeof(float));
    int64_t done = 0;
    while (done < nt) {
        int64_t s = nt - done < T ? nt - done : T;
        for (int64_t i = 0; i < N; ++i) e[i] = 0.0f;
        for (int64_t k = 0; k < s; ++k) {
            step_ring_f32c(u, e, un, en, N, rh, rl);
            float *t1 = u; u = un; un = t1;
            float *t2 = e; e = en; en = t2;
        }
        done += s;
        if (done < nt || e_out == NULL)
            for (int64_t i = 0; i < N; ++i) u[i] = u[i] + e[i];
    }
    memcpy(out, u, (size_t)N * sizeof(float));
    if (e_out) {
        if (nt > 0) memcpy(e_out, e, (size_t)N * sizeof(float));
        else memset(e_out, 0, (size_t)N * sizeof(float));
    }
    free(u); free(e); free(un); free(en);
}

/*
 * Light cone of one cell for the compensated form: w holds the 2*nt+1 initial
 * binary32 values centred on the cell.  Rounds of T steps as above; the fold
 * u := fl32(u + e) is applied to every still-exact cell of the window.
 */
float heat_oracle_cone_f32c(const float *w, int64_t nt, double r, int64_t T)
{
    if (T < 1) T = 1;
    float rh, rl;
    split_r(r, &rh, &rl);
    int64_t len = 2 * nt + 1;
    float *u = (float *)malloc((size_t)len * sizeof(float));
    float *e = (float *)calloc((size_t)len, sizeof(float));
    float *un = (float *)malloc((size_t)len * sizeof(float));
    float *en = (float *)malloc((size_t)len * sizeof(float));
    memcpy(u, w, (size_t)len * sizeof(float));
    int64_t s = 0;
    while (s < nt) {
        int64_t rs = nt - s < T ? nt - s : T;
        for (int64_t j = 0; j < len; ++j) e[j] = 0.0f;
        for (int64_t k = 0; k < rs; ++k) {
            ++s;
            for (int64_t j = s; j <= len - 1 - s; ++j)
                comp_cell(u[j - 1], u[j], u[j + 1], e[j - 1], e[j], e[j + 1], rh, rl, &un[j],
                          &en[j]);
            float *t1 = u; u = un; un = t1;
            float *t2 = e; e = en; en = t2;
        }
        for (int64_t j = s; j <= len - 1 - s; ++j) u[j] = u[j] + e[j];
    }
    float v = u[nt];
    free(u); free(e); free(un); free(en);
    return v;
}
