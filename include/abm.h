/*
 * abm.h -- C ABI of the MI355X (gfx950) fractional Adams-Bashforth-Moulton
 * history-sum library (libabm.so).
 *
 * The method (Bonchis, Kaslik, Rosu, arXiv 1710.01133, Section 2): for a
 * Caputo system D^alpha y = f(t, y), y(0) = x0 (and y'(0) = x1 when
 * 1 < alpha <= 2: the ceil(alpha) initial values of eq. fde), on the grid
 * t_n = n h, step s = n+1 computes
 *   predictor  yP_s = T(t_s) + h^alpha * sum_{k=0..n} b_{n-k} f_k                (eq. abm)
 *   corrector  y_s  = T(t_s) + h^alpha * ( c_n f_0 + sum_{k=1..n} a_{n-k} f_k
 *                                        + f(t_s, yP_s) / Gamma(alpha+2) )
 * with T(t) = x0 (alpha <= 1) or x0 + t x1 (alpha > 1) the Taylor sum of
 * eq. abm, f_k = f(t_k, y_k), b, a, c the product-rectangle /
 * product-trapezoid weights given right after eq. abm (b with a minus sign
 * between its two powers) and one corrector evaluation per step.  Systems are
 * handled component by component; an incommensurate system (eq. sys.LRC with
 * alpha_1 != alpha_2) gives each component the scheme of its own order.  The
 * O(N^2) history sums are the work this library does on the GPU.
 *
 * Conventions for every entry point:
 *  - Return value is an abm_status: 0 on success, a negative code otherwise.
 *    No exception or process exit crosses this boundary.  abm_last_error()
 *    gives a thread-local text describing the most recent failure.
 *  - "device pointer" means memory of the context's GPU (hipMalloc or a torch
 *    tensor's data_ptr()); the caller owns it and the library never frees it.
 *  - Work is enqueued on the context's HIP stream and the call returns; the
 *    caller synchronises that stream before reading outputs (abm_submit /
 *    abm_poll are the exception: they run on the library's own server thread).
 *  - Every floating-point value on the path is IEEE double except the
 *    far-field products when a reduced far_prec is chosen (see abm_prec).
 */
#ifndef ABM_H
#define ABM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t abm_status;
#define ABM_OK 0
#define ABM_EINVAL -1    /* invalid argument (message in abm_last_error) */
#define ABM_ENOMEM -2    /* device allocation failed, or request larger than the arena */
#define ABM_EDEVICE -3   /* a HIP call failed, a device-side wait timed out, or the state became non-finite */
#define ABM_EAGAIN -4    /* not finished yet (abm_poll) */
#define ABM_ENOENT -5    /* unknown ticket */
#define ABM_ECANCELED -6 /* request cancelled before completion */

/* Right-hand sides f(t, y) (the problem of eq. fde with f from a fixed set). */
enum abm_rhs {
    ABM_RHS_LINEAR = 0,  /* d=1: f = -lambda y;                         p = {lambda} */
    ABM_RHS_DUFFING = 1, /* d=2: f = (y2, -delta y2 - y1 - y1^3 + A cos(omega t)); p = {delta, A, omega} */
    ABM_RHS_LORENZ = 2,  /* d=3: f = (s(y2-y1), y1(r-y3)-y2, y1 y2 - b y3);   p = {s, r, b} */
    ABM_RHS_POLY = 3,    /* d=1: f = c0 + c1 t;                          p = {c0, c1} */
    ABM_RHS_LCR = 4,     /* d=2: forced LCR circuit of eq. sys.LRC:
                            f = (y2 - g(y1), -sigma y2 - y1 + F sin(omega t)),
                            g(x) = b x - a + b (x <= -1), a x (|x| < 1), b x + a - b (x >= 1);
                            p = {sigma, omega, a, b, F} */
    ABM_RHS_DIAG = 5     /* d=2: two uncoupled equations, a test system for per-component
                            orders: f = (-l1 y1 + m1, -l2 y2 + m2);  p = {l1, l2, m1, m2} */
};

/* Precision of the far-field history products of abm_solve_batch.  The near
 * band, the weight generation and the predictor/corrector state are always
 * double.  Reduced floating-point modes round F and the weights once to the
 * stated type, accumulate in float inside one K-tile and add tile partials in
 * double; the integer mode accumulates exactly and adds per-block partials in
 * double. */
enum abm_prec {
    ABM_FAR_FP64 = 0,   /* double products, double accumulation */
    ABM_FAR_FP32 = 1,   /* float products (MFMA f32), float accumulation per tile */
    ABM_FAR_BF16X3 = 2, /* two-term bf16 split (hi+lo) of both operands, 3 products */
    ABM_FAR_BF16X6 = 3, /* three-term bf16 split (hi+mid+lo), 6 products */
    ABM_FAR_FP16X3 = 4, /* two-term fp16 split (hi+lo) of operands scaled by powers of two
                           (history per 32 rows and column, weights per window), 3 products */
    ABM_FAR_DD = 5,     /* double-double (about 106 significant bits) for everything: weights,
                           Gamma(alpha+1), Gamma(alpha+2), h^alpha, t_s, the right-hand side,
                           history, sums and state -- the counterpart of the paper's
                           long-double runs.  Plain path only (abm_plan with B = 1, abm_solve);
                           y_out holds 2d doubles per state, the (hi, lo) pair of each
                           component, value hi + lo */
    ABM_FAR_I8 = 6      /* integer limbs on the int8 matrix cores: each weight window scaled by
                           a power of two and cut into four balanced base-256 int8 digits (30
                           bits), the history per block of L rows and column into three (22
                           bits); the nine digit products whose weight is at least 2^-24 of
                           the leading one, summed exactly in int32 over each block of history
                           rows and converted to double once per block.  Block lengths 128 and
                           256 only */
};

typedef struct abm_problem {
    int32_t rhs;        /* enum abm_rhs */
    int32_t d;          /* state dimension; must equal the rhs dimension */
    double alpha;       /* order of every component, 0 < alpha <= 2 (unless alphas[0] > 0) */
    double h;           /* step, > 0 and finite; t_s = (double)s * h */
    int64_t N;          /* number of steps, >= 1 */
    double x0[4];       /* y(0) (first d entries used) */
    double p[8];        /* rhs parameters, see enum abm_rhs */
    int32_t far_prec;   /* enum abm_prec (abm_solve_batch only) */
    int32_t out_stride; /* 0: write y_N only; k>0: write y_s for s = 0, k, 2k, ... and y_N */
    double alphas[4];   /* incommensurate orders: if alphas[0] > 0, component i has order
                           alphas[i] (first d entries, each in (0, 2]) and alpha is not read */
    double x1[4];       /* y'(0) (first d entries), read for components of order above 1 */
} abm_problem;

typedef struct abm_stats {
    int32_t block_L;      /* near-band block length used by abm_solve_batch */
    int32_t n_groups;     /* trajectory groups sharing one weight table */
    int64_t history_macs; /* sum over trajectories of d*N*(N+1)/2 */
    int64_t far_macs;     /* multiply-adds issued by the far-field kernels (useful ones) */
    int32_t far_launches; /* far-field kernel launches enqueued */
    int32_t chain_launches;
    double far_ms;        /* summed device time of the far-field launches (timing on, else 0) */
    double chain_ms;      /* summed device time of the chain launches (timing on, else 0) */
    int32_t narrow_groups; /* groups of at most a few columns whose far field runs as a
                              blocked convolution instead of column tiles */
    int32_t reserved_;
} abm_stats;

typedef struct abm_result {
    abm_status status;    /* ABM_OK; ABM_EDEVICE: a state of this request became non-finite
                             (the chains raise a status word of the request's own, so its
                             batch-mates are not affected), or the server stopped after a
                             device error; ABM_ENOMEM: larger than the arena; ABM_ECANCELED */
    double t_submit;      /* seconds, library monotonic clock, when abm_submit accepted it */
    double t_start;       /* when its first kernel was enqueued */
    double t_done;        /* when its completion was observed */
    double max_abs_y;     /* max |y_N| over the components of the final state */
} abm_result;

/* Blocking of the batched method.  A zero field takes the default (or the
 * ABM_BLOCK_L / ABM_KCHUNK / ABM_MAX_SPLIT / ABM_NARROW environment override). */
typedef struct abm_tuning {
    int32_t block_L;            /* near-band block length: 64 (double far field only), 128, 256, 512 */
    int32_t kchunk;             /* history rows per far-field chunk: a multiple of 512 (lowered
                                   until the chunk's weight window fits the LDS) */
    int32_t max_split;          /* most far-field workgroups along the history per column tile */
    int32_t column_tiles_only;  /* 1: no blocked convolution for narrow groups */
} abm_tuning;

/* One configuration tried by abm_autotune and the device time of one solve
 * with it (status != ABM_OK if the plan or the solve failed). */
typedef struct abm_tune_trial {
    abm_tuning cfg;
    abm_status status;
    int32_t reserved_;
    double ms;
} abm_tune_trial;

typedef struct abm_ctx abm_ctx;
typedef struct abm_plan_s abm_plan_t;

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  arena_bytes sizes the device
 * memory pool of the serving loop (abm_submit); 0 means 1 GiB.
 * Errors: ABM_EINVAL (bad device), ABM_ENOMEM, ABM_EDEVICE. */
abm_status abm_ctx_create(int device, void *hip_stream, size_t arena_bytes, abm_ctx **out);
/* Stops the context's server (cancelling queued requests, letting running
 * ones finish) and frees it, with every request not yet collected by
 * abm_poll.  Every plan made on the context must be destroyed before: a plan
 * keeps a pointer to its context.  No other thread may be inside a call on
 * this context meanwhile. */
void abm_ctx_destroy(abm_ctx *ctx);

/* Validate and size B problems, allocate their device state, generate their
 * weight tables on the device (Section 2 weights, cancellation-free double
 * evaluation) and choose the block length and tiles.  The plan fixes, per
 * trajectory, rhs, d, the orders, N, far_prec and out_stride; later solves
 * may change x0, x1, p and h.  Components of equal order share one weight
 * table.  Trajectories whose components have different orders are grouped
 * by their order tuple; their far field runs once per component with that
 * component's table. 
 * Errors: ABM_EINVAL (any invalid problem; the message names its index),
 * ABM_ENOMEM, ABM_EDEVICE. */
abm_status abm_plan(abm_ctx *ctx, const abm_problem *probs, int32_t B, abm_plan_t **out);
void abm_plan_destroy(abm_plan_t *plan);

/* abm_plan with an explicit blocking (tune may be NULL: defaults).  The
 * blocked method's results depend on the blocking only through rounding.
 * Errors: as abm_plan; ABM_EINVAL for a block length or chunk out of range. */
abm_status abm_plan_tuned(abm_ctx *ctx, const abm_problem *probs, int32_t B,
                          const abm_tuning *tune, abm_plan_t **out);

/* The blocking a plan uses (after defaults, overrides and the LDS limit). */
abm_status abm_plan_config(abm_plan_t *plan, abm_tuning *out);

/* Choose the blocking for these problems by timing whole abm_solve_batch
 * runs on the device (the batched method's launch sequence, block lengths,
 * chunk sizes and split counts interact through the overlap of far field and
 * chain, so candidates are measured, not modelled): every block length
 * first, then the split count and the chunk at the best one, then column
 * tiles instead of the blocked convolution if the problems have narrow
 * groups.  Stops starting new trials once budget_s seconds have passed (the
 * block-length stage always runs at least one).  Device memory for one plan
 * at a time plus scratch outputs.  best receives the fastest configuration,
 * where a trial replaces an earlier, slower one only if it is more than 2%
 * faster (so that run-to-run noise does not decide); trials (may be NULL)
 * receives up to max_trials of the trials made, in
 * order, and n_trials their count.  Synchronises the context's stream.
 * Errors: ABM_EINVAL, ABM_EDEVICE (no configuration could be run). */
abm_status abm_autotune(abm_ctx *ctx, const abm_problem *probs, int32_t B, double budget_s,
                        abm_tuning *best, abm_tune_trial *trials, int32_t max_trials,
                        int32_t *n_trials);

/* One trajectory (problem 0 of a plan made with B = 1) by the plain per-step
 * method: every step's two history sums are split over workgroups that each
 * own a fixed slice of the history, reduced across the grid, and the
 * predictor/corrector update is taken redundantly by every workgroup (the
 * partition and single reduction per step of Algorithm 1, with the per-node
 * reduction of Algorithm 2 done by wavefronts).
 * y_out: device pointer to n_out*d doubles, n_out = 1 (stride 0) or
 * N/stride + 1 (+1 if stride does not divide N), states in step order.
 * Errors: ABM_EINVAL (prob does not match the plan), ABM_EDEVICE. */
abm_status abm_solve(abm_plan_t *plan, const abm_problem *prob, double *y_out);

/* B trajectories by the blocked method: history older than the current block
 * of L steps enters through a Toeplitz-weight x history product on the matrix
 * cores, the last steps through a near band kept on chip, and the sequential
 * predictor/corrector runs per trajectory in double.  y_out is a host array of
 * B device pointers, each sized as for abm_solve.  stats may be NULL.
 * Errors: ABM_EINVAL, ABM_EDEVICE. */
abm_status abm_solve_batch(abm_plan_t *plan, const abm_problem *probs, int32_t B,
                           double *const *y_out, abm_stats *stats);

/* Wait for the context's stream and report device-side failures of the
 * solves enqueued so far on this plan: ABM_EDEVICE if a state became
 * non-finite or a bounded device-side wait gave up (the flags are then
 * cleared), ABM_OK otherwise. */
abm_status abm_plan_check(abm_plan_t *plan);

/* Per-kernel timing of abm_solve_batch: when enable != 0 every far-field and
 * chain launch is bracketed by HIP events on the context's stream, and
 * abm_solve_batch waits for the stream before returning so that far_ms and
 * chain_ms of abm_stats are filled.  Off by default.  Errors: ABM_EINVAL,
 * ABM_EDEVICE. */
abm_status abm_plan_timing(abm_plan_t *plan, int32_t enable);

/* Replay the launch sequence of abm_solve_batch from a HIP graph.  When
 * enable != 0, the next abm_solve_batch records its far-field, chain and
 * initialisation launches (with the fork/join between the far-field stream
 * and the context's stream) into a graph once, from a private stream, and
 * every later call only uploads that solve's descriptors (x0, p, h, output
 * pointers) and launches the graph on the context's stream.  Results are
 * bitwise those of the eager sequence.  Timed solves (abm_plan_timing) run
 * eagerly.  Off by default.  Errors: ABM_EINVAL (plan NULL); a failed capture
 * is reported by abm_solve_batch as ABM_EDEVICE. */
abm_status abm_plan_graph(abm_plan_t *plan, int32_t enable);

/* Copy the first n entries of the weight tables b_k, a_k, c_k (Section 2,
 * generated on the device by abm_plan) used by component 0 of problem idx of
 * the plan into host arrays of n doubles each (any of them may be NULL); a
 * double-double plan (ABM_FAR_DD) copies n (hi, lo) pairs, 2n doubles each.
 * Synchronises the context's stream.  Errors: ABM_EINVAL (idx or n out of
 * range), ABM_EDEVICE. */
abm_status abm_plan_weights(abm_plan_t *plan, int32_t idx, int64_t n, double *b, double *a,
                            double *c);

/* Serving: queue one problem on the context's server, which admits it when
 * its history memory fits the arena, batches it with the requests already
 * running and writes y_out (device pointer, sized as for abm_solve).  The
 * problem struct is copied; y_out must stay valid until abm_poll reports it
 * done.  Thread-safe: any number of threads may submit, poll and cancel on
 * one context at once (the serving state is made with the context; tickets
 * are unique).  Errors: ABM_EINVAL, ABM_ENOMEM (larger than the whole arena),
 * ABM_EDEVICE (the server stopped after a device error). */
abm_status abm_submit(abm_ctx *ctx, const abm_problem *prob, double *y_out, uint64_t *ticket);

/* Device memory the serving loop takes from the context's arena for one
 * request (its weight tables, history, carried sums and far-field partials),
 * for sizing arenas: a request is admitted once this many bytes are free in
 * one piece, and rejected by abm_submit with ABM_ENOMEM if it exceeds the
 * whole arena.  Errors: ABM_EINVAL. */
abm_status abm_request_bytes(abm_ctx *ctx, const abm_problem *prob, size_t *bytes);

/* ABM_EAGAIN while the request runs; ABM_OK once done (res filled, ticket
 * released); ABM_ENOENT for an unknown or already-collected ticket.  A
 * request that failed reports ABM_OK here with res->status set.  Thread-safe. */
abm_status abm_poll(abm_ctx *ctx, uint64_t ticket, abm_result *res);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): abm_solve
 * without a plan.  One trajectory by the plain per-step method, on the
 * current HIP device, enqueued on hip_stream (a hipStream_t; NULL = the null
 * stream), results bitwise those of abm_solve for the same problem.  prob and
 * y_out as for abm_solve (y_out: device memory of n_out*d doubles, owned by
 * the caller).  Allocates nothing: the weight tables, the status word and the
 * cooperative form's step flags and partial sums live in a library-wide
 * device array of 8 MiB that each GPU holds until the process ends.
 * Limit: (distinct orders among the components) * 3 * (N + 2048) * 8 bytes
 * plus about 130 KiB must fit those 8 MiB (one order: N <= 341952), and the plain
 * path's own limit applies; larger problems return ABM_EINVAL.  Calls on one
 * GPU share the array and keep the last call's contents: calls that overlap
 * on one GPU (different streams or host threads) race and must be serialised
 * by the caller; one stream orders them.  No plan means no abm_plan_check: a
 * run whose device-side wait gave up, or whose state became non-finite,
 * leaves a non-finite final state in y_out.  Errors: ABM_EINVAL, ABM_EDEVICE. */
abm_status abm_solve_noalloc(const abm_problem *prob, double *y_out, void *hip_stream);

/* Cancel a queued or running request (its poll then reports ABM_ECANCELED). */
abm_status abm_cancel(abm_ctx *ctx, uint64_t ticket);

const char *abm_strerror(abm_status status);
const char *abm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ABM_H */
