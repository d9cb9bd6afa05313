/*
 * tron.h -- C ABI of the MI355X batched trust-region Newton library.
 *
 * The library solves many small bound-constrained nonlinear programs at once,
 *     minimize f(x)  subject to  l <= x <= u,   x in R^n            (eq. prob, section 1)
 * with the trust-region Newton method of Algorithm 1 ("ExaTron's algorithm", section 3):
 * Cauchy point, free-subspace identification, complete Cholesky preconditioner of the
 * shifted reduced Hessian (section 4.3), trust-region preconditioned CG, back-transform,
 * projected line search, convergence on the infinity norm of the projected gradient
 * (section 5.1), with the ratio test and radius update of the TRON method the paper cites.
 * It also runs the component ADMM of the paper's power-flow application (section 6.1:
 * generator and branch subproblems, then buses, then multipliers), whose branch
 * subproblems (eq. exp-branch) are the batched solves.
 *
 * Conventions shared by every call:
 *  - All d_* pointers are device memory owned by the caller (any HIP allocation on the
 *    current device). Host pointers are named without the prefix and are copied before the
 *    call returns.
 *  - Every call is stream-ordered and asynchronous on `stream` (a hipStream_t, NULL = the
 *    null stream); results are valid once the stream has been synchronised.
 *  - Calls never throw and never abort; they return a tron_err. tron_last_error() returns a
 *    message for the calling thread's last failure.
 *  - A handle is not thread-safe; different handles may be used from different threads.
 *  - Problem-level failures (l_i > u_i, non-finite values) are reported per instance in
 *    d_status and never affect other instances.
 *  - FP64 throughout.
 */
#ifndef MI355X_TRON_H
#define MI355X_TRON_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TRON_OK = 0,
    TRON_ERR_INVALID = 1,      /* bad argument (null pointer, size, family/n mismatch)      */
    TRON_ERR_NOMEM = 2,        /* device or host allocation failed                          */
    TRON_ERR_DEVICE = 3,       /* a HIP call failed                                         */
    TRON_ERR_UNSUPPORTED = 4,  /* n outside the supported range for the family              */
    TRON_ERR_BUSY = 5          /* server admission refused: over the memory budget          */
} tron_err;

/* Per-instance outcome written to d_status. */
enum {
    TRON_CONVERGED = 0,   /* ||grad_[l,u] f(x)||_inf <= gtol                              */
    TRON_MAX_ITER = 1,    /* max_iter trust-region iterations taken                       */
    TRON_STALLED = 2,     /* no model decrease possible / reductions at rounding level    */
    TRON_NONFINITE = 3,   /* f or grad f not finite at an accepted point                  */
    TRON_BAD_BOUNDS = 4,  /* some l_i > u_i (or a NaN bound); x is left at x0             */
    TRON_AL_MAX_OUTER = 5 /* tron_al_solve: outer_max solves without ||h||_inf <= ctol    */
};

/* Problem families. Parameter block sizes (doubles per instance):
 *   QP4:   n(n+1)/2 + n + 1 -- f = x'Qx/2 + c'x + kappa sum x_i^4; packed lower triangle of
 *          Q row by row (Q00 Q10 Q11 Q20 ...), then c, then kappa. 1 <= n <= 512.
 *   BR6:   36, n = 6 -- the branch subproblem of eq. exp-branch in x = (v_i, v_j, th_i,
 *          th_j, z_ij, z_ji): [0..7] g_ij b_ij gc_ij bc_ij g_ji b_ji gc_ji bc_ji,
 *          [8..15] targets of (p_ij q_ij p_ji q_ji w_i w_j th_i th_j), [16..23] their
 *          multipliers, [24..25] multipliers of z_ij - p_ij and z_ji - p_ji, [26..33]
 *          penalties of the eight couplings, [34..35] penalties of the two z couplings;
 *          flows per eqs. pij..qji with w = v^2, wR = v_i v_j cos(th_i - th_j),
 *          wI = v_i v_j sin(th_i - th_j).
 *   HS45M: 0 -- f = 120 - prod x_i (the variant of hs45 in section 4.2). 1 <= n <= 128.
 *   BR8L:  40, n = 8 -- BR6 with the line limits of eq. LineLimit on both ends written as
 *          equalities with slacks (the footnote on inequalities in section 1),
 *          h_lm = p_lm^2 + q_lm^2 + sigma_lm - smax^2, added as the augmented-Lagrangian
 *          terms lambda_lm h_lm + rho_h/2 h_lm^2 of section 1. x = (v_i, v_j, th_i, th_j,
 *          z_ij, z_ji, sigma_ij, sigma_ji); [0..35] as BR6, [36] smax^2, [37] lambda_ij,
 *          [38] lambda_ji, [39] rho_h. */
typedef enum {
    TRON_FAMILY_QP4 = 0,
    TRON_FAMILY_BR6 = 1,
    TRON_FAMILY_HS45M = 2,
    TRON_FAMILY_BR8L = 3
} tron_family;

typedef struct {
    double gtol;       /* absolute tolerance on ||grad_[l,u] f||_inf (default 1e-6)          */
    int32_t max_iter;  /* trust-region iterations (default 500)                             */
    uint32_t flags;    /* TRON_FLAG_*                                                        */
    double cg_rtol;    /* CG stops when ||r|| <= cg_rtol ||r0|| (default 0.1)               */
    double delta0;     /* > 0: initial radius of every instance; <= 0: ||grad_[l,u] f(x0)||_2 */
} tron_options;

/* Start from the radius and Cauchy step length the handle kept from its previous solve
 * (per instance), instead of the cold rule. x0 is always the caller's. */
#define TRON_FLAG_WARM 1u
/* Capture the whole solve (all size buckets, forked over the handle's streams) into a HIP
 * graph on the first call with a given set of pointers, and replay that graph on later calls
 * with the same pointers (new pointers or options re-capture). */
#define TRON_FLAG_GRAPH 2u

void tron_default_options(tron_options *opt);
const char *tron_last_error(void);
/* Parameter doubles per instance for (family, n); -1 if unsupported. */
int64_t tron_param_size(tron_family family, int32_t n);

typedef struct tron_batch tron_batch;

/* Create a handle for `batch` instances of `family`. n_host (host, length batch) gives
 * each instance's n, or is NULL and every instance has n_uniform. Instances are packed
 * back to back in instance order: parameter block b starts at the sum of the sizes of
 * blocks 0..b-1, and vector b (lo, hi, x0, x) at the sum of n over 0..b-1.
 * The handle builds its launch plan (size buckets, kernel geometry, captured graph) here
 * and owns per-instance resident state (trust radius, Cauchy step length) on the device.
 * opt may be NULL (defaults). Errors: INVALID (batch < 0, n out of range, family/n
 * mismatch), UNSUPPORTED, NOMEM, DEVICE. */
tron_err tron_batch_create(tron_batch **out, tron_family family, int64_t batch,
                           const int32_t *n_host, int32_t n_uniform, const tron_options *opt,
                           void *stream);

/* Launch plan of a handle: instances with n <= lane_max_n are solved one per GPU lane (a
 * kernel per exact n); larger ones one per wavefront, grouped into buckets by the first of
 * `edges` (increasing, <= 128) that holds them, with LDS sized for that edge. Buckets run
 * concurrently on `streams` streams; lane kernels use workgroups of lane_block (64 or 256).
 * pool_waves > 0 selects the persistent size-bucketed form instead (section 4.1, a single
 * kernel rather than one per size) for batches of mixed sizes up to n = 128: one launch
 * solves every wavefront instance, with one workgroup of pool_waves (8 or 12) wavefronts
 * per CU sharing the CU's LDS as a pool; each wave claims instances from the batch's list
 * (largest n first, each of the largest followed by as many of the smallest as fill the
 * CU's other waves while its pool holds the largest) and reserves exactly the LDS its
 * instance needs; a second launch
 * solves every lane instance, in packs of 64 of one size. Edges and streams are then unused. */
typedef struct {
    int32_t lane_max_n;   /* 0..8 */
    int32_t nedges;       /* 1..16 */
    int32_t edges[16];
    int32_t streams;      /* 1..8 */
    int32_t lane_block;   /* 64 or 256 */
    int32_t pool_waves;   /* 0 (bucketed), 8 or 12 (persistent; mixed-size batches only)      */
    int32_t lane_group;   /* lanes per instance for n <= lane_max_n: 1 (lane kernel), 2, 4 or 8
                             (the group kernel: one instance per group of lanes, rows split
                             over the group, section 4.2's thread configuration), or 0:
                             automatic, 8 for a uniform quartic batch with n = 7 or 8 of at
                             most 16,384 instances (where it is the faster), else 1          */
    int32_t group16;      /* 0, 8 or 16: instances with lane_max_n < n <= 16 go to the group
                             kernel of that width instead of the wavefront kernel            */
    int32_t wave_global;  /* 1: quartic-family wavefront buckets up to n = 128 keep the Hessian
                             and its factor in a global-memory workspace (L2) instead of LDS,
                             as beyond n = 128 (section 4.5's workspace comparison)          */
} tron_plan_spec;

/* lane_max_n 8, edges 16/24/32/40/48/56/64/80/96/112/128, 4 streams, lane_block 64,
 * pool_waves 12 (a batch of mixed sizes up to n = 128 runs the persistent launch; uniform
 * batches and mixed batches beyond 128 use the buckets), lane_group 0 (automatic),
 * group16 0, wave_global 0. */
void tron_default_plan_spec(tron_plan_spec *spec);
/* tron_batch_create with an explicit plan (spec NULL = default). INVALID for a bad spec,
 * UNSUPPORTED when some n exceeds the largest edge. */
tron_err tron_batch_create_ex(tron_batch **out, tron_family family, int64_t batch,
                              const int32_t *n_host, int32_t n_uniform, const tron_options *opt,
                              const tron_plan_spec *spec, void *stream);
/* Autotuner: time candidate plans (bucket edge sets, streams, lane/wave split, lane
 * workgroup size, group widths, the persistent launch) on the caller's own batch, each
 * captured as a graph (its device time) and replayed `reps` times after the capturing solve
 * (the fastest replay counts); then the four fastest distinct
 * candidates are timed again in three interleaved rounds and the lowest median wins; it is
 * returned in *best (and that median time per solve in *best_ms). The outputs are written
 * by the trial solves. When cache_path is not NULL the result is looked up in / appended to
 * that text file, keyed by the family and the histogram of sizes (a cached entry returns
 * without timing). Errors as tron_batch_create / solve, plus DEVICE for timing failures. */
tron_err tron_autotune(tron_family family, int64_t batch, const int32_t *n_host,
                       const double *d_params, const double *d_lo, const double *d_hi,
                       const double *d_x0, double *d_x, double *d_f, int32_t *d_status,
                       int32_t *d_iters, int32_t reps, const char *cache_path,
                       tron_plan_spec *best, double *best_ms, void *stream);

/* Solve every instance (Algorithm 1 per instance). d_x0 (read) and d_x (written) may be the
 * same buffer for an in-place warm start. d_f (batch doubles), d_status and d_iters (batch
 * int32 each) are written. d_params, d_lo, d_hi are read only. Bounds may be +-inf.
 * Instances with n <= 8 are solved one per GPU lane, larger ones one per wavefront (up to
 * n = 128 with the Hessian and factor in LDS, beyond that in a global-memory workspace of
 * n ((n+1)|1) doubles per instance, rounded up to n = 256 or 512, that the handle allocates
 * at creation); the size buckets run concurrently on the handle's own streams, joined back
 * into `stream`.
 * Errors: INVALID (null pointers), DEVICE (launch or capture failure). */
tron_err tron_batch_solve(tron_batch *h, const double *d_params, const double *d_lo,
                          const double *d_hi, const double *d_x0, double *d_x, double *d_f,
                          int32_t *d_status, int32_t *d_iters, void *stream);

/* Augmented-Lagrangian loop (section 1: general constraints h(x) = 0 through a sequence of
 * bound-constrained minimisations of L_rho(x; lambda, rho) with (lambda, rho) updated in
 * between). The paper leaves the update to the literature it cites; this one is the
 * first-order multiplier step lambda <- lambda + rho h(x) with
 * rho <- min(rho_growth * rho, rho_max) whenever ||h||_inf > decrease * its previous value,
 * stopping when ||h||_inf <= ctol. */
typedef struct {
    double ctol;        /* stop when ||h(x)||_inf <= ctol (default 1e-6)                      */
    int32_t outer_max;  /* bound-constrained solves per instance at most (default 50)         */
    double rho_growth;  /* >= 1 (default 10)                                                  */
    double decrease;    /* >= 0 (default 0.25)                                                */
    double rho_max;     /* > 0 (default 1e6)                                                  */
} tron_al_options;

void tron_default_al_options(tron_al_options *o);

/* Run the loop on every instance of a BR8L handle, one GPU lane per instance, entirely on
 * the device. Each solve uses the handle's tron_options; the first starts from d_x0 (and
 * from the resident radius when TRON_FLAG_WARM is set), later ones from the previous x and
 * radius. d_params (batch x 40 doubles) is read and updated in place: on return [37..38]
 * hold the last multipliers and [39] the last penalty, ready for a warm restart. Outputs:
 * d_x (batch x 8), d_f (L_rho at the last solve), d_status (TRON_CONVERGED when the last
 * solve converged and ||h||_inf <= ctol, TRON_AL_MAX_OUTER, or the failing solve's status),
 * d_iters (TRON iterations over all solves), d_outer (solves taken) and d_viol (the last
 * ||h||_inf). Asynchronous on `stream`.
 * Errors: INVALID (null pointers, bad options), UNSUPPORTED (not a BR8L handle), DEVICE. */
tron_err tron_al_solve(tron_batch *h, const tron_al_options *opt, double *d_params,
                       const double *d_lo, const double *d_hi, const double *d_x0, double *d_x,
                       double *d_f, int32_t *d_status, int32_t *d_iters, int32_t *d_outer,
                       double *d_viol, void *stream);

/* Copy the resident per-instance state out of / into the handle: d_state holds 2*batch
 * doubles, the radii then the Cauchy step lengths. Used for checkpoint and resume. */
tron_err tron_batch_get_state(tron_batch *h, double *d_state, void *stream);
tron_err tron_batch_set_state(tron_batch *h, const double *d_state, void *stream);

/* Replace the options used by later solves (the plan is kept). */
tron_err tron_batch_set_options(tron_batch *h, const tron_options *opt);

/* Describe the launch plan: number of buckets, and for each bucket (up to max_buckets)
 * its largest n, its lanes per instance and its instance count, as 3 int32 per bucket. */
tron_err tron_batch_plan(const tron_batch *h, int32_t *nbuckets, int32_t *desc,
                         int32_t max_buckets);

/* Record, for every instance of later solves, the device wall clock when its solve started
 * and ended: d_ts holds 2*batch int64 (start, end) written at solve time, or NULL to stop.
 * The buffer stays the caller's and must outlive the solves that write it. The clock
 * runs at tron_clock_rate_hz() (0 if unknown). Used for per-instance solve latency. */
tron_err tron_batch_set_timestamps(tron_batch *h, int64_t *d_ts);
int64_t tron_clock_rate_hz(void);

tron_err tron_batch_destroy(tron_batch *h);

/* Allocation-free solve, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc). One cold-start
 * solve of `batch` instances that all have size n, with the same kernels and results as
 * tron_batch_create(n_uniform = n) + tron_batch_solve: instances with n <= 8 one per GPU
 * lane, larger ones one per wavefront. The solve's working memory (per-instance radius and
 * Cauchy step length, 16 bytes each, and for n > 128 the matrix workspace of
 * n ((n+1)|1) doubles per instance) lives in a fixed device array of the library,
 * tron_noalloc_scratch_bytes() = 64 MiB on every device the call runs on, held until the
 * process ends; the call makes no device allocation. The caller passes inputs and outputs
 * as for tron_batch_solve (d_x0 and d_x may alias). opt may be NULL; its flags must be 0.
 * The array is shared by every call on a device and keeps the last call's contents (a call
 * writes every word it reads first), so calls that overlap in time on one device race:
 * issue them on one stream. Asynchronous on `stream`.
 * Errors: INVALID (bad family/n/batch, nonzero flags, null pointers, or a batch whose
 * working memory exceeds the array), UNSUPPORTED (device index above 63), DEVICE. */
tron_err tron_solve_noalloc(tron_family family, int64_t batch, int32_t n, const tron_options *opt,
                            const double *d_params, const double *d_lo, const double *d_hi,
                            const double *d_x0, double *d_x, double *d_f, int32_t *d_status,
                            int32_t *d_iters, void *stream);
int64_t tron_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------------------ */
/* Continuous-batching server. Solve requests (each a batch of instances of one family,   */
/* sizes mixed, the same Algorithm 1 per instance) are queued from any host thread and    */
/* admitted in arrival order as the device-memory budget and the in-flight LDS budget     */
/* allow; consecutive queued requests share one launch group; groups run concurrently on   */
/* the server's streams, so requests that arrive while others are on the GPU overlap with */
/* them. An instance's result does not depend on what it was batched with.                */
/* ------------------------------------------------------------------------------------ */
typedef struct tron_server tron_server;

typedef struct {
    size_t hbm_budget;            /* device bytes for requests in flight and open sessions;
                                     also the size of the pinned host staging area          */
    size_t lds_budget;            /* LDS bytes of wavefront-kernel instances in flight      */
    int32_t max_inflight;         /* launch groups on the device at once (>= 1)             */
    int32_t streams;              /* device streams the groups are dealt to (>= 1)          */
    int32_t coalesce;             /* 1: a launch group may take several queued requests     */
    int32_t max_group_instances;  /* instances per launch group (>= 1)                      */
    tron_options opt;             /* solver options of every request (flags ignored)        */
} tron_server_config;

void tron_server_default_config(tron_server_config *cfg);
/* Allocates the device arena and pinned staging up front and starts the scheduler thread.
 * Errors: INVALID (configuration), NOMEM, DEVICE. */
tron_err tron_server_create(tron_server **out, tron_family family, const tron_server_config *cfg);
/* Queue `batch` instances given as host arrays packed as for tron_batch_create (copied before
 * the call returns). session != 0 keeps the instances' solution, radius and Cauchy step
 * resident on the device after the solve; a later request of the same session (same sizes)
 * may pass x0 = NULL to start from them. A session holds at most one request at a time.
 * Instances must have n <= 128 (the server keeps every matrix in LDS).
 * Errors: INVALID, UNSUPPORTED (n > 128), BUSY (larger than the device budget, or its
 * session is busy). */
tron_err tron_server_submit(tron_server *s, int64_t batch, const int32_t *n, const double *params,
                            const double *lo, const double *hi, const double *x0, uint64_t session,
                            int64_t *ticket);
/* *state: 0 queued, 1 on the device, 2 done. */
tron_err tron_server_poll(tron_server *s, int64_t ticket, int32_t *state);
/* Block until the request is done (timeout_s < 0: no limit); BUSY on timeout. */
tron_err tron_server_wait(tron_server *s, int64_t ticket, double timeout_s);
/* Copy a finished request's outputs to host arrays (any may be NULL) and release the ticket;
 * latency_s is the time from submission to completion. BUSY if not finished. */
tron_err tron_server_result(tron_server *s, int64_t ticket, double *x, double *f, int32_t *status,
                            int32_t *iters, double *latency_s);
/* Take a queued request off the queue before it is admitted: it completes without a solve
 * (waiters wake; tron_server_result then returns BUSY with a cancellation message and
 * releases the ticket). BUSY when the request is already on the device or finished,
 * INVALID for an unknown ticket. */
tron_err tron_server_cancel(tron_server *s, int64_t ticket);
/* Free a session's resident state (BUSY while it has a request outstanding). */
tron_err tron_server_close_session(tron_server *s, uint64_t session);
/* out4: requests done, instances done, device bytes in use, LDS bytes in flight. */
tron_err tron_server_stats(tron_server *s, int64_t *out4);
/* Stops the scheduler, waits for the groups on the device, frees everything. */
tron_err tron_server_destroy(tron_server *s);

/* ------------------------------------------------------------------------------------ */
/* Component ADMM of the power-flow application (section 6.1).                           */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t nbus, nbranch, ngen, ref_bus;
    double rho;                        /* penalty of every coupling                        */
    double base_mva;                   /* generator costs are per MW, powers per unit      */
    const int32_t *br_from, *br_to;    /* host, nbranch each                               */
    const double *br_adm;              /* host, nbranch x 8 (BR6 order)                    */
    const double *br_lo, *br_hi;       /* host, nbranch x 6 bounds on the BR6 variables    */
    const int32_t *gen_bus;            /* host, ngen                                       */
    const double *gen_cost;            /* host, ngen x 2: c2 (per MW^2), c1 (per MW)       */
    const double *gen_lim;             /* host, ngen x 4: pmin pmax qmin qmax (per unit)   */
    const double *bus_load;            /* host, nbus x 4: pd qd gsh bsh (per unit)         */
} admm_network;

typedef struct admm admm;

/* Doubles in the flat ADMM state:
 *   generators (ngen each, in this order): pg qg pg~ qg~ lambda_pg lambda_qg
 *   branches: x (nbranch x 6), couplings y (nbranch x 8: p_ij q_ij p_ji q_ji w_i w_j th_i
 *             th_j), bus copies of the flows (nbranch x 4), lambda (nbranch x 8),
 *             mu (nbranch x 2), radius (nbranch), Cauchy step length (nbranch)
 *   buses: w~ (nbus), theta~ (nbus)
 * = 6 ngen + 30 nbranch + 2 nbus. */
int64_t admm_state_size(const admm_network *net);

/* Copy the network to the device and set the initial state (v = 1, theta = 0, z = 0,
 * generator powers at mid-range, copies equal to the component values, multipliers 0).
 * Every bus must be the end of at least one branch. */
tron_err admm_create(admm **out, const admm_network *net, const tron_options *branch_opt,
                     void *stream);

/* Run `iters` ADMM iterations. Per iteration: generator updates and the batched branch
 * solves (warm-started from the resident x, radius, step length), then the bus updates,
 * then the multiplier updates. d_resid (2*iters doubles) receives (primal, dual) residual
 * norms per iteration, or is NULL. */
tron_err admm_step(admm *a, int32_t iters, double *d_resid, void *stream);

/* Copy the state out / in (count must equal admm_state_size). */
tron_err admm_get_state(admm *a, double *d_buf, int64_t count, void *stream);
tron_err admm_set_state(admm *a, const double *d_buf, int64_t count, void *stream);
tron_err admm_destroy(admm *a);

#ifdef __cplusplus
}
#endif
#endif
