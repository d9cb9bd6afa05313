/*
 * Oracle for the batched trust-region Newton (TRON) solve and the component ADMM step.
 *
 * TEST INFRASTRUCTURE ONLY. A plain, slow, FP64 CPU implementation of what the GPU
 * library computes. It exists to check the GPU library and to time a CPU baseline.
 * The GPU library includes nothing from here and this code includes nothing from the
 * GPU library; only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg load it.
 *
 * Paper: Y. Kim, F. Pacaud, K. Kim, M. Anitescu, "Leveraging GPU batching for scalable
 * nonlinear programming through massive Lagrangian decomposition", arXiv 2106.14995.
 * Citations below name the paper's sections, equations, algorithm and figures.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC (no contraction, so every
 * product and sum rounds on its own, in the order written).
 */
#ifndef TRON_ORACLE_H
#define TRON_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Problem families (same numbering as the GPU library's public enum; an interface). */
enum { OR_QP4 = 0, OR_BR6 = 1, OR_HS45M = 2, OR_BR8L = 3 };
/* Per-instance outcomes (OR_AL_MAX_OUTER: the multiplier loop hit its iteration cap). */
enum { OR_CONVERGED = 0, OR_MAX_ITER = 1, OR_STALLED = 2, OR_NONFINITE = 3, OR_BAD_BOUNDS = 4,
       OR_AL_MAX_OUTER = 5 };

typedef struct {
    double gtol;     /* absolute bound on the infinity norm of the projected gradient      */
    int32_t max_iter;
    int32_t use_warm;/* 1: take delta / alpha_c from the in/out arrays where they are > 0 */
    double cg_rtol;  /* relative residual tolerance of the conjugate-gradient solve        */
    double delta0;   /* > 0: initial trust radius for all instances; <= 0: cold rule      */
} or_opts;

/* Number of doubles in one instance's parameter block. */
int64_t or_param_size(int32_t family, int32_t n);

/* Per-instance statistics written by or_tron_batch when stats != NULL, OR_NSTAT doubles each:
 * [0] algorithmic flops (textbook counts; minimal family counts for QP4 and BR6), [1] outer iterations, [2] CG iterations, [3] Cholesky attempts,
 * [4] Cauchy trials, [5] projected-search trials, [6] subspace passes, [7] accepted steps. */
#define OR_NSTAT 8

/* Solve `batch` independent problems min f(x) s.t. lo <= x <= hi (eq. prob, Algorithm 1).
 * n_per (length batch) gives each instance's size, or is NULL and n_uniform is used.
 * Parameter blocks and vectors are packed back to back in instance order.
 * delta / alphac (length batch, may be NULL) are read when opt->use_warm and written on exit.
 * nthreads <= 0 uses every online host core. Returns the number of threads used. */
int32_t or_tron_batch(int32_t family, int64_t batch, const int32_t *n_per, int32_t n_uniform,
                      const double *params, const double *lo, const double *hi, const double *x0,
                      double *x, double *f, int32_t *status, int32_t *iters,
                      double *delta, double *alphac, double *stats,
                      const or_opts *opt, int32_t nthreads);

/* Family evaluations (for the tests): f, gradient, dense row-major Hessian. */
double or_eval_f(int32_t family, int32_t n, const double *params, const double *x);
void or_eval_g(int32_t family, int32_t n, const double *params, const double *x, double *g);
void or_eval_h(int32_t family, int32_t n, const double *params, const double *x, double *h);
/* f and ||grad_[l,u] f||_inf at the points x of a packed batch (as or_tron_batch). */
void or_eval_batch(int32_t family, int64_t batch, const int32_t *n_per, int32_t n_uniform,
                   const double *params, const double *lo, const double *hi, const double *x,
                   double *f_out, double *pg_out);
/* Branch flows (p_ij, q_ij, p_ji, q_ji) at x for a BR6 parameter block. */
void or_br6_flows(const double *params, const double *x, double *pq4);

/* Core operations (Fig. "Core operations"), exposed for the tests. */
int32_t or_ccf(int32_t m, const double *a, double alpha, double *l);      /* 0 on success   */
void or_trsv_lower(int32_t m, const double *l, double *b);               /* L y = b, in place   */
void or_trsv_lower_t(int32_t m, const double *l, double *b);             /* L^T y = b, in place */
double or_trqsol(int32_t m, const double *x, const double *p, double delta);
void or_breakpt(int32_t n, const double *x, const double *lo, const double *hi, const double *w,
                int32_t *nbrpt, double *brptmin, double *brptmax);
void or_gpstep(int32_t n, const double *x, const double *lo, const double *hi, double alpha,
               const double *w, double *s);
double or_projgrad_inf(int32_t n, const double *x, const double *lo, const double *hi,
                       const double *g);
/* Preconditioned CG of the subspace step on a dense m x m block (for the tests).
 * r: model gradient on the block; returns the exit code (0 converged, 1 max iterations,
 * 2 negative curvature, 3 trust boundary); w receives L^{-T} s_hat, *iters the count. */
int32_t or_subspace_cg(int32_t m, const double *a, const double *r, double delta, double cg_rtol,
                       double *w, double *shat, int32_t *iters, double *shift_out);

/* Single steps of one iteration (Algorithm 1 and the readings of section 3), for the tests.
 * or_radius_update: the new radius after a trial with ratio rho (reading S2); ft is f at
 *   the trial point, gts = g's, snorm the step length in the norm of reading S31.
 * or_cauchy_step: the Cauchy search from alpha (reading S4) on the model with gradient g
 *   and dense row-major Hessian h at x; returns the accepted alpha, writes P[x - alpha g]
 *   to xs_out and the number of trial points to *trials.
 * or_projected_search: the search along dir from xs with model gradient r = g + Hs at xs
 *   (reading S13); returns 1 when a step was accepted, writes the new xs, the last beta
 *   tried and the number of trials.
 * or_step_norm: ||L^T s_F|| on the m free indices free_idx (L the m x m row-major factor of
 *   that block), combined with ||s|| on the other indices (reading S31); m = 0 gives ||s||.
 * or_actual_reduction: f - ft, or -(g + gt)'s / 2 when pred is at the rounding level of f
 *   (reading S30).
 * or_family_flops: the minimal count charged for one evaluation (which = 0 f, 1 gradient
 *   after f at the same point, 2 Hessian after both) of QP4 or BR6; -1 otherwise. */
double or_radius_update(double delta, double rho, double f, double ft, double gts, double snorm,
                        int32_t finite_trial);
double or_cauchy_step(int32_t n, const double *x, const double *lo, const double *hi,
                      const double *g, const double *h, double delta, double alpha,
                      double *xs_out, int32_t *trials);
int32_t or_projected_search(int32_t n, const double *xs, const double *lo, const double *hi,
                            const double *dir, const double *r, const double *h,
                            double *xs_out, double *beta_out, int32_t *trials);
double or_step_norm(int32_t n, const double *s, int32_t m, const int32_t *free_idx,
                    const double *l);
double or_actual_reduction(int32_t n, double f, double ft, double pred, const double *g,
                           const double *gt, const double *s);
double or_family_flops(int32_t family, int32_t n, int32_t which);

/* ---------------- augmented-Lagrangian loop (section 1) for BR8L instances ---------------- */
typedef struct {
    double ctol;       /* stop when ||h(x)||_inf <= ctol                                  */
    int32_t outer_max; /* at most this many bound-constrained solves                       */
    double rho_growth; /* penalty factor applied when the violation did not shrink enough  */
    double decrease;   /* ... i.e. when ||h|| > decrease * previous ||h||                  */
    double rho_max;    /* the penalty never grows beyond this                              */
} or_al_opts;

/* Per instance (n = 8, 40 parameters): solve, update lambda (params[37..38]) and rho_h
 * (params[39]) in place, repeat. iters: total TRON iterations; outer: bound-constrained
 * solves; viol: final ||h||_inf; f: the augmented Lagrangian at the last solve. */
int32_t or_al_batch(int64_t batch, double *params, const double *lo, const double *hi,
                    const double *x0, double *x, double *f, int32_t *status, int32_t *iters,
                    int32_t *outer, double *viol, const or_opts *opt, const or_al_opts *al,
                    int32_t nthreads);

/* ---------------- component ADMM (section "Distributed control of ACOPF") ---------------- */
typedef struct {
    int32_t nbus, nbranch, ngen, ref_bus;
    double rho, base_mva;
    const int32_t *br_from, *br_to;   /* nbranch each                                      */
    const double *br_adm;             /* nbranch x 8: g_ij b_ij gc_ij bc_ij g_ji b_ji gc_ji bc_ji */
    const double *br_lo, *br_hi;      /* nbranch x 6 bounds on (v_i v_j th_i th_j z_ij z_ji) */
    const int32_t *gen_bus;           /* ngen                                              */
    const double *gen_cost;           /* ngen x 2: c2 c1 (per MW^2, per MW)                 */
    const double *gen_lim;            /* ngen x 4: pmin pmax qmin qmax (per unit)           */
    const double *bus_load;           /* nbus x 4: pd qd gsh bsh (per unit)                 */
} or_network;

/* Flat state layout (doubles): 6*ngen + 30*nbranch + 2*nbus, see or_admm_state_size. */
int64_t or_admm_state_size(const or_network *net);
void or_admm_init(const or_network *net, double *state);
/* Run `iters` iterations in place; resid receives (primal, dual) per iteration (2*iters). */
int32_t or_admm_run(const or_network *net, double *state, int32_t iters, double *resid,
                    const or_opts *opt, int32_t nthreads);
/* One phase (0 generators, 1 branches, 2 buses, 3 multipliers) in place, for the tests. */
int32_t or_admm_phase(const or_network *net, double *state, int32_t phase, double *out,
                      const or_opts *opt, int32_t nthreads);

#ifdef __cplusplus
}
#endif
#endif
