/*
 * Oracle for the batched trust-region Newton (TRON) solve and the component ADMM step.
 *
 * TEST INFRASTRUCTURE ONLY (see tron_oracle.h). Plain scalar FP64 loops, one instance per
 * thread, no blocking, no fusion, compiled without floating-point contraction.
 *
 * The solver follows Algorithm 1 ("ExaTron's algorithm") of the paper step by step:
 *   evaluate f, grad f, Hessian            (Algorithm 1, evaluation step)
 *   Cauchy point x_c = P[x - alpha g]      (Algorithm 1, Cauchy step; section 3)
 *   free set F = { l < x_c < u }           (Algorithm 1, subspace identification)
 *   L L^T = A + alpha I, A = H_FF          (Algorithm 1, preconditioner; section 4.3)
 *   trust-region CG on L^-1 A L^-T         (Algorithm 1, CG step; section 3, Steihaug)
 *   w = L^-T s                              (Algorithm 1, back-transform)
 *   x+ = P[x + beta w]                      (Algorithm 1, projected line search)
 *   convergence on ||grad_[l,u] f||_inf    (section 5.1)
 * with the core operations of the "Core operations" figure (axpy, ccf, copy, dot, gemv,
 * nrm2, scal, trtrs, breakpt, ccfs, gpstep, trqsol). The paper leaves the ratio test, the
 * radius update, the Cauchy and line-search constants and the shift rule to the TRON
 * method it cites (Lin and More); the readings used are listed where they are applied.
 *
 * Algorithmic flop counts (the `fl` accumulators) use textbook counts: a multiply or an
 * add is 1, a division 1, a square root 1, a sine or cosine 1; comparisons and copies 0.
 * Core operations are charged by their textbook formulas (dot 2m, nrm2 2m+1, axpy 2m,
 * gemv 2m^2, triangular solve m^2, Cholesky column j: 2j+1 for the pivot and 2j+1 per
 * entry below it, gpstep 3n, breakpt 2 per breakpoint). The evaluations of the QP4 and
 * BR6 families are charged the minimal counts of the method's own work, each quantity
 * formed once per point (FAM_FLOPS below), not the loops this file happens to use to
 * evaluate them; BR8L and HS45M are charged as written.
 */
#include "tron_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdatomic.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

/* ------------------------------------------------------------------------------------ */
/* Constants of the readings (TRON defaults where the paper is silent).                 */
/* ------------------------------------------------------------------------------------ */
static const double MU0 = 0.01;        /* sufficient-decrease constant, Cauchy and search  */
static const double ETA0 = 1e-4, ETA1 = 0.25, ETA2 = 0.75;         /* ratio thresholds   */
static const double SIG1 = 0.25, SIG2 = 0.5, SIG3 = 4.0;           /* radius factors     */
static const int CAUCHY_MAX = 60;      /* extrapolation / interpolation steps             */
static const int SEARCH_HALVINGS = 20; /* projected search: beta = 1, 1/2, ..., 2^-20     */
static const int SHIFT_TRIES = 64;     /* Cholesky attempts with growing shift            */
static const double STALL_REL = 1e-15; /* |ared|, pred <= this * max(1,|f|)  -> stalled    */
static const double ARED_SWITCH = 1e-10;/* pred <= this * max(1,|f|): gradient-based ared   */

/* ------------------------------------------------------------------------------------ */
/* Core operations (figure "Core operations").                                         */
/* ------------------------------------------------------------------------------------ */
static double dot(int n, const double *a, const double *b, double *fl)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    *fl += 2.0 * n;
    return s;
}

static double nrm2(int n, const double *a, double *fl)
{
    double s = dot(n, a, a, fl);
    *fl += 1.0;
    return sqrt(s);
}

/* y <- y + alpha x */
static void axpy(int n, double alpha, const double *x, double *y, double *fl)
{
    for (int i = 0; i < n; i++) y[i] = y[i] + alpha * x[i];
    *fl += 2.0 * n;
}

/* y <- A x, A dense n x n row-major (gemv with alpha = 1, beta = 0) */
static void gemv(int n, const double *a, const double *x, double *y, double *fl)
{
    for (int i = 0; i < n; i++) {
        double s = 0.0;
        for (int j = 0; j < n; j++) s += a[i * n + j] * x[j];
        y[i] = s;
    }
    *fl += 2.0 * n * n;
}

/* trtrs, forward substitution: solve L y = b in place, L lower triangular row-major. */
void or_trsv_lower(int32_t m, const double *l, double *b)
{
    for (int i = 0; i < m; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= l[i * m + k] * b[k];
        b[i] = s / l[i * m + i];
    }
}

/* trtrs, backward substitution: solve L^T y = b in place. */
void or_trsv_lower_t(int32_t m, const double *l, double *b)
{
    for (int i = m - 1; i >= 0; i--) {
        double s = b[i];
        for (int k = i + 1; k < m; k++) s -= l[k * m + i] * b[k];
        b[i] = s / l[i * m + i];
    }
}

static void trsv_fwd(int m, const double *l, double *b, double *fl)
{
    or_trsv_lower(m, l, b);
    *fl += (double)m * m;
}

static void trsv_bwd(int m, const double *l, double *b, double *fl)
{
    or_trsv_lower_t(m, l, b);
    *fl += (double)m * m;
}

/* ccfs + ccf: left-looking (lazy-update) complete Cholesky of A + alpha I (section 4.3).
 * Column j is formed from the already-finished columns 0..j-1 just before it is scaled.
 * Returns 0 on success, j+1 when the pivot of column j is not positive (failure, S8). */
static int ccf_count(int m, const double *a, double alpha, double *l, double *fl)
{
    for (int i = 0; i < m * m; i++) l[i] = 0.0;
    for (int j = 0; j < m; j++) {
        double d = a[j * m + j] + alpha;          /* ccfs: A + alpha I on the diagonal */
        for (int k = 0; k < j; k++) d -= l[j * m + k] * l[j * m + k];
        *fl += 1.0 + 2.0 * j;
        if (!(d > 0.0)) return j + 1;
        double piv = sqrt(d);
        *fl += 1.0;
        l[j * m + j] = piv;
        for (int i = j + 1; i < m; i++) {
            double s = a[i * m + j];
            for (int k = 0; k < j; k++) s -= l[i * m + k] * l[j * m + k];
            l[i * m + j] = s / piv;
            *fl += 2.0 * j + 1.0;
        }
    }
    return 0;
}

int32_t or_ccf(int32_t m, const double *a, double alpha, double *l)
{
    double fl = 0.0;
    return ccf_count(m, a, alpha, l, &fl);
}

/* Componentwise median of (l, v, u): the projection P onto the box [l, u]. */
static double proj1(double v, double lo, double hi)
{
    if (v < lo) return lo;
    if (v > hi) return hi;
    return v;
}

/* gpstep: s = P[x + alpha w] - x; also returns the projected point xn. */
static void gpstep_pt(int n, const double *x, const double *lo, const double *hi, double alpha,
                      const double *w, double *xn, double *s, double *fl)
{
    for (int i = 0; i < n; i++) {
        xn[i] = proj1(x[i] + alpha * w[i], lo[i], hi[i]);
        s[i] = xn[i] - x[i];
    }
    *fl += 3.0 * n;
}

void or_gpstep(int32_t n, const double *x, const double *lo, const double *hi, double alpha,
               const double *w, double *s)
{
    double fl = 0.0;
    double *xn = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    gpstep_pt(n, x, lo, hi, alpha, w, xn, s, &fl);
    free(xn);
}

/* breakpt: breakpoints b_i = (u_i - x_i)/w_i (w_i > 0) or (l_i - x_i)/w_i (w_i < 0) along
 * x + t w. A zero w_i or an infinite bound gives no breakpoint (S12). With none, min and max
 * are returned as +inf. */
static void breakpt_count(int n, const double *x, const double *lo, const double *hi,
                          const double *w, int *nb, double *bmin, double *bmax, double *fl)
{
    int cnt = 0;
    double mn = INFINITY, mx = 0.0;
    for (int i = 0; i < n; i++) {
        double b;
        if (w[i] > 0.0 && isfinite(hi[i])) b = (hi[i] - x[i]) / w[i];
        else if (w[i] < 0.0 && isfinite(lo[i])) b = (lo[i] - x[i]) / w[i];
        else continue;
        *fl += 2.0;
        if (cnt == 0) { mn = b; mx = b; }
        else { if (b < mn) mn = b; if (b > mx) mx = b; }
        cnt++;
    }
    if (cnt == 0) mx = INFINITY;
    *nb = cnt; *bmin = mn; *bmax = mx;
}

void or_breakpt(int32_t n, const double *x, const double *lo, const double *hi, const double *w,
                int32_t *nbrpt, double *brptmin, double *brptmax)
{
    double fl = 0.0;
    int nb;
    breakpt_count(n, x, lo, hi, w, &nb, brptmin, brptmax, &fl);
    *nbrpt = nb;
}

/* trqsol: the sigma >= 0 with ||x + sigma p||_2 = delta, for ||x|| <= delta. The positive
 * root of ptp s^2 + 2 ptx s + (xtx - delta^2) = 0, written in the form that avoids
 * cancellation for either sign of ptx. */
static double trqsol_count(int m, const double *x, const double *p, double delta, double *fl)
{
    double ptx = dot(m, p, x, fl);
    double ptp = dot(m, p, p, fl);
    double xtx = dot(m, x, x, fl);
    double dsq = delta * delta;
    double disc = ptx * ptx + ptp * (dsq - xtx);
    if (disc < 0.0) disc = 0.0;
    double rad = sqrt(disc);
    double sigma;
    if (ptx >= 0.0) sigma = (dsq - xtx) / (ptx + rad);
    else sigma = (rad - ptx) / ptp;
    *fl += 9.0;
    return sigma > 0.0 ? sigma : 0.0;
}

double or_trqsol(int32_t m, const double *x, const double *p, double delta)
{
    double fl = 0.0;
    return trqsol_count(m, x, p, delta, &fl);
}

/* Component i of the projected gradient grad_[l,u] f (section 5.1). */
static double pg_comp(double x, double lo, double hi, double g)
{
    if (lo == hi) return 0.0;
    if (x <= lo) return g < 0.0 ? g : 0.0;
    if (x >= hi) return g > 0.0 ? g : 0.0;
    return g;
}

double or_projgrad_inf(int32_t n, const double *x, const double *lo, const double *hi,
                       const double *g)
{
    double m = 0.0;
    for (int i = 0; i < n; i++) {
        double v = fabs(pg_comp(x[i], lo[i], hi[i], g[i]));
        if (!(v <= m)) m = v; /* NaN propagates */
    }
    return m;
}

static double projgrad_nrm2(int n, const double *x, const double *lo, const double *hi,
                            const double *g)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) {
        double v = pg_comp(x[i], lo[i], hi[i], g[i]);
        s += v * v;
    }
    return sqrt(s);
}

/* ------------------------------------------------------------------------------------ */
/* Problem families.                                                                    */
/* ------------------------------------------------------------------------------------ */
int64_t or_param_size(int32_t family, int32_t n)
{
    if (family == OR_QP4) return (int64_t)n * (n + 1) / 2 + n + 1;
    if (family == OR_BR6) return 36;
    if (family == OR_BR8L) return 40;
    return 0;
}

/* QP4: f = 1/2 x'Qx + c'x + kappa sum x_i^4, parameters = packed lower triangle of Q
 * (row by row: Q00 Q10 Q11 Q20 ...), then c, then kappa. */
static double qp4_q(const double *p, int i, int j)
{
    if (j > i) { int t = i; i = j; j = t; }
    return p[i * (i + 1) / 2 + j];
}

static double qp4_f(int n, const double *p, const double *x, double *fl)
{
    const double *c = p + n * (n + 1) / 2;
    double kap = c[n];
    double quad = 0.0, lin = 0.0, quart = 0.0;
    for (int i = 0; i < n; i++) {
        double qi = 0.0;
        for (int j = 0; j < n; j++) qi += qp4_q(p, i, j) * x[j];
        quad += x[i] * qi;
        lin += c[i] * x[i];
        double x2 = x[i] * x[i];
        quart += x2 * x2;
    }
    *fl += 2.0 * n * n + 7.0 * n + 4.0;
    return 0.5 * quad + lin + kap * quart;
}

static void qp4_g(int n, const double *p, const double *x, double *g, double *fl)
{
    const double *c = p + n * (n + 1) / 2;
    double kap4 = 4.0 * c[n];
    for (int i = 0; i < n; i++) {
        double qi = 0.0;
        for (int j = 0; j < n; j++) qi += qp4_q(p, i, j) * x[j];
        g[i] = qi + c[i] + kap4 * x[i] * x[i] * x[i];
    }
    *fl += 2.0 * n * n + 5.0 * n + 1.0;
}

static void qp4_h(int n, const double *p, const double *x, double *h, double *fl)
{
    const double *c = p + n * (n + 1) / 2;
    double kap12 = 12.0 * c[n];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) h[i * n + j] = qp4_q(p, i, j);
    for (int i = 0; i < n; i++) h[i * n + i] += kap12 * x[i] * x[i];
    *fl += 3.0 * n + 1.0;
}

/* BR6: the branch subproblem (eq. exp-branch) in the variables
 *   x = (v_i, v_j, th_i, th_j, z_ij, z_ji),
 * with the flows of eqs. pij..qji at w_i = v_i^2, w_j = v_j^2, wR = v_i v_j cos(th_i - th_j),
 * wI = v_i v_j sin(th_i - th_j), and two flow copies z coupled to p_ij, p_ji by augmented-
 * Lagrangian terms (the paper's route from general constraints to bounds, section 1).
 * Parameters (36):
 *   [0..7]   g_ij b_ij gc_ij bc_ij g_ji b_ji gc_ji bc_ji
 *   [8..15]  targets of the couplings y = (p_ij q_ij p_ji q_ji w_i w_j th_i th_j)
 *   [16..23] multipliers lambda of the same couplings
 *   [24..25] multipliers mu_ij, mu_ji of z_ij - p_ij, z_ji - p_ji
 *   [26..33] penalties rho of the couplings, [34..35] penalties of the z couplings.
 * The objective is sum_k lambda_k (y_k - t_k) + rho_k/2 (y_k - t_k)^2
 *                + sum_lm mu_lm (z_lm - p_lm) + rho_lm/2 (z_lm - p_lm)^2.            */

/* Couplings y (8) and, when order >= 1, their gradients w.r.t. (v_i, v_j, th_i, th_j), and
 * when order >= 2, their Hessians. Each flow is a*own^2 + v_i v_j (al cos + be sin) with
 * (own, a, al, be) read off eqs. pij..qji. */
static void br6_couplings(const double *p, const double *x, int order, double y[8],
                          double dy[8][4], double d2y[8][4][4], double *fl)
{
    double vi = x[0], vj = x[1];
    double dth = x[2] - x[3];
    double cs = cos(dth), sn = sin(dth);
    double vv = vi * vj;
    *fl += 4.0;
    /* (own index, a, alpha, beta) for p_ij, q_ij, p_ji, q_ji */
    const int own[4] = {0, 0, 1, 1};
    double a[4] = {p[2], p[3], p[6], p[7]};
    double al[4] = {-p[0], -p[1], -p[4], -p[5]};
    double be[4] = {p[1], -p[0], -p[5], p[4]};
    if (order >= 1) memset(dy, 0, sizeof(double) * 8 * 4);
    if (order >= 2) memset(d2y, 0, sizeof(double) * 8 * 4 * 4);
    for (int k = 0; k < 4; k++) {
        double w = x[own[k]];
        double phi = al[k] * cs + be[k] * sn;
        y[k] = a[k] * w * w + vv * phi;
        *fl += 7.0;
        if (order >= 1) {
            double dphi = -al[k] * sn + be[k] * cs; /* d phi / d th_i */
            dy[k][0] = vj * phi;
            dy[k][1] = vi * phi;
            dy[k][own[k]] += 2.0 * a[k] * w;
            dy[k][2] = vv * dphi;
            dy[k][3] = -vv * dphi;
            *fl += 10.0;
            if (order >= 2) {
                double d2phi = -phi;
                d2y[k][own[k]][own[k]] = 2.0 * a[k];
                d2y[k][0][1] = d2y[k][1][0] = phi;
                d2y[k][0][2] = d2y[k][2][0] = vj * dphi;
                d2y[k][0][3] = d2y[k][3][0] = -vj * dphi;
                d2y[k][1][2] = d2y[k][2][1] = vi * dphi;
                d2y[k][1][3] = d2y[k][3][1] = -vi * dphi;
                d2y[k][2][2] = d2y[k][3][3] = vv * d2phi;
                d2y[k][2][3] = d2y[k][3][2] = -vv * d2phi;
                *fl += 8.0;
            }
        }
    }
    y[4] = vi * vi;
    y[5] = vj * vj;
    y[6] = x[2];
    y[7] = x[3];
    *fl += 2.0;
    if (order >= 1) {
        dy[4][0] = 2.0 * vi;
        dy[5][1] = 2.0 * vj;
        dy[6][2] = 1.0;
        dy[7][3] = 1.0;
        *fl += 2.0;
        if (order >= 2) {
            d2y[4][0][0] = 2.0;
            d2y[5][1][1] = 2.0;
        }
    }
}

void or_br6_flows(const double *params, const double *x, double *pq4)
{
    double y[8], fl = 0.0;
    br6_couplings(params, x, 0, y, NULL, NULL, &fl);
    for (int k = 0; k < 4; k++) pq4[k] = y[k];
}

static double br6_f(const double *p, const double *x, double *fl)
{
    double y[8];
    br6_couplings(p, x, 0, y, NULL, NULL, fl);
    double f = 0.0;
    for (int k = 0; k < 8; k++) {
        double e = y[k] - p[8 + k];
        f += p[16 + k] * e + 0.5 * p[26 + k] * e * e;
    }
    for (int s = 0; s < 2; s++) {
        double r = x[4 + s] - y[2 * s];
        f += p[24 + s] * r + 0.5 * p[34 + s] * r * r;
    }
    *fl += 8.0 * 7.0 + 2.0 * 7.0;
    return f;
}

static void br6_g(const double *p, const double *x, double *g, double *fl)
{
    double y[8], dy[8][4];
    br6_couplings(p, x, 1, y, dy, NULL, fl);
    for (int i = 0; i < 6; i++) g[i] = 0.0;
    for (int k = 0; k < 8; k++) {
        double coef = p[16 + k] + p[26 + k] * (y[k] - p[8 + k]);
        for (int i = 0; i < 4; i++) g[i] += coef * dy[k][i];
        *fl += 3.0 + 8.0;
    }
    for (int s = 0; s < 2; s++) {
        int pk = 2 * s;
        double coef = p[24 + s] + p[34 + s] * (x[4 + s] - y[pk]);
        /* grad of r = z - p_lm is e_z - grad p_lm */
        for (int i = 0; i < 4; i++) g[i] -= coef * dy[pk][i];
        g[4 + s] += coef;
        *fl += 3.0 + 9.0;
    }
}

static void br6_h(const double *p, const double *x, double *h, double *fl)
{
    double y[8], dy[8][4], d2y[8][4][4];
    br6_couplings(p, x, 2, y, dy, d2y, fl);
    for (int i = 0; i < 36; i++) h[i] = 0.0;
    for (int k = 0; k < 8; k++) {
        double rho = p[26 + k];
        double coef = p[16 + k] + rho * (y[k] - p[8 + k]);
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++)
                h[i * 6 + j] += rho * dy[k][i] * dy[k][j] + coef * d2y[k][i][j];
        *fl += 3.0 + 16.0 * 5.0;
    }
    for (int s = 0; s < 2; s++) {
        int pk = 2 * s, zi = 4 + s;
        double rho = p[34 + s];
        double coef = p[24 + s] + rho * (x[zi] - y[pk]);
        /* r = z - p: grad r = (-grad p, e_z); Hess r = -Hess p (on the first four) */
        double dr[6] = {0, 0, 0, 0, 0, 0};
        for (int i = 0; i < 4; i++) dr[i] = -dy[pk][i];
        dr[zi] = 1.0;
        for (int i = 0; i < 6; i++)
            for (int j = 0; j < 6; j++) h[i * 6 + j] += rho * dr[i] * dr[j];
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) h[i * 6 + j] -= coef * d2y[pk][i][j];
        *fl += 3.0 + 36.0 * 3.0 + 16.0 * 2.0;
    }
}

/* BR8L: the branch subproblem with the line limits p_lm^2 + q_lm^2 <= smax^2 (eq. LineLimit)
 * turned into equalities with slacks (the footnote of section 1 on inequalities):
 *   h_lm(x) = p_lm^2 + q_lm^2 + sigma_lm - smax^2 = 0,   sigma_lm >= 0,   lm in {ij, ji},
 * and added to the BR6 objective as the augmented-Lagrangian terms of section 1:
 *   f = f_BR6(x_0..5) + sum_lm lambda_lm h_lm + rho_h/2 h_lm^2.
 * x = (v_i, v_j, th_i, th_j, z_ij, z_ji, sigma_ij, sigma_ji); parameters: [0..35] as BR6,
 * [36] smax^2, [37] lambda_ij, [38] lambda_ji, [39] rho_h.                               */
static void br8l_limits(const double *p, const double *x, double hv[2])
{
    double y[8], fl = 0.0;
    br6_couplings(p, x, 0, y, NULL, NULL, &fl);
    for (int s = 0; s < 2; s++)
        hv[s] = y[2 * s] * y[2 * s] + y[2 * s + 1] * y[2 * s + 1] + x[6 + s] - p[36];
}

static double br8l_f(const double *p, const double *x, double *fl)
{
    double f = br6_f(p, x, fl);
    double hv[2];
    br8l_limits(p, x, hv);
    for (int s = 0; s < 2; s++) f += p[37 + s] * hv[s] + 0.5 * p[39] * hv[s] * hv[s];
    *fl += 2.0 * 5.0 + 2.0 * 5.0;
    return f;
}

static void br8l_g(const double *p, const double *x, double *g, double *fl)
{
    br6_g(p, x, g, fl);
    double y[8], dy[8][4];
    br6_couplings(p, x, 1, y, dy, NULL, fl);
    for (int s = 0; s < 2; s++) {
        int kp = 2 * s, kq = 2 * s + 1;
        double hv = y[kp] * y[kp] + y[kq] * y[kq] + x[6 + s] - p[36];
        double c = p[37 + s] + p[39] * hv;          /* d/dh of lambda h + rho/2 h^2 */
        for (int i = 0; i < 4; i++) g[i] += c * (2.0 * y[kp] * dy[kp][i] + 2.0 * y[kq] * dy[kq][i]);
        g[6 + s] = c;
        *fl += 6.0 + 4.0 * 6.0;
    }
}

static void br8l_h(const double *p, const double *x, double *h, double *fl)
{
    double h6[36];
    br6_h(p, x, h6, fl);
    for (int i = 0; i < 64; i++) h[i] = 0.0;
    for (int i = 0; i < 6; i++)
        for (int j = 0; j < 6; j++) h[i * 8 + j] = h6[i * 6 + j];
    double y[8], dy[8][4], d2y[8][4][4];
    br6_couplings(p, x, 2, y, dy, d2y, fl);
    for (int s = 0; s < 2; s++) {
        int kp = 2 * s, kq = 2 * s + 1, si = 6 + s;
        double hv = y[kp] * y[kp] + y[kq] * y[kq] + x[si] - p[36];
        double c = p[37 + s] + p[39] * hv;
        /* gradient of h_lm over all 8 variables */
        double u[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        for (int i = 0; i < 4; i++) u[i] = 2.0 * y[kp] * dy[kp][i] + 2.0 * y[kq] * dy[kq][i];
        u[si] = 1.0;
        /* rho_h grad h grad h' + c Hess h, Hess h = 2 sum_{k in p,q} (dy dy' + y d2y) */
        for (int i = 0; i < 8; i++)
            for (int j = 0; j < 8; j++) h[i * 8 + j] += p[39] * u[i] * u[j];
        for (int i = 0; i < 4; i++)
            for (int j = 0; j < 4; j++) {
                double hh = 2.0 * (dy[kp][i] * dy[kp][j] + y[kp] * d2y[kp][i][j] +
                                   dy[kq][i] * dy[kq][j] + y[kq] * d2y[kq][i][j]);
                h[i * 8 + j] += c * hh;
            }
        *fl += 6.0 + 4.0 * 6.0 + 64.0 * 3.0 + 16.0 * 11.0;
    }
}

/* HS45M: f = 120 - prod x_i with 0 <= x_i <= i (footnote of section 4.2). */
static double hs45_f(int n, const double *x, double *fl)
{
    double pr = 1.0;
    for (int i = 0; i < n; i++) pr *= x[i];
    *fl += n + 1.0;
    return 120.0 - pr;
}

static void hs45_g(int n, const double *x, double *g, double *fl)
{
    for (int i = 0; i < n; i++) {
        double pr = 1.0;
        for (int k = 0; k < n; k++) if (k != i) pr *= x[k];
        g[i] = -pr;
    }
    *fl += (double)n * (n - 1);
}

static void hs45_h(int n, const double *x, double *h, double *fl)
{
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) {
            if (i == j) { h[i * n + j] = 0.0; continue; }
            double pr = 1.0;
            for (int k = 0; k < n; k++) if (k != i && k != j) pr *= x[k];
            h[i * n + j] = -pr;
            *fl += n - 2.0;
        }
}

/* Minimal algorithmic counts of one evaluation (FAM_FLOPS). The solver evaluates f first
 * at every point, then the gradient at the same point, and the Hessian only at points
 * whose f and gradient it has, so the gradient and Hessian counts exclude what the
 * earlier evaluations at that point already formed.
 *   QP4  f: Qx 2n^2, x'Qx 2n, c'x 2n, x_i^2 and x_i^4 2n, their sum n, the combination 4
 *          = 2n^2 + 7n + 4;
 *        g (Qx and x_i^2 from f): + c n, x_i^3 n, 4 kappa 1, times x_i^3 n, add n = 4n + 1;
 *        H (Q as given, x_i^2 from f): 12 kappa 1, times x_i^2 n, add to Q_ii n = 2n + 1.
 *   BR6  shared: th_i - th_j 1, sin and cos 2, v_i v_j 1, v_i^2 and v_j^2 2, per flow
 *          phi = al cos + be sin 3 and a w_own + V phi 3 (four flows) = 30;
 *        f: ten residuals 10, ten terms (lambda + (rho/2) e) e 4 each, nine sums = 89;
 *        g: ten coefficients lambda + rho e 2 each 20, copy couplings folded into the p
 *          flows 2, dphi/dD 3 per flow 12, two 4-term sums over the flows 14, d/dv_i and
 *          d/dv_j 8 each 16, d/dth_i and d/dth_j 3 = 67;
 *        H: flow derivatives in (v_i, v_j, D) 6 per flow 24, Gauss-Newton weights of the
 *          p flows with their copies 2, per flow the six distinct (v_i, v_j, D) entries
 *          (weighted products 9, second derivatives 3, curvature terms 5, sums 11) 28 each
 *          112, the v^2 couplings 5 each 10, the angle couplings 2, the copy rows 6 = 156. */
static double fam_flops(int fam, int n, int which)
{
    if (fam == OR_QP4) {
        if (which == 0) return 2.0 * n * n + 7.0 * n + 4.0;
        if (which == 1) return 4.0 * n + 1.0;
        return 2.0 * n + 1.0;
    }
    /* OR_BR6 */
    if (which == 0) return 89.0;
    if (which == 1) return 67.0;
    return 156.0;
}

static double fam_f(int fam, int n, const double *p, const double *x, double *fl)
{
    double as_written = 0.0;
    if (fam == OR_QP4) { double v = qp4_f(n, p, x, &as_written); *fl += fam_flops(fam, n, 0); return v; }
    if (fam == OR_BR6) { double v = br6_f(p, x, &as_written); *fl += fam_flops(fam, n, 0); return v; }
    if (fam == OR_BR8L) return br8l_f(p, x, fl);
    return hs45_f(n, x, fl);
}

static void fam_g(int fam, int n, const double *p, const double *x, double *g, double *fl)
{
    double as_written = 0.0;
    if (fam == OR_QP4) { qp4_g(n, p, x, g, &as_written); *fl += fam_flops(fam, n, 1); }
    else if (fam == OR_BR6) { br6_g(p, x, g, &as_written); *fl += fam_flops(fam, n, 1); }
    else if (fam == OR_BR8L) br8l_g(p, x, g, fl);
    else hs45_g(n, x, g, fl);
}

static void fam_h(int fam, int n, const double *p, const double *x, double *h, double *fl)
{
    double as_written = 0.0;
    if (fam == OR_QP4) { qp4_h(n, p, x, h, &as_written); *fl += fam_flops(fam, n, 2); }
    else if (fam == OR_BR6) { br6_h(p, x, h, &as_written); *fl += fam_flops(fam, n, 2); }
    else if (fam == OR_BR8L) br8l_h(p, x, h, fl);
    else hs45_h(n, x, h, fl);
}

double or_family_flops(int32_t family, int32_t n, int32_t which)
{
    if (family != OR_QP4 && family != OR_BR6) return -1.0;
    if (which < 0 || which > 2) return -1.0;
    return fam_flops(family, n, which);
}

double or_eval_f(int32_t family, int32_t n, const double *params, const double *x)
{
    double fl = 0.0;
    return fam_f(family, n, params, x, &fl);
}

void or_eval_g(int32_t family, int32_t n, const double *params, const double *x, double *g)
{
    double fl = 0.0;
    fam_g(family, n, params, x, g, &fl);
}

void or_eval_h(int32_t family, int32_t n, const double *params, const double *x, double *h)
{
    double fl = 0.0;
    fam_h(family, n, params, x, h, &fl);
}

/* ------------------------------------------------------------------------------------ */
/* TRON steps.                                                                          */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int n;
    const double *lo, *hi;
    double *x, *g, *gt, *H;       /* iterate, gradient, trial gradient, Hessian (n x n)  */
    double *xs, *s, *xt, *st;     /* subspace point, its step, trial point, trial step   */
    double *r, *w, *d, *hv;       /* model gradient, search direction, search step, H*v  */
    int *idx;                     /* free set                                             */
    double *A, *L;                /* m x m block of H and its factor                       */
    double *rF, *rh, *sh, *pp, *z, *yv, *qh, *tv, *wF;
    int *lidx;                    /* free set of the last factored pass (L is its factor)  */
    int lm;                       /* its size; 0 when no pass factored this iteration      */
    double fl;                    /* algorithmic flops                                     */
    int cauchy_trials, search_trials, passes, cg_iters, chol_tries;
} ws_t;

/* One Cauchy trial (section 3, Algorithm 1 Cauchy step): x_t = P[x - alpha g], s_t = x_t - x.
 * Acceptable when ||s_t||_2 <= delta and q(s_t) <= mu0 g's_t, q(s) = g's + s'Hs/2.   */
static int cauchy_ok(ws_t *w, double alpha, double delta)
{
    int n = w->n;
    w->cauchy_trials++;
    gpstep_pt(n, w->x, w->lo, w->hi, -alpha, w->g, w->xt, w->st, &w->fl);
    double sn = nrm2(n, w->st, &w->fl);
    if (!(sn <= delta)) return 0;
    gemv(n, w->H, w->st, w->hv, &w->fl);
    double gts = dot(n, w->g, w->st, &w->fl);
    double q = gts + 0.5 * dot(n, w->st, w->hv, &w->fl);
    w->fl += 3.0;
    return q <= MU0 * gts;
}

/* Cauchy step (reading S4): start from the previous alpha_c; if it is acceptable, multiply
 * by 10 while the new value stays acceptable and alpha is below the largest breakpoint along
 * -g; otherwise multiply by 0.1 until acceptable. Leaves xs = P[x - alpha g]. */
static double cauchy_step(ws_t *w, double delta, double alpha)
{
    int n = w->n, nb;
    double bmin, bmax;
    for (int i = 0; i < n; i++) w->d[i] = -w->g[i];
    breakpt_count(n, w->x, w->lo, w->hi, w->d, &nb, &bmin, &bmax, &w->fl);
    if (cauchy_ok(w, alpha, delta)) {
        memcpy(w->xs, w->xt, sizeof(double) * n);
        for (int t = 0; t < CAUCHY_MAX; t++) {
            if (!(alpha < bmax)) break;
            double a2 = 10.0 * alpha;
            w->fl += 1.0;
            if (!cauchy_ok(w, a2, delta)) break;
            alpha = a2;
            memcpy(w->xs, w->xt, sizeof(double) * n);
        }
    } else {
        for (int t = 0; t < CAUCHY_MAX; t++) {
            alpha = 0.1 * alpha;
            w->fl += 1.0;
            if (cauchy_ok(w, alpha, delta)) break;
        }
        memcpy(w->xs, w->xt, sizeof(double) * n);
    }
    return alpha;
}

/* Preconditioner (Algorithm 1, "L L^T = A + alpha I for some alpha >= 0"; reading S7):
 * alpha = 0 when every diagonal entry of A is positive, otherwise beta - min A_ii with
 * beta = 1e-3 max(1, max |A_ii|); on failure alpha <- max(2 alpha, beta). After
 * SHIFT_TRIES failures L = diag(sqrt(max(|A_ii|, beta))). Returns the shift used. */
static double precond(ws_t *w, int m)
{
    double dmin = w->A[0], dmax = 0.0;
    for (int a = 0; a < m; a++) {
        double v = w->A[a * m + a];
        if (v < dmin) dmin = v;
        if (fabs(v) > dmax) dmax = fabs(v);
    }
    double beta = 1e-3 * (dmax > 1.0 ? dmax : 1.0);
    double alpha = dmin > 0.0 ? 0.0 : beta - dmin;
    w->fl += 2.0;
    for (int t = 0; t < SHIFT_TRIES; t++) {
        w->chol_tries++;
        if (ccf_count(m, w->A, alpha, w->L, &w->fl) == 0) return alpha;
        alpha = 2.0 * alpha > beta ? 2.0 * alpha : beta;
        w->fl += 1.0;
    }
    for (int i = 0; i < m * m; i++) w->L[i] = 0.0;
    for (int a = 0; a < m; a++) {
        double v = fabs(w->A[a * m + a]);
        w->L[a * m + a] = sqrt(v > beta ? v : beta);
    }
    w->fl += m;
    return alpha;
}

enum { CG_CONVERGED = 0, CG_MAXIT = 1, CG_NEGCURV = 2, CG_BOUNDARY = 3 };

/* Trust-region preconditioned CG (Algorithm 1 CG step; section 3; Steihaug). Solves
 * L^-1 A L^-T s_hat = -L^-1 r within ||s_hat||_2 <= delta (readings S5, S6, S9, S10):
 *   stop after |F| iterations, on negative curvature, at the boundary, or when the
 *   residual drops below cg_rtol times its initial norm. Result in w->sh.
 * exact (reading S33): the preconditioner needed no shift, so L L^T = A and the
 *   preconditioned matrix is the identity; section 3 notes that CG then ends after one
 *   iteration, whose step along p = r_hat has length exactly 1: s_hat = r_hat, or the
 *   boundary point along it when ||r_hat|| >= delta. That step is taken directly.       */
static int pcg(ws_t *w, int m, double delta, double cg_rtol, int exact)
{
    for (int a = 0; a < m; a++) {
        w->rh[a] = -w->rF[a];
        w->sh[a] = 0.0;
    }
    trsv_fwd(m, w->L, w->rh, &w->fl);
    memcpy(w->pp, w->rh, sizeof(double) * m);
    double rr = dot(m, w->rh, w->rh, &w->fl);
    if (rr == 0.0) return CG_CONVERGED;
    if (exact) {
        w->cg_iters++;
        w->fl += 1.0;                                  /* delta^2 */
        if (rr >= delta * delta) {
            double sig = trqsol_count(m, w->sh, w->pp, delta, &w->fl);
            axpy(m, sig, w->pp, w->sh, &w->fl);
            return CG_BOUNDARY;
        }
        memcpy(w->sh, w->pp, sizeof(double) * m);
        return CG_CONVERGED;
    }
    double tol = cg_rtol * sqrt(rr);
    w->fl += 2.0;
    for (int j = 0; j < m; j++) {
        w->cg_iters++;
        memcpy(w->z, w->pp, sizeof(double) * m);
        trsv_bwd(m, w->L, w->z, &w->fl);               /* z = L^-T p     */
        gemv(m, w->A, w->z, w->yv, &w->fl);            /* y = A z        */
        memcpy(w->qh, w->yv, sizeof(double) * m);
        trsv_fwd(m, w->L, w->qh, &w->fl);              /* q = L^-1 y     */
        double kap = dot(m, w->pp, w->qh, &w->fl);
        if (!(kap > 0.0)) {
            double sig = trqsol_count(m, w->sh, w->pp, delta, &w->fl);
            axpy(m, sig, w->pp, w->sh, &w->fl);
            return CG_NEGCURV;
        }
        double alpha = rr / kap;
        w->fl += 1.0;
        memcpy(w->tv, w->sh, sizeof(double) * m);
        axpy(m, alpha, w->pp, w->tv, &w->fl);
        if (nrm2(m, w->tv, &w->fl) >= delta) {
            double sig = trqsol_count(m, w->sh, w->pp, delta, &w->fl);
            axpy(m, sig, w->pp, w->sh, &w->fl);
            return CG_BOUNDARY;
        }
        memcpy(w->sh, w->tv, sizeof(double) * m);
        axpy(m, -alpha, w->qh, w->rh, &w->fl);
        double rrn = dot(m, w->rh, w->rh, &w->fl);
        w->fl += 1.0;
        if (sqrt(rrn) <= tol) return CG_CONVERGED;
        double bet = rrn / rr;
        for (int a = 0; a < m; a++) w->pp[a] = w->rh[a] + bet * w->pp[a];
        w->fl += 1.0 + 2.0 * m;
        rr = rrn;
    }
    return CG_MAXIT;
}

/* Projected search along w from the subspace point xs (Algorithm 1, projected line search;
 * reading S13): the first beta in 1, 1/2, ..., 2^-20 with
 *   q(s + d) - q(s) = r'd + d'Hd/2 <= mu0 r'd,   d = P[xs + beta w] - xs,
 * where r = g + H s is the model gradient at xs. On acceptance xs moves to P[xs + beta w];
 * otherwise it stays. Returns 1 on acceptance; *beta_out is the last beta tried. */
static int projected_search(ws_t *w, double *beta_out)
{
    int n = w->n;
    double beta = 1.0, tried = 1.0;
    int acc = 0;
    for (int t = 0; t <= SEARCH_HALVINGS; t++) {
        w->search_trials++;
        tried = beta;
        gpstep_pt(n, w->xs, w->lo, w->hi, beta, w->w, w->xt, w->d, &w->fl);
        gemv(n, w->H, w->d, w->hv, &w->fl);
        double rd = dot(n, w->r, w->d, &w->fl);
        double dq = rd + 0.5 * dot(n, w->d, w->hv, &w->fl);
        w->fl += 3.0;
        if (dq <= MU0 * rd) { acc = 1; break; }
        beta *= 0.5;
        w->fl += 1.0;
    }
    if (acc) memcpy(w->xs, w->xt, sizeof(double) * n);
    *beta_out = tried;
    return acc;
}

/* Subspace passes (Algorithm 1: free set, preconditioner, CG, back-transform, projected
 * search; reading S13). Starts from xs (the Cauchy point) and moves it. */
static void subspace(ws_t *w, double delta, double cg_rtol)
{
    int n = w->n;
    w->lm = 0;
    for (int pass = 0; pass < n; pass++) {
        int m = 0;
        for (int i = 0; i < n; i++)
            if (w->lo[i] < w->xs[i] && w->xs[i] < w->hi[i]) w->idx[m++] = i;
        if (m == 0) break;
        w->passes++;
        /* model gradient at the current step: r = g + H s, s = xs - x */
        for (int i = 0; i < n; i++) w->s[i] = w->xs[i] - w->x[i];
        gemv(n, w->H, w->s, w->r, &w->fl);
        for (int i = 0; i < n; i++) w->r[i] += w->g[i];
        w->fl += n;
        for (int a = 0; a < m; a++) {
            w->rF[a] = w->r[w->idx[a]];
            for (int b = 0; b < m; b++) w->A[a * m + b] = w->H[w->idx[a] * n + w->idx[b]];
        }
        double shift = precond(w, m);
        w->lm = m;
        memcpy(w->lidx, w->idx, sizeof(int) * m);
        int ex = pcg(w, m, delta, cg_rtol, shift == 0.0);
        memcpy(w->wF, w->sh, sizeof(double) * m);
        trsv_bwd(m, w->L, w->wF, &w->fl);              /* w = L^-T s_hat */
        for (int i = 0; i < n; i++) w->w[i] = 0.0;
        for (int a = 0; a < m; a++) w->w[w->idx[a]] = w->wF[a];
        double beta;
        projected_search(w, &beta);
        int newly_bound = 0;
        for (int a = 0; a < m; a++) {
            int i = w->idx[a];
            if (!(w->lo[i] < w->xs[i] && w->xs[i] < w->hi[i])) newly_bound = 1;
        }
        if (!((ex == CG_CONVERGED || ex == CG_MAXIT) && newly_bound)) break;
    }
}

/* Length of the step s in the norm of the trust region that bounded it (reading S31): the
 * conjugate-gradient step is bounded by ||L^T w|| <= delta (Algorithm 1 CG step), so on the
 * free set of the last factored pass the step is measured as ||L^T s_F||, and outside it
 * in the Euclidean norm. With no factored pass this is ||s||_2. */
static double step_norm(ws_t *w)
{
    int n = w->n, m = w->lm;
    if (m == 0) return nrm2(n, w->s, &w->fl);
    double ss = 0.0;
    for (int a = 0; a < m; a++) {
        double t = 0.0;
        for (int b = a; b < m; b++) t += w->L[b * m + a] * w->s[w->lidx[b]];
        ss += t * t;
    }
    int k = 0;
    for (int i = 0; i < n; i++) {
        if (k < m && w->lidx[k] == i) { k++; continue; }
        ss += w->s[i] * w->s[i];
    }
    w->fl += (double)m * (m + 1) + 2.0 * n + 1.0;
    return sqrt(ss);
}

/* Radius update after a trial (reading S2, the interval rule of TRON). */
static double radius_update(double delta, double rho, double f, double ft, double gts,
                            double snorm, int finite_trial, double *fl)
{
    double astar;
    if (!finite_trial) {
        astar = SIG1;
        rho = -INFINITY;
    } else {
        double gam = ft - f - gts;
        *fl += 2.0;
        if (gam <= 0.0) astar = SIG3;
        else {
            astar = -0.5 * gts / gam;
            if (astar < SIG1) astar = SIG1;
            *fl += 2.0;
        }
    }
    double nd;
    if (rho <= ETA0) {
        double a = astar > SIG1 ? astar : SIG1;
        double t1 = a * snorm, t2 = SIG2 * delta;
        nd = t1 < t2 ? t1 : t2;
    } else if (rho <= ETA1) {
        double t1 = astar * snorm, t2 = SIG2 * delta;
        double mn = t1 < t2 ? t1 : t2;
        nd = SIG1 * delta > mn ? SIG1 * delta : mn;
    } else if (rho < ETA2) {
        double t1 = astar * snorm, t2 = SIG3 * delta;
        double mn = t1 < t2 ? t1 : t2;
        nd = SIG1 * delta > mn ? SIG1 * delta : mn;
    } else {
        double t1 = astar * snorm, t2 = SIG3 * delta;
        double mn = t1 < t2 ? t1 : t2;
        nd = delta > mn ? delta : mn;
    }
    *fl += 3.0;
    return nd;
}

/* Actual reduction of a trial with finite f(x + s) (reading S30): f - ft, except when the
 * predicted reduction is at the rounding level of f, pred <= 1e-10 max(1, |f|); the
 * difference f - ft is then noise and the reduction is taken from the gradients at both
 * ends, -(g + gt)'s / 2 (the trapezoid rule, exact when f is quadratic along s). */
static double actual_reduction(int n, double f, double ft, double pred, const double *g,
                               const double *gt, const double *s, double *fl)
{
    if (pred <= ARED_SWITCH * (fabs(f) > 1.0 ? fabs(f) : 1.0)) {
        double sg = 0.0;
        for (int i = 0; i < n; i++) sg += (g[i] + gt[i]) * s[i];
        *fl += 3.0 * n + 1.0;
        return -0.5 * sg;
    }
    return f - ft;
}

static int all_finite(int n, const double *v)
{
    for (int i = 0; i < n; i++) if (!isfinite(v[i])) return 0;
    return 1;
}

/* One instance of Algorithm 1 with the ratio test and radius update of TRON. */
static int tron_one(int fam, int n, const double *prm, const double *lo, const double *hi,
                    const double *x0, double *xout, double *fout, double *delta_io,
                    double *alphac_io, const or_opts *o, double *st)
{
    size_t nv = (size_t)n;
    size_t need = nv * 15 + nv * nv * 3 + nv * 10;
    double *buf = (double *)calloc(need + 8, sizeof(double));
    int *idx = (int *)calloc(2 * nv + 2, sizeof(int));
    ws_t w;
    memset(&w, 0, sizeof(w));
    w.n = n; w.lo = lo; w.hi = hi; w.idx = idx; w.lidx = idx + nv + 1;
    double *q = buf;
    w.x = q; q += nv; w.g = q; q += nv; w.gt = q; q += nv; w.xs = q; q += nv; w.s = q; q += nv;
    w.xt = q; q += nv; w.st = q; q += nv; w.r = q; q += nv; w.w = q; q += nv;
    w.d = q; q += nv; w.hv = q; q += nv;
    w.H = q; q += nv * nv; w.A = q; q += nv * nv; w.L = q; q += nv * nv;
    w.rF = q; q += nv; w.rh = q; q += nv; w.sh = q; q += nv; w.pp = q; q += nv;
    w.z = q; q += nv; w.yv = q; q += nv; w.qh = q; q += nv; w.tv = q; q += nv;
    w.wF = q; q += nv;

    int status = OR_CONVERGED, k = 0, accepted = 0;
    double f = NAN, delta = 0.0, alphac = 1.0;

    for (int i = 0; i < n; i++)
        if (!(lo[i] <= hi[i])) status = OR_BAD_BOUNDS;
    if (status == OR_BAD_BOUNDS) {
        memcpy(xout, x0, sizeof(double) * nv);
        *fout = NAN;
        goto done;
    }
    /* start (reading S16): project x0 onto the box, then check convergence at x^0 */
    for (int i = 0; i < n; i++) w.x[i] = proj1(x0[i], lo[i], hi[i]);
    f = fam_f(fam, n, prm, w.x, &w.fl);
    fam_g(fam, n, prm, w.x, w.g, &w.fl);
    if (!isfinite(f) || !all_finite(n, w.g)) { status = OR_NONFINITE; goto out; }
    if (or_projgrad_inf(n, w.x, lo, hi, w.g) <= o->gtol) { status = OR_CONVERGED; goto out; }
    /* initial radius (reading S3) and Cauchy parameter */
    if (o->use_warm && delta_io && *delta_io > 0.0) delta = *delta_io;
    else if (o->delta0 > 0.0) delta = o->delta0;
    else {
        delta = projgrad_nrm2(n, w.x, lo, hi, w.g);
        w.fl += 2.0 * n + 1.0;
        if (delta == 0.0) delta = 1.0;
    }
    if (o->use_warm && alphac_io && *alphac_io > 0.0) alphac = *alphac_io;
    fam_h(fam, n, prm, w.x, w.H, &w.fl);

    for (;;) {
        /* Cauchy point, then the subspace passes from it */
        alphac = cauchy_step(&w, delta, alphac);
        subspace(&w, delta, o->cg_rtol);
        /* trial point and model reduction */
        for (int i = 0; i < n; i++) w.s[i] = w.xs[i] - w.x[i];
        w.fl += n;
        double snorm = step_norm(&w);
        gemv(n, w.H, w.s, w.hv, &w.fl);
        double gts = dot(n, w.g, w.s, &w.fl);
        double qs = gts + 0.5 * dot(n, w.s, w.hv, &w.fl);
        double pred = -qs;
        w.fl += 2.0;
        k++;
        if (!(pred > 0.0)) { status = OR_STALLED; break; }
        /* trial values: f and its gradient at the trial point */
        double ft = fam_f(fam, n, prm, w.xs, &w.fl);
        int fin = isfinite(ft);
        double ared = f - ft;
        w.fl += 1.0;
        if (fin) {
            fam_g(fam, n, prm, w.xs, w.gt, &w.fl);
            ared = actual_reduction(n, f, ft, pred, w.g, w.gt, w.s, &w.fl);
        }
        double rho = fin ? ared / pred : -INFINITY;
        w.fl += 1.0;
        delta = radius_update(delta, rho, f, f - ared, gts, snorm, fin, &w.fl);
        if (rho > ETA0) {
            memcpy(w.x, w.xs, sizeof(double) * nv);
            memcpy(w.g, w.gt, sizeof(double) * nv);
            f = ft;
            accepted++;
        }
        if (!isfinite(f) || !all_finite(n, w.g)) { status = OR_NONFINITE; break; }
        if (or_projgrad_inf(n, w.x, lo, hi, w.g) <= o->gtol) { status = OR_CONVERGED; break; }
        if (k >= o->max_iter) { status = OR_MAX_ITER; break; }
        double tiny = STALL_REL * (fabs(f) > 1.0 ? fabs(f) : 1.0);
        if (fin && fabs(ared) <= tiny && pred <= tiny) { status = OR_STALLED; break; }
        if (rho > ETA0) fam_h(fam, n, prm, w.x, w.H, &w.fl);
    }
out:
    memcpy(xout, w.x, sizeof(double) * nv);
    *fout = f;
done:
    if (delta_io) *delta_io = delta;
    if (alphac_io) *alphac_io = alphac;
    if (st) {
        st[0] = w.fl; st[1] = k; st[2] = w.cg_iters; st[3] = w.chol_tries;
        st[4] = w.cauchy_trials; st[5] = w.search_trials; st[6] = w.passes; st[7] = accepted;
    }
    free(buf);
    free(idx);
    return status;
}

/* Subspace CG on one dense block, for the tests. */
int32_t or_subspace_cg(int32_t m, const double *a, const double *r, double delta, double cg_rtol,
                       double *wout, double *shat, int32_t *iters, double *shift_out)
{
    ws_t w;
    memset(&w, 0, sizeof(w));
    size_t mv = (size_t)m;
    double *buf = (double *)calloc(mv * mv * 2 + mv * 10 + 8, sizeof(double));
    double *q = buf;
    w.A = q; q += mv * mv; w.L = q; q += mv * mv;
    w.rF = q; q += mv; w.rh = q; q += mv; w.sh = q; q += mv; w.pp = q; q += mv;
    w.z = q; q += mv; w.yv = q; q += mv; w.qh = q; q += mv; w.tv = q; q += mv;
    memcpy(w.A, a, sizeof(double) * mv * mv);
    memcpy(w.rF, r, sizeof(double) * mv);
    double shift = precond(&w, m);
    int ex = pcg(&w, m, delta, cg_rtol, shift == 0.0);
    memcpy(shat, w.sh, sizeof(double) * mv);
    memcpy(wout, w.sh, sizeof(double) * mv);
    double fl = 0.0;
    trsv_bwd(m, w.L, wout, &fl);
    *iters = w.cg_iters;
    *shift_out = shift;
    free(buf);
    return ex;
}

/* ------------------------------------------------------------------------------------ */
/* Single steps of one TRON iteration, exposed for the tests.                            */
/* ------------------------------------------------------------------------------------ */
static ws_t step_ws(int n, const double *lo, const double *hi, double *buf)
{
    ws_t w;
    memset(&w, 0, sizeof(w));
    w.n = n; w.lo = lo; w.hi = hi;
    double *q = buf;
    w.x = q; q += n; w.g = q; q += n; w.xs = q; q += n; w.s = q; q += n; w.xt = q; q += n;
    w.st = q; q += n; w.r = q; q += n; w.w = q; q += n; w.d = q; q += n; w.hv = q; q += n;
    w.H = q;
    return w;
}

double or_radius_update(double delta, double rho, double f, double ft, double gts, double snorm,
                        int32_t finite_trial)
{
    double fl = 0.0;
    return radius_update(delta, rho, f, ft, gts, snorm, finite_trial, &fl);
}

double or_cauchy_step(int32_t n, const double *x, const double *lo, const double *hi,
                      const double *g, const double *h, double delta, double alpha,
                      double *xs_out, int32_t *trials)
{
    double *buf = (double *)calloc((size_t)n * 10 + (size_t)n * n + 1, sizeof(double));
    ws_t w = step_ws(n, lo, hi, buf);
    memcpy(w.x, x, sizeof(double) * n);
    memcpy(w.g, g, sizeof(double) * n);
    memcpy(w.H, h, sizeof(double) * n * n);
    double a = cauchy_step(&w, delta, alpha);
    memcpy(xs_out, w.xs, sizeof(double) * n);
    *trials = w.cauchy_trials;
    free(buf);
    return a;
}

int32_t or_projected_search(int32_t n, const double *xs, const double *lo, const double *hi,
                            const double *dir, const double *r, const double *h,
                            double *xs_out, double *beta_out, int32_t *trials)
{
    double *buf = (double *)calloc((size_t)n * 10 + (size_t)n * n + 1, sizeof(double));
    ws_t w = step_ws(n, lo, hi, buf);
    memcpy(w.xs, xs, sizeof(double) * n);
    memcpy(w.w, dir, sizeof(double) * n);
    memcpy(w.r, r, sizeof(double) * n);
    memcpy(w.H, h, sizeof(double) * n * n);
    int acc = projected_search(&w, beta_out);
    memcpy(xs_out, w.xs, sizeof(double) * n);
    *trials = w.search_trials;
    free(buf);
    return acc;
}

double or_step_norm(int32_t n, const double *s, int32_t m, const int32_t *free_idx,
                    const double *l)
{
    ws_t w;
    memset(&w, 0, sizeof(w));
    int *idx = (int *)calloc((size_t)(m > 0 ? m : 1), sizeof(int));
    for (int a = 0; a < m; a++) idx[a] = free_idx[a];
    w.n = n; w.lm = m; w.lidx = idx; w.L = (double *)l; w.s = (double *)s;
    double v = step_norm(&w);
    free(idx);
    return v;
}

double or_actual_reduction(int32_t n, double f, double ft, double pred, const double *g,
                           const double *gt, const double *s)
{
    double fl = 0.0;
    return actual_reduction(n, f, ft, pred, g, gt, s, &fl);
}

/* f and the infinity norm of the projected gradient at given points, instance by instance
 * (packed like or_tron_batch), for the parity checks. */
void or_eval_batch(int32_t family, int64_t batch, const int32_t *n_per, int32_t n_uniform,
                   const double *params, const double *lo, const double *hi, const double *x,
                   double *f_out, double *pg_out)
{
    int64_t po = 0, vo = 0;
    double *g = NULL;
    int gcap = 0;
    for (int64_t b = 0; b < batch; b++) {
        int n = n_per ? n_per[b] : n_uniform;
        if (n > gcap) {
            free(g);
            gcap = n;
            g = (double *)malloc(sizeof(double) * (size_t)gcap);
        }
        double fl = 0.0;
        f_out[b] = fam_f(family, n, params + po, x + vo, &fl);
        fam_g(family, n, params + po, x + vo, g, &fl);
        pg_out[b] = or_projgrad_inf(n, x + vo, lo + vo, hi + vo, g);
        po += or_param_size(family, n);
        vo += n;
    }
    free(g);
}

/* ------------------------------------------------------------------------------------ */
/* Batch driver: instances are claimed from an atomic counter by host threads.          */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int fam;
    int64_t batch;
    const int32_t *n_per;
    int32_t n_uniform;
    const int64_t *poff, *voff;
    const double *params, *lo, *hi, *x0;
    double *x, *f, *delta, *alphac, *stats;
    int32_t *status, *iters;
    const or_opts *opt;
    atomic_llong next;
} job_t;

static void *worker(void *arg)
{
    job_t *j = (job_t *)arg;
    for (;;) {
        long long b = atomic_fetch_add(&j->next, 1);
        if (b >= j->batch) break;
        int n = j->n_per ? j->n_per[b] : j->n_uniform;
        int64_t po = j->poff[b], vo = j->voff[b];
        double st[OR_NSTAT];
        int code = tron_one(j->fam, n, j->params + po, j->lo + vo, j->hi + vo, j->x0 + vo,
                            j->x + vo, j->f + b, j->delta ? j->delta + b : NULL,
                            j->alphac ? j->alphac + b : NULL, j->opt, st);
        j->status[b] = code;
        j->iters[b] = (int32_t)st[1];
        if (j->stats) memcpy(j->stats + b * OR_NSTAT, st, sizeof(st));
    }
    return NULL;
}

int32_t or_tron_batch(int32_t family, int64_t batch, const int32_t *n_per, int32_t n_uniform,
                      const double *params, const double *lo, const double *hi, const double *x0,
                      double *x, double *f, int32_t *status, int32_t *iters,
                      double *delta, double *alphac, double *stats,
                      const or_opts *opt, int32_t nthreads)
{
    if (batch <= 0) return 0;
    int64_t *poff = (int64_t *)malloc(sizeof(int64_t) * batch);
    int64_t *voff = (int64_t *)malloc(sizeof(int64_t) * batch);
    int64_t pacc = 0, vacc = 0;
    for (int64_t b = 0; b < batch; b++) {
        int n = n_per ? n_per[b] : n_uniform;
        poff[b] = pacc;
        voff[b] = vacc;
        pacc += or_param_size(family, n);
        vacc += n;
    }
    job_t j;
    j.fam = family; j.batch = batch; j.n_per = n_per; j.n_uniform = n_uniform;
    j.poff = poff; j.voff = voff; j.params = params; j.lo = lo; j.hi = hi; j.x0 = x0;
    j.x = x; j.f = f; j.delta = delta; j.alphac = alphac; j.stats = stats;
    j.status = status; j.iters = iters; j.opt = opt;
    atomic_init(&j.next, 0);
    int nt = nthreads;
    if (nt <= 0) nt = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > batch) nt = (int)batch;
    if (nt == 1) worker(&j);
    else {
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nt);
        for (int t = 0; t < nt; t++) pthread_create(&th[t], NULL, worker, &j);
        for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
        free(th);
    }
    free(poff);
    free(voff);
    return nt;
}

/* ------------------------------------------------------------------------------------ */
/* Augmented-Lagrangian outer loop for the equality constraints of a BR8L instance        */
/* (section 1: a sequence of bound-constrained minimisations of L_rho(x; lambda, rho) with */
/* updates of (lambda, rho) between them). The paper leaves the update scheme to the      */
/* literature it cites; reading S32 takes the first-order multiplier update with a penalty */
/* increase when the violation did not shrink enough:                                    */
/*   solve min_{l<=x<=u} L_rho(x; lambda) from the last x (warm radius after the first);  */
/*   v = ||h(x)||_inf; stop when v <= ctol;                                               */
/*   lambda <- lambda + rho h(x);                                                         */
/*   rho <- min(growth * rho, rho_max) when v > decrease * v_previous.                    */
/* The cap keeps the bound-constrained problems solvable to gtol: the gradient of the     */
/* penalty term carries rounding noise of order rho * eps * |smax^2| * |grad h|.           */
/* ------------------------------------------------------------------------------------ */
static int al_one(const double *prm_in, const double *lo, const double *hi, const double *x0,
                  double *prm_out, double *xout, double *fout, int32_t *iters, int32_t *outer,
                  double *viol, const or_opts *o, const or_al_opts *al)
{
    double prm[40];
    memcpy(prm, prm_in, sizeof(prm));
    double xc[8], delta = 0.0, alphac = 0.0, f = NAN, v = INFINITY, vprev = INFINITY;
    memcpy(xc, x0, sizeof(xc));
    or_opts oi = *o;
    int status = OR_AL_MAX_OUTER, total = 0, k = 0;
    for (k = 0; k < al->outer_max; k++) {
        double xn[8], st[OR_NSTAT];
        int code = tron_one(OR_BR8L, 8, prm, lo, hi, xc, xn, &f, &delta, &alphac, &oi, st);
        total += (int)st[1];
        memcpy(xc, xn, sizeof(xc));
        oi.use_warm = 1;
        if (code != OR_CONVERGED) { status = code; k++; break; }
        double hv[2];
        br8l_limits(prm, xc, hv);
        v = fabs(hv[0]) > fabs(hv[1]) ? fabs(hv[0]) : fabs(hv[1]);
        if (!(v == v)) { status = OR_NONFINITE; k++; break; }
        if (v <= al->ctol) { status = OR_CONVERGED; k++; break; }
        prm[37] += prm[39] * hv[0];
        prm[38] += prm[39] * hv[1];
        if (v > al->decrease * vprev) {
            double r = prm[39] * al->rho_growth;
            prm[39] = r < al->rho_max ? r : al->rho_max;
        }
        vprev = v;
    }
    memcpy(prm_out, prm, sizeof(prm));
    memcpy(xout, xc, sizeof(xc));
    *fout = f;
    *iters = total;
    *outer = k;
    *viol = v;
    return status;
}

typedef struct {
    int64_t batch;
    double *params;
    const double *lo, *hi, *x0;
    double *x, *f, *viol;
    int32_t *status, *iters, *outer;
    const or_opts *opt;
    const or_al_opts *al;
    atomic_llong next;
} al_job_t;

static void *al_worker(void *arg)
{
    al_job_t *j = (al_job_t *)arg;
    for (;;) {
        long long b = atomic_fetch_add(&j->next, 1);
        if (b >= j->batch) break;
        double *pb = j->params + 40 * b;
        j->status[b] = al_one(pb, j->lo + 8 * b, j->hi + 8 * b, j->x0 + 8 * b, pb, j->x + 8 * b,
                              j->f + b, j->iters + b, j->outer + b, j->viol + b, j->opt, j->al);
    }
    return NULL;
}

int32_t or_al_batch(int64_t batch, double *params, const double *lo, const double *hi,
                    const double *x0, double *x, double *f, int32_t *status, int32_t *iters,
                    int32_t *outer, double *viol, const or_opts *opt, const or_al_opts *al,
                    int32_t nthreads)
{
    if (batch <= 0) return 0;
    al_job_t j;
    j.batch = batch; j.params = params; j.lo = lo; j.hi = hi; j.x0 = x0; j.x = x; j.f = f;
    j.viol = viol; j.status = status; j.iters = iters; j.outer = outer; j.opt = opt; j.al = al;
    atomic_init(&j.next, 0);
    int nt = nthreads;
    if (nt <= 0) nt = (int)sysconf(_SC_NPROCESSORS_ONLN);
    if (nt < 1) nt = 1;
    if (nt > batch) nt = (int)batch;
    if (nt == 1) al_worker(&j);
    else {
        pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nt);
        for (int t = 0; t < nt; t++) pthread_create(&th[t], NULL, al_worker, &j);
        for (int t = 0; t < nt; t++) pthread_join(th[t], NULL);
        free(th);
    }
    return nt;
}

/* ------------------------------------------------------------------------------------ */
/* Component ADMM (section "Distributed control of ACOPF"): generators and branches, then */
/* buses, then multipliers, every iteration. The paper states only that the generator and */
/* bus subproblems have closed forms; the forms below are the exact minimizers of their   */
/* augmented Lagrangians (reading S25).                                                   */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    double *pg, *qg, *pgt, *qgt, *lpg, *lqg;             /* generators                     */
    double *x, *y, *yt, *lam, *mu, *delta, *alphac;       /* branches (6, 8, 4, 8, 2, 1, 1)  */
    double *wt, *tht;                                     /* buses                           */
} admm_view;

int64_t or_admm_state_size(const or_network *net)
{
    return 6LL * net->ngen + 30LL * net->nbranch + 2LL * net->nbus;
}

static admm_view admm_split(const or_network *net, double *s)
{
    admm_view v;
    int64_t G = net->ngen, L = net->nbranch, B = net->nbus;
    v.pg = s; v.qg = s + G; v.pgt = s + 2 * G; v.qgt = s + 3 * G; v.lpg = s + 4 * G;
    v.lqg = s + 5 * G;
    double *b = s + 6 * G;
    v.x = b; v.y = b + 6 * L; v.yt = b + 14 * L; v.lam = b + 18 * L; v.mu = b + 26 * L;
    v.delta = b + 28 * L; v.alphac = b + 29 * L;
    v.wt = b + 30 * L; v.tht = v.wt + B;
    return v;
}

/* Component values y of branch l at its variables x: flows, v_i^2, v_j^2, th_i, th_j. */
static void branch_couplings(const or_network *net, int l, const double *x, double *y)
{
    double prm[36];
    memset(prm, 0, sizeof(prm));
    memcpy(prm, net->br_adm + 8 * l, sizeof(double) * 8);
    double fl = 0.0;
    br6_couplings(prm, x, 0, y, NULL, NULL, &fl);
}

void or_admm_init(const or_network *net, double *state)
{
    admm_view v = admm_split(net, state);
    for (int g = 0; g < net->ngen; g++) {
        const double *lim = net->gen_lim + 4 * g;
        v.pg[g] = 0.5 * (lim[0] + lim[1]);
        v.qg[g] = 0.5 * (lim[2] + lim[3]);
        v.pgt[g] = v.pg[g];
        v.qgt[g] = v.qg[g];
        v.lpg[g] = 0.0;
        v.lqg[g] = 0.0;
    }
    const double start[6] = {1.0, 1.0, 0.0, 0.0, 0.0, 0.0};
    for (int l = 0; l < net->nbranch; l++) {
        double *x = v.x + 6 * l;
        for (int i = 0; i < 6; i++) x[i] = proj1(start[i], net->br_lo[6 * l + i], net->br_hi[6 * l + i]);
        branch_couplings(net, l, x, v.y + 8 * l);
        for (int k = 0; k < 4; k++) v.yt[4 * l + k] = v.y[8 * l + k];
        for (int k = 0; k < 8; k++) v.lam[8 * l + k] = 0.0;
        v.mu[2 * l] = v.mu[2 * l + 1] = 0.0;
        v.delta[l] = 0.0;
        v.alphac[l] = 0.0;
    }
    for (int b = 0; b < net->nbus; b++) {
        v.wt[b] = 1.0;
        v.tht[b] = 0.0;
    }
}

/* Generator subproblem: min c2' p^2 + c1' p + lam (p - pt) + rho/2 (p - pt)^2 on [pmin, pmax]
 * and min lam_q (q - qt) + rho/2 (q - qt)^2 on [qmin, qmax]; c2' = S^2 c2, c1' = S c1 with
 * S the MVA base (costs per MW, powers per unit). Each is a clipped 1-D stationary point. */
static void admm_generators(const or_network *net, admm_view *v)
{
    double rho = net->rho, S = net->base_mva;
    for (int g = 0; g < net->ngen; g++) {
        double c2 = S * S * net->gen_cost[2 * g], c1 = S * net->gen_cost[2 * g + 1];
        const double *lim = net->gen_lim + 4 * g;
        double p = (rho * v->pgt[g] - v->lpg[g] - c1) / (2.0 * c2 + rho);
        double q = v->qgt[g] - v->lqg[g] / rho;
        v->pg[g] = proj1(p, lim[0], lim[1]);
        v->qg[g] = proj1(q, lim[2], lim[3]);
    }
}

/* Branch subproblems: a BR6 batch whose targets are the current bus copies and whose
 * multipliers are the current lambda, mu; warm-started from the previous x, delta, alpha. */
static void admm_branches(const or_network *net, admm_view *v, const or_opts *opt, int nthreads)
{
    int L = net->nbranch;
    double *prm = (double *)malloc(sizeof(double) * 36 * (size_t)L);
    double *x0 = (double *)malloc(sizeof(double) * 6 * (size_t)L);
    double *f = (double *)malloc(sizeof(double) * (size_t)L);
    int32_t *st = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    int32_t *it = (int32_t *)malloc(sizeof(int32_t) * (size_t)L);
    for (int l = 0; l < L; l++) {
        double *p = prm + 36 * l;
        int i = net->br_from[l], j = net->br_to[l];
        memcpy(p, net->br_adm + 8 * l, sizeof(double) * 8);
        for (int k = 0; k < 4; k++) p[8 + k] = v->yt[4 * l + k];
        p[12] = v->wt[i]; p[13] = v->wt[j]; p[14] = v->tht[i]; p[15] = v->tht[j];
        for (int k = 0; k < 8; k++) p[16 + k] = v->lam[8 * l + k];
        p[24] = v->mu[2 * l]; p[25] = v->mu[2 * l + 1];
        for (int k = 0; k < 10; k++) p[26 + k] = net->rho;
        memcpy(x0 + 6 * l, v->x + 6 * l, sizeof(double) * 6);
    }
    or_opts o = *opt;
    o.use_warm = 1;
    or_tron_batch(OR_BR6, L, NULL, 6, prm, net->br_lo, net->br_hi, x0, v->x, f, st, it, v->delta,
                  v->alphac, NULL, &o, nthreads);
    for (int l = 0; l < L; l++) branch_couplings(net, l, v->x + 6 * l, v->y + 8 * l);
    free(prm); free(x0); free(f); free(st); free(it);
}

/* Bus subproblem (closed form): minimise sum_k rho_k/2 (yt_k - t_k)^2 with t_k = y_k +
 * lam_k / rho over the bus copies of generator powers and incident branch-end flows, and
 * over the bus's w and theta (w and theta are shared by the incident branch ends, so their
 * target is the mean and their weight deg * rho), subject to the two balance rows of eqs.
 * PowerBalanceRealRect / PowerBalanceReactiveRect. The solution is t - W^-1 A' (A W^-1 A')^-1
 * (A t - b), a 2 x 2 solve. The reference bus keeps theta = 0. Accumulates the squared
 * change of every coupling copy into *dual2. */
static void admm_buses(const or_network *net, admm_view *v, double *dual2)
{
    int B = net->nbus, G = net->ngen, L = net->nbranch;
    double rho = net->rho;
    double *sp = (double *)calloc((size_t)B * 8, sizeof(double));
    /* per bus: [0] sum gen p targets, [1] sum gen q targets, [2] sum end p targets,
     * [3] sum end q targets, [4] sum w targets, [5] sum theta targets, [6] ngen, [7] deg */
    for (int g = 0; g < G; g++) {
        int b = net->gen_bus[g];
        sp[8 * b + 0] += v->pg[g] + v->lpg[g] / rho;
        sp[8 * b + 1] += v->qg[g] + v->lqg[g] / rho;
        sp[8 * b + 6] += 1.0;
    }
    for (int l = 0; l < L; l++) {
        const double *y = v->y + 8 * l, *la = v->lam + 8 * l;
        int ends[2] = {net->br_from[l], net->br_to[l]};
        for (int e = 0; e < 2; e++) {
            int b = ends[e];
            sp[8 * b + 2] += y[2 * e] + la[2 * e] / rho;
            sp[8 * b + 3] += y[2 * e + 1] + la[2 * e + 1] / rho;
            sp[8 * b + 4] += y[4 + e] + la[4 + e] / rho;
            sp[8 * b + 5] += y[6 + e] + la[6 + e] / rho;
            sp[8 * b + 7] += 1.0;
        }
    }
    /* solve each bus: multipliers (muP, muQ) of the two balance rows */
    double *mult = (double *)calloc((size_t)B * 2, sizeof(double));
    double *wnew = (double *)malloc(sizeof(double) * (size_t)B);
    double *tnew = (double *)malloc(sizeof(double) * (size_t)B);
    for (int b = 0; b < B; b++) {
        double *a = sp + 8 * b;
        double ng = a[6], deg = a[7];
        const double *ld = net->bus_load + 4 * b;
        double pd = ld[0], qd = ld[1], gs = ld[2], bs = ld[3];
        double tw = a[4] / deg, tth = a[5] / deg;
        double ww = deg * rho;
        /* rows: P: +pg copies, -end p copies, -gs*w = pd;  Q: +qg, -end q, +bs*w = qd */
        double ep = a[0] - a[2] - gs * tw - pd;
        double eq = a[1] - a[3] + bs * tw - qd;
        double mpp = (ng + deg) / rho + gs * gs / ww;
        double mqq = (ng + deg) / rho + bs * bs / ww;
        double mpq = -gs * bs / ww;
        double det = mpp * mqq - mpq * mpq;
        double up = (mqq * ep - mpq * eq) / det;
        double uq = (mpp * eq - mpq * ep) / det;
        mult[2 * b] = up;
        mult[2 * b + 1] = uq;
        wnew[b] = tw - (-gs * up + bs * uq) / ww;
        tnew[b] = b == net->ref_bus ? 0.0 : tth;
    }
    double d2 = 0.0;
    for (int g = 0; g < G; g++) {
        int b = net->gen_bus[g];
        double np = v->pg[g] + v->lpg[g] / rho - mult[2 * b] / rho;
        double nq = v->qg[g] + v->lqg[g] / rho - mult[2 * b + 1] / rho;
        d2 += (np - v->pgt[g]) * (np - v->pgt[g]) + (nq - v->qgt[g]) * (nq - v->qgt[g]);
        v->pgt[g] = np;
        v->qgt[g] = nq;
    }
    for (int l = 0; l < L; l++) {
        const double *y = v->y + 8 * l, *la = v->lam + 8 * l;
        double *yt = v->yt + 4 * l;
        int ends[2] = {net->br_from[l], net->br_to[l]};
        for (int e = 0; e < 2; e++) {
            int b = ends[e];
            double np = y[2 * e] + la[2 * e] / rho + mult[2 * b] / rho;
            double nq = y[2 * e + 1] + la[2 * e + 1] / rho + mult[2 * b + 1] / rho;
            d2 += (np - yt[2 * e]) * (np - yt[2 * e]) + (nq - yt[2 * e + 1]) * (nq - yt[2 * e + 1]);
            yt[2 * e] = np;
            yt[2 * e + 1] = nq;
            double dw = wnew[b] - v->wt[b], dt = tnew[b] - v->tht[b];
            d2 += dw * dw + dt * dt;
        }
    }
    for (int b = 0; b < B; b++) {
        v->wt[b] = wnew[b];
        v->tht[b] = tnew[b];
    }
    *dual2 = d2;
    free(sp); free(mult); free(wnew); free(tnew);
}

/* Multiplier update: lam_k += rho (y_k - yt_k) for every coupling, mu += rho (z - p).
 * Returns the squared primal residual sum (y - yt)^2 over the couplings. */
static double admm_duals(const or_network *net, admm_view *v)
{
    double rho = net->rho, p2 = 0.0;
    for (int g = 0; g < net->ngen; g++) {
        double rp = v->pg[g] - v->pgt[g], rq = v->qg[g] - v->qgt[g];
        v->lpg[g] += rho * rp;
        v->lqg[g] += rho * rq;
        p2 += rp * rp + rq * rq;
    }
    for (int l = 0; l < net->nbranch; l++) {
        const double *y = v->y + 8 * l, *yt = v->yt + 4 * l, *x = v->x + 6 * l;
        double *la = v->lam + 8 * l;
        int i = net->br_from[l], j = net->br_to[l];
        double copy[8] = {yt[0], yt[1], yt[2], yt[3], v->wt[i], v->wt[j], v->tht[i], v->tht[j]};
        for (int k = 0; k < 8; k++) {
            double r = y[k] - copy[k];
            la[k] += rho * r;
            p2 += r * r;
        }
        v->mu[2 * l] += rho * (x[4] - y[0]);
        v->mu[2 * l + 1] += rho * (x[5] - y[2]);
    }
    return p2;
}

int32_t or_admm_run(const or_network *net, double *state, int32_t iters, double *resid,
                    const or_opts *opt, int32_t nthreads)
{
    /* every bus must touch at least one branch (its w and theta copies are branch-owned) */
    int *deg = (int *)calloc((size_t)net->nbus, sizeof(int));
    for (int l = 0; l < net->nbranch; l++) { deg[net->br_from[l]]++; deg[net->br_to[l]]++; }
    for (int b = 0; b < net->nbus; b++)
        if (deg[b] == 0) { free(deg); return -1; }
    free(deg);
    admm_view v = admm_split(net, state);
    for (int it = 0; it < iters; it++) {
        admm_generators(net, &v);
        admm_branches(net, &v, opt, nthreads);
        double d2 = 0.0;
        admm_buses(net, &v, &d2);
        double p2 = admm_duals(net, &v);
        if (resid) {
            resid[2 * it] = sqrt(p2);
            resid[2 * it + 1] = net->rho * sqrt(d2);
        }
    }
    return 0;
}

/* One phase of an iteration, for the tests: 0 generators, 1 branches, 2 buses (out[0] =
 * squared dual change), 3 multipliers (out[0] = squared primal residual). */
int32_t or_admm_phase(const or_network *net, double *state, int32_t phase, double *out,
                      const or_opts *opt, int32_t nthreads)
{
    admm_view v = admm_split(net, state);
    double r = 0.0;
    if (phase == 0) admm_generators(net, &v);
    else if (phase == 1) admm_branches(net, &v, opt, nthreads);
    else if (phase == 2) admm_buses(net, &v, &r);
    else if (phase == 3) r = admm_duals(net, &v);
    else return -1;
    if (out) out[0] = r;
    return 0;
}
