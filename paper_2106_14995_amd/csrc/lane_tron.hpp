// lane_tron.hpp -- one trust-region Newton solve per GPU lane, state in VGPRs.
//
// For small n (n <= 8) every instance lives in one lane of a wave64: x, g, the packed
// lower triangle of the Hessian, the packed Cholesky factor and the CG vectors are
// fixed-size arrays indexed only by compile-time constants after unrolling, so they are
// registers (the branch family alone keeps its 36 parameters in the workgroup's LDS, see
// BR6T). 64 instances share a wave and 4 waves a CU; there are no cross-lane operations at
// all (the paper's warp-per-problem reductions, section 5.1, become plain per-lane sums).
//
// Algorithm 1 (section 3) per lane, with the readings of the method that the paper leaves
// to the TRON method it cites:
//   * Cauchy step: s(a) = P[x - a g] - x acceptable when ||s|| <= delta and
//     q(s) <= mu0 g's; from the previous step length, extrapolate by 10 while acceptable
//     and below the largest breakpoint, else interpolate by 0.1 (at most 60 steps each).
//   * Free set F = { l < xs < u } as a bitmask; the reduced Hessian H_FF is never gathered:
//     rows and columns outside F are replaced by the identity, which gives the same
//     Cholesky factor and the same CG iterates as the gathered block (the extra terms are
//     exact zeros).
//   * Preconditioner: complete left-looking Cholesky of H_FF + alpha I (section 4.3) with
//     alpha = 0 when the diagonal is positive, else a shift grown by doubling (at most 64
//     tries, then a diagonal factor).
//   * Steihaug CG on L^-1 A L^-T s = -L^-1 (g + Hs)_F within ||s|| <= delta, at most |F|
//     iterations, or its one exact step when the factorisation needed no shift (then the
//     preconditioned matrix is the identity); w = L^-T s; projected search with halving (at
//     most 20 halvings);
//     another pass while CG ended inside the region and a free variable hit a bound.
//   * Ratio test and radius update of TRON; the step is measured in the norm of the trust
//     region that bounded it (||L^T s|| on the last factored free set); when the predicted
//     reduction is at the rounding level of f the actual reduction is taken from the
//     gradients (trapezoid).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mt {

#define MT_INLINE __device__ __forceinline__
#define MT_UNROLL _Pragma("unroll")

constexpr double kMu0 = 0.01;
constexpr double kEta0 = 1e-4, kEta1 = 0.25, kEta2 = 0.75;
constexpr double kSig1 = 0.25, kSig2 = 0.5, kSig3 = 4.0;
constexpr int kCauchyMax = 60;
constexpr int kSearchHalvings = 20;
constexpr int kShiftTries = 64;
constexpr double kStallRel = 1e-15;
constexpr double kAredSwitch = 1e-10;

enum : int32_t { kConverged = 0, kMaxIter = 1, kStalled = 2, kNonfinite = 3, kBadBounds = 4, kAlMaxOuter = 5 };
enum : int { kCgConv = 0, kCgMaxit = 1, kCgNeg = 2, kCgBnd = 3 };

// packed lower-triangular index, row by row
MT_INLINE constexpr int tri(int i, int j) { return i >= j ? i * (i + 1) / 2 + j : j * (j + 1) / 2 + i; }

// projection onto [lo, hi] that keeps a NaN (used on the caller's x0)
MT_INLINE double clampb(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }
// projection for finite v (two min/max instructions; used once x and g are known finite)
MT_INLINE double clampf(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }
MT_INLINE double dmax(double a, double b) { return a > b ? a : b; }
MT_INLINE double dmin(double a, double b) { return a < b ? a : b; }

// 1/sqrt(d) for a positive finite d: the hardware estimate y (about single precision) and
// one third-order correction from the binomial series (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + ...
// with e = 1 - d y^2, which leaves a relative error of order e^3. Four dependent operations
// after the estimate; a pivot of the factorisation is on a serial chain, so this matters.
MT_INLINE double rsqrt_pos(double d)
{
    const double y = __builtin_amdgcn_rsq(d);
    const double e = fma(-(d * y), y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// projected-gradient component (section 5.1): g inside, min(g,0) at l, max(g,0) at u, 0 if
// l = u; g is finite wherever this is called (finiteness is checked first)
MT_INLINE double pg_comp(double x, double lo, double hi, double g)
{
    const double v = x <= lo ? fmin(g, 0.0) : (x >= hi ? fmax(g, 0.0) : g);
    return lo == hi ? 0.0 : v;
}

struct Options {
    double gtol, cg_rtol, delta0;
    int32_t max_iter;
    int32_t warm;
};

// ------------------------------------------------------------------------------------
// Problem families. Each provides: pad (value of padded variables), load(p, n),
// fg(x, g) -> f (caches what hess needs), hess(x) (at the point of the last fg),
// H(i, j) (compile-time i, j).
// ------------------------------------------------------------------------------------

// QP4: f = x'Qx/2 + c'x + kappa sum x^4; H = Q + diag(12 kappa x^2).
template <int N>
struct QP4 {
    static constexpr int T = N * (N + 1) / 2;
    static constexpr double pad = 0.0;
    static constexpr int kLdsDoubles = 0;  // per lane, in the lane kernel's dynamic LDS
    double q[T];
    double c[N];
    double hd[N];
    double kap;

    MT_INLINE void load(const double *__restrict__ p, int n)
    {
        // padded rows (i >= n) are zero; the address is clamped so no load leaves the block
        MT_UNROLL for (int i = 0; i < N; i++)
            MT_UNROLL for (int j = 0; j <= i; j++) q[tri(i, j)] = (i < n) ? p[(i < n) ? tri(i, j) : 0] : 0.0;
        const double *cp = p + n * (n + 1) / 2;
        MT_UNROLL for (int i = 0; i < N; i++) c[i] = (i < n) ? cp[(i < n) ? i : 0] : 0.0;
        kap = cp[n];
    }
    MT_INLINE double fg(const double (&x)[N], double (&g)[N])
    {
        double quad = 0.0, lin = 0.0, qrt = 0.0;
        const double k4 = 4.0 * kap;
        MT_UNROLL for (int i = 0; i < N; i++) {
            double qi = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) qi = fma(q[tri(i, j)], x[j], qi);
            const double x2 = x[i] * x[i];
            quad = fma(x[i], qi, quad);
            lin = fma(c[i], x[i], lin);
            qrt = fma(x2, x2, qrt);
            g[i] = fma(k4 * x2, x[i], qi + c[i]);
        }
        return fma(kap, qrt, fma(0.5, quad, lin));
    }
    MT_INLINE void hess(const double (&x)[N])
    {
        const double k12 = 12.0 * kap;
        MT_UNROLL for (int i = 0; i < N; i++) hd[i] = fma(k12 * x[i], x[i], q[tri(i, i)]);
    }
    MT_INLINE double H(int i, int j) const { return i == j ? hd[i] : q[tri(i, j)]; }
};

// HS45M: f = 120 - prod x_i (the hs45 variant of section 4.2); padded variables are 1.
template <int N>
struct HS45M {
    static constexpr int T = N * (N + 1) / 2;
    static constexpr double pad = 1.0;
    static constexpr int kLdsDoubles = 0;
    double h[T];
    MT_INLINE void load(const double *__restrict__, int) {}
    MT_INLINE double fg(const double (&x)[N], double (&g)[N])
    {
        double pr = 1.0;
        MT_UNROLL for (int i = 0; i < N; i++) pr *= x[i];
        MT_UNROLL for (int i = 0; i < N; i++) {
            double q = 1.0;
            MT_UNROLL for (int k = 0; k < N; k++) if (k != i) q *= x[k];
            g[i] = -q;
        }
        return 120.0 - pr;
    }
    MT_INLINE void hess(const double (&x)[N])
    {
        MT_UNROLL for (int i = 0; i < N; i++)
            MT_UNROLL for (int j = 0; j <= i; j++) {
                double q = 1.0;
                MT_UNROLL for (int k = 0; k < N; k++) if (k != i && k != j) q *= x[k];
                h[tri(i, j)] = (i == j) ? 0.0 : -q;
            }
    }
    MT_INLINE double H(int i, int j) const { return h[tri(i, j)]; }
};

// The lane kernel's dynamic LDS (families with kLdsDoubles > 0 keep data there).
MT_INLINE double *lane_lds()
{
    extern __shared__ double mt_lane_lds[];
    return mt_lane_lds;
}

// BR6: the branch subproblem (eq. exp-branch) with the flows of eqs. pij..qji and two
// flow copies z coupled to p_ij, p_ji. Derivatives are taken in (v_i, v_j, D = th_i - th_j)
// and mapped to (th_i, th_j) with dD/dth_i = 1, dD/dth_j = -1.
// kLds: the 36 parameters live in the workgroup's LDS and are read at each evaluation; the
// lane's registers then hold only the solver state. Each wave has a block of 36 x 64 doubles,
// parameter k of lane l at k 64 + l, so that the 36 reads share one address register and
// differ by immediate offsets. The index passes through an empty asm statement at each
// evaluation, so that the loads stay there instead of being hoisted out of the solve loop
// into registers. Otherwise the parameters stay in registers for the whole solve (the form
// the group kernel and BR8L use).
template <bool kLds>
struct BR6T {
    static constexpr int N = 6;
    static constexpr int T = 21;
    static constexpr double pad = 0.0;
    static constexpr int kLdsDoubles = kLds ? 36 : 0;
    double prm_r[kLds ? 1 : 36];
    double cth, sth;       // cos, sin of th_i - th_j at the last fg point
    double h[T];

    // the lane's first parameter in the workgroup's LDS (its wave's block, then the lane)
    static MT_INLINE int lds_base() { return ((int)threadIdx.x >> 6) * (36 * 64) + ((int)threadIdx.x & 63); }

    MT_INLINE void load(const double *__restrict__ p, int)
    {
        if constexpr (kLds) {
            double *L = lane_lds() + lds_base();
            MT_UNROLL for (int k = 0; k < 36; k++) L[64 * k] = p[k];
        } else {
            MT_UNROLL for (int k = 0; k < 36; k++) prm_r[k] = p[k];
        }
    }
    MT_INLINE void params(double (&q)[36]) const
    {
        if constexpr (kLds) {
            int o = lds_base();
            asm volatile("" : "+v"(o));
            const double *L = lane_lds() + o;
            MT_UNROLL for (int k = 0; k < 36; k++) q[k] = L[64 * k];
        } else {
            MT_UNROLL for (int k = 0; k < 36; k++) q[k] = prm_r[k];
        }
    }
    // flow k = a own^2 + V (al cos D + be sin D), own = v_i for k < 2 and v_j otherwise
    static MT_INLINE double fa(const double (&p)[36], int k) { return k == 0 ? p[2] : k == 1 ? p[3] : k == 2 ? p[6] : p[7]; }
    static MT_INLINE double fal(const double (&p)[36], int k) { return k == 0 ? -p[0] : k == 1 ? -p[1] : k == 2 ? -p[4] : -p[5]; }
    static MT_INLINE double fbe(const double (&p)[36], int k) { return k == 0 ? p[1] : k == 1 ? -p[0] : k == 2 ? -p[5] : p[4]; }

    // flows y[0..3], phi, psi = dphi/dD, and first-derivative coefficients of the flows
    // (c_k, with the z couplings folded into p_ij and p_ji) at x
    MT_INLINE double flows(const double (&prm)[36], const double (&x)[6], double (&y)[4], double (&phi)[4],
                           double (&psi)[4], double (&ck)[4], double (&cz)[2], double (&cw)[2],
                           double (&cth_)[2]) const
    {
        const double vi = x[0], vj = x[1], V = vi * vj;
        double f = 0.0;
        MT_UNROLL for (int k = 0; k < 4; k++) {
            const double al = fal(prm, k), be = fbe(prm, k), a = fa(prm, k);
            const double own = k < 2 ? vi : vj;
            phi[k] = fma(al, cth, be * sth);
            psi[k] = fma(-al, sth, be * cth);
            y[k] = fma(a * own, own, V * phi[k]);
            const double e = y[k] - prm[8 + k];
            ck[k] = fma(prm[26 + k], e, prm[16 + k]);
            f = fma(fma(0.5 * prm[26 + k], e, prm[16 + k]), e, f);
        }
        // w and theta couplings
        const double ew0 = vi * vi - prm[12], ew1 = vj * vj - prm[13];
        const double et0 = x[2] - prm[14], et1 = x[3] - prm[15];
        cw[0] = fma(prm[30], ew0, prm[20]);
        cw[1] = fma(prm[31], ew1, prm[21]);
        cth_[0] = fma(prm[32], et0, prm[22]);
        cth_[1] = fma(prm[33], et1, prm[23]);
        f = fma(fma(0.5 * prm[30], ew0, prm[20]), ew0, f);
        f = fma(fma(0.5 * prm[31], ew1, prm[21]), ew1, f);
        f = fma(fma(0.5 * prm[32], et0, prm[22]), et0, f);
        f = fma(fma(0.5 * prm[33], et1, prm[23]), et1, f);
        // flow copies: r = z - p
        const double r0 = x[4] - y[0], r1 = x[5] - y[2];
        cz[0] = fma(prm[34], r0, prm[24]);
        cz[1] = fma(prm[35], r1, prm[25]);
        f = fma(fma(0.5 * prm[34], r0, prm[24]), r0, f);
        f = fma(fma(0.5 * prm[35], r1, prm[25]), r1, f);
        return f;
    }

    MT_INLINE double fg(const double (&x)[6], double (&g)[6])
    {
        double prm[36];
        params(prm);
        sincos(x[2] - x[3], &sth, &cth);
        double y[4], phi[4], psi[4], ck[4], cz[2], cw[2], ct[2];
        const double f = flows(prm, x, y, phi, psi, ck, cz, cw, ct);
        const double vi = x[0], vj = x[1], V = vi * vj;
        // effective coefficients of the flow gradients (z couplings subtract from p flows)
        const double e0 = ck[0] - cz[0], e1 = ck[1], e2 = ck[2] - cz[1], e3 = ck[3];
        const double sphi = e0 * phi[0] + e1 * phi[1] + e2 * phi[2] + e3 * phi[3];
        const double spsi = e0 * psi[0] + e1 * psi[1] + e2 * psi[2] + e3 * psi[3];
        const double own_i = 2.0 * (e0 * fa(prm, 0) + e1 * fa(prm, 1)) * vi;
        const double own_j = 2.0 * (e2 * fa(prm, 2) + e3 * fa(prm, 3)) * vj;
        g[0] = fma(vj, sphi, own_i) + 2.0 * cw[0] * vi;
        g[1] = fma(vi, sphi, own_j) + 2.0 * cw[1] * vj;
        const double gD = V * spsi;
        g[2] = gD + ct[0];
        g[3] = ct[1] - gD;
        g[4] = cz[0];
        g[5] = cz[1];
        return f;
    }

    MT_INLINE void hess(const double (&x)[6])
    {
        double prm[36];
        params(prm);
        double y[4], phi[4], psi[4], ck[4], cz[2], cw[2], ct[2];
        flows(prm, x, y, phi, psi, ck, cz, cw, ct);
        const double vi = x[0], vj = x[1], V = vi * vj;
        const double e[4] = {ck[0] - cz[0], ck[1], ck[2] - cz[1], ck[3]};
        // Gauss-Newton weights: the z couplings add their penalty to p_ij and p_ji
        const double w[4] = {prm[26] + prm[34], prm[27], prm[28] + prm[35], prm[29]};
        double hvv[3] = {0, 0, 0};  // (vi,vi), (vj,vj), (vi,vj)
        double hvD[2] = {0, 0};     // (vi,D), (vj,D)
        double hDD = 0.0;
        double dp[2][3];            // gradients of p_ij, p_ji in (vi, vj, D)
        MT_UNROLL for (int k = 0; k < 4; k++) {
            const double a2 = 2.0 * fa(prm, k);
            const double di = k < 2 ? fma(vj, phi[k], a2 * vi) : vj * phi[k];
            const double dj = k < 2 ? vi * phi[k] : fma(vi, phi[k], a2 * vj);
            const double dD = V * psi[k];
            if (k == 0) { dp[0][0] = di; dp[0][1] = dj; dp[0][2] = dD; }
            if (k == 2) { dp[1][0] = di; dp[1][1] = dj; dp[1][2] = dD; }
            hvv[0] = fma(w[k] * di, di, fma(e[k], k < 2 ? a2 : 0.0, hvv[0]));
            hvv[1] = fma(w[k] * dj, dj, fma(e[k], k < 2 ? 0.0 : a2, hvv[1]));
            hvv[2] = fma(w[k] * di, dj, fma(e[k], phi[k], hvv[2]));
            hvD[0] = fma(w[k] * di, dD, fma(e[k], vj * psi[k], hvD[0]));
            hvD[1] = fma(w[k] * dj, dD, fma(e[k], vi * psi[k], hvD[1]));
            hDD = fma(w[k] * dD, dD, fma(e[k], -V * phi[k], hDD));
        }
        // w couplings: v^2
        hvv[0] = fma(4.0 * prm[30] * vi, vi, fma(2.0, cw[0], hvv[0]));
        hvv[1] = fma(4.0 * prm[31] * vj, vj, fma(2.0, cw[1], hvv[1]));
        // map (vi, vj, D) -> (vi, vj, th_i, th_j); z rows from r = z - p
        h[tri(0, 0)] = hvv[0];
        h[tri(1, 0)] = hvv[2];
        h[tri(1, 1)] = hvv[1];
        h[tri(2, 0)] = hvD[0];
        h[tri(2, 1)] = hvD[1];
        h[tri(2, 2)] = hDD + prm[32];
        h[tri(3, 0)] = -hvD[0];
        h[tri(3, 1)] = -hvD[1];
        h[tri(3, 2)] = -hDD;
        h[tri(3, 3)] = hDD + prm[33];
        const double rz0 = prm[34], rz1 = prm[35];
        h[tri(4, 0)] = -rz0 * dp[0][0];
        h[tri(4, 1)] = -rz0 * dp[0][1];
        h[tri(4, 2)] = -rz0 * dp[0][2];
        h[tri(4, 3)] = rz0 * dp[0][2];
        h[tri(4, 4)] = rz0;
        h[tri(5, 0)] = -rz1 * dp[1][0];
        h[tri(5, 1)] = -rz1 * dp[1][1];
        h[tri(5, 2)] = -rz1 * dp[1][2];
        h[tri(5, 3)] = rz1 * dp[1][2];
        h[tri(5, 4)] = 0.0;
        h[tri(5, 5)] = rz1;
    }
    MT_INLINE double H(int i, int j) const { return h[tri(i, j)]; }
};

// the lane kernel's form (parameters in LDS) and the register form
struct BR6 : BR6T<true> {};
using BR6R = BR6T<false>;

// BR8L: BR6 plus the line limits of both ends as equalities with slacks,
//   h_lm = p_lm^2 + q_lm^2 + sigma_lm - smax^2,  lm in {ij, ji},
// entering through the augmented-Lagrangian terms lambda_lm h_lm + rho_h/2 h_lm^2 (section 1
// and its footnote on inequalities). x = (v_i, v_j, th_i, th_j, z_ij, z_ji, sigma_ij,
// sigma_ji); parameters [0..35] as BR6, [36] smax^2, [37..38] lambda, [39] rho_h.
// The limit terms are differentiated in (v_i, v_j, D, sigma) like BR6's flows and mapped
// to (th_i, th_j) the same way.
struct BR8L {
    static constexpr int N = 8;
    static constexpr int T = 36;
    static constexpr double pad = 0.0;
    static constexpr int kLdsDoubles = 0;
    BR6R b6;               // the BR6 part; its Hessian block also receives the limit terms
    double smax2, lam[2], rhoh;
    double hs[2][4];       // slack rows of the Hessian against (v_i, v_j, th_i, th_j)

    MT_INLINE void load(const double *__restrict__ p, int n)
    {
        b6.load(p, n);
        smax2 = p[36];
        lam[0] = p[37];
        lam[1] = p[38];
        rhoh = p[39];
    }

    // flow k (p_ij, q_ij, p_ji, q_ji) at (vi, vj) with the cached cos/sin of D: value,
    // gradient in (vi, vj, D) and the six distinct second derivatives
    // (vi vi, vj vj, vi vj, vi D, vj D, D D)
    MT_INLINE void flow(int k, double vi, double vj, double &y, double (&d)[3], double (&d2)[6]) const
    {
        const double al = b6.fal(b6.prm_r, k), be = b6.fbe(b6.prm_r, k), a = b6.fa(b6.prm_r, k), V = vi * vj;
        const double phi = fma(al, b6.cth, be * b6.sth);
        const double psi = fma(-al, b6.sth, be * b6.cth);
        const double a2 = 2.0 * a;
        const bool own_i = k < 2;
        y = own_i ? fma(a * vi, vi, V * phi) : fma(a * vj, vj, V * phi);
        d[0] = own_i ? fma(vj, phi, a2 * vi) : vj * phi;
        d[1] = own_i ? vi * phi : fma(vi, phi, a2 * vj);
        d[2] = V * psi;
        d2[0] = own_i ? a2 : 0.0;
        d2[1] = own_i ? 0.0 : a2;
        d2[2] = phi;
        d2[3] = vj * psi;
        d2[4] = vi * psi;
        d2[5] = -V * phi;
    }

    // the two limit residuals at x (sets the cached angle of b6 to x's)
    MT_INLINE void limits(const double (&x)[8], double (&hv)[2])
    {
        sincos(x[2] - x[3], &b6.sth, &b6.cth);
        MT_UNROLL for (int l = 0; l < 2; l++) {
            double yp, yq, d[3], d2[6];
            flow(2 * l, x[0], x[1], yp, d, d2);
            flow(2 * l + 1, x[0], x[1], yq, d, d2);
            hv[l] = fma(yp, yp, fma(yq, yq, x[6 + l] - smax2));
        }
    }

    MT_INLINE double fg(const double (&x)[8], double (&g)[8])
    {
        double x6[6], g6[6];
        MT_UNROLL for (int i = 0; i < 6; i++) x6[i] = x[i];
        double f = b6.fg(x6, g6);  // caches cos/sin of th_i - th_j at x
        MT_UNROLL for (int i = 0; i < 6; i++) g[i] = g6[i];
        MT_UNROLL for (int l = 0; l < 2; l++) {
            double yp, yq, dp[3], dq[3], d2[6];
            flow(2 * l, x[0], x[1], yp, dp, d2);
            flow(2 * l + 1, x[0], x[1], yq, dq, d2);
            const double hv = fma(yp, yp, fma(yq, yq, x[6 + l] - smax2));
            const double c = fma(rhoh, hv, lam[l]);
            f = fma(fma(0.5 * rhoh, hv, lam[l]), hv, f);
            const double c2 = 2.0 * c;
            const double uD = c2 * fma(yp, dp[2], yq * dq[2]);
            g[0] = fma(c2, fma(yp, dp[0], yq * dq[0]), g[0]);
            g[1] = fma(c2, fma(yp, dp[1], yq * dq[1]), g[1]);
            g[2] += uD;
            g[3] -= uD;
            g[6 + l] = c;
        }
        return f;
    }

    MT_INLINE void hess(const double (&x)[8])
    {
        double x6[6];
        MT_UNROLL for (int i = 0; i < 6; i++) x6[i] = x[i];
        b6.hess(x6);  // uses the angle cached by the last fg, which was at x
        MT_UNROLL for (int l = 0; l < 2; l++) {
            double yp, yq, dp[3], dq[3], d2p[6], d2q[6];
            flow(2 * l, x[0], x[1], yp, dp, d2p);
            flow(2 * l + 1, x[0], x[1], yq, dq, d2q);
            const double hv = fma(yp, yp, fma(yq, yq, x[6 + l] - smax2));
            const double c2 = 2.0 * fma(rhoh, hv, lam[l]);
            // grad h in (vi, vj, D); sigma_l enters with 1
            double u[3];
            MT_UNROLL for (int a = 0; a < 3; a++) u[a] = 2.0 * fma(yp, dp[a], yq * dq[a]);
            // M = rho u u' + 2c (dp dp' + yp d2p + dq dq' + yq d2q) on (vi, vj, D)
            const int ia[6] = {0, 1, 0, 0, 1, 2}, ib[6] = {0, 1, 1, 2, 2, 2};
            double m[6];
            MT_UNROLL for (int e = 0; e < 6; e++) {
                const int a = ia[e], bb = ib[e];
                const double cur = fma(dp[a], dp[bb], fma(yp, d2p[e], fma(dq[a], dq[bb], yq * d2q[e])));
                m[e] = fma(rhoh * u[a], u[bb], c2 * cur);
            }
            // (vi, vj, D) -> (vi, vj, th_i, th_j), added to the BR6 block in place
            double *h6 = b6.h;
            h6[tri(0, 0)] += m[0];
            h6[tri(1, 1)] += m[1];
            h6[tri(1, 0)] += m[2];
            h6[tri(2, 0)] += m[3];
            h6[tri(3, 0)] -= m[3];
            h6[tri(2, 1)] += m[4];
            h6[tri(3, 1)] -= m[4];
            h6[tri(2, 2)] += m[5];
            h6[tri(3, 3)] += m[5];
            h6[tri(3, 2)] -= m[5];
            // the slack row: rho (u_vi, u_vj, u_D, -u_D) against (v_i, v_j, th_i, th_j)
            hs[l][0] = rhoh * u[0];
            hs[l][1] = rhoh * u[1];
            hs[l][2] = rhoh * u[2];
            hs[l][3] = -rhoh * u[2];
        }
    }
    // i, j are compile-time after unrolling, so the selection costs nothing
    MT_INLINE double H(int i, int j) const
    {
        if (i < 6 && j < 6) return b6.h[tri(i, j)];
        const int r = i > j ? i : j, c = i > j ? j : i;  // r is a slack row (6 or 7)
        if (c == r) return rhoh;
        return c < 4 ? hs[r - 6][c] : 0.0;
    }
};

// ------------------------------------------------------------------------------------
// The solver for one lane.
// ------------------------------------------------------------------------------------
template <class F, int N>
struct LaneTron {
    static constexpr int T = N * (N + 1) / 2;
    F fam;
    double lo[N], hi[N];
    double x[N], g[N];     // iterate and gradient
    double xs[N];          // subspace point (Cauchy point, then moved by the passes)
    double L[T], dinv[N];  // preconditioner factor and reciprocal pivots
    uint32_t lfm;          // free set of the last factored pass (0: none this iteration)
    double f, delta, alphac;
    int32_t iters;
    int32_t cg_iters, cauchy_trials, search_trials, chol_tries;

    MT_INLINE double dot(const double (&a)[N], const double (&b)[N]) const
    {
        double s = 0.0;
        MT_UNROLL for (int i = 0; i < N; i++) s = fma(a[i], b[i], s);
        return s;
    }
    MT_INLINE void hmul(const double (&v)[N], double (&out)[N]) const
    {
        MT_UNROLL for (int i = 0; i < N; i++) {
            double s = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) s = fma(fam.H(i, j), v[j], s);
            out[i] = s;
        }
    }
    MT_INLINE double pg_inf() const
    {
        double m = 0.0;
        MT_UNROLL for (int i = 0; i < N; i++) m = fmax(m, fabs(pg_comp(x[i], lo[i], hi[i], g[i])));
        return m;
    }
    MT_INLINE double pg_nrm2() const
    {
        double s = 0.0;
        MT_UNROLL for (int i = 0; i < N; i++) {
            const double v = pg_comp(x[i], lo[i], hi[i], g[i]);
            s = fma(v, v, s);
        }
        return sqrt(s);
    }
    MT_INLINE void fwd(double (&b)[N]) const
    {
        MT_UNROLL for (int i = 0; i < N; i++) {
            double s = b[i];
            MT_UNROLL for (int k = 0; k < i; k++) s = fma(-L[tri(i, k)], b[k], s);
            b[i] = s * dinv[i];
        }
    }
    MT_INLINE void bwd(double (&b)[N]) const
    {
        MT_UNROLL for (int i = N - 1; i >= 0; i--) {
            double s = b[i];
            MT_UNROLL for (int k = i + 1; k < N; k++) s = fma(-L[tri(k, i)], b[k], s);
            b[i] = s * dinv[i];
        }
    }
    // sigma >= 0 with ||v + sigma p|| = delta (trqsol), cancellation-free root
    MT_INLINE double trqsol(const double (&v)[N], const double (&p)[N]) const
    {
        const double ptx = dot(p, v), ptp = dot(p, p), xtx = dot(v, v);
        const double dsq = delta * delta;
        double disc = fma(ptx, ptx, ptp * (dsq - xtx));
        disc = disc < 0.0 ? 0.0 : disc;
        const double rad = sqrt(disc);
        const double sig = ptx >= 0.0 ? (dsq - xtx) / (ptx + rad) : (rad - ptx) / ptp;
        return sig > 0.0 ? sig : 0.0;
    }

    // One Cauchy trial at step length a: xt = P[x - a g]; acceptable when ||xt - x|| <= delta
    // and q(xt - x) <= mu0 g'(xt - x).
    MT_INLINE bool cauchy_trial(double a, double (&xt)[N])
    {
        cauchy_trials++;
        double st[N];
        MT_UNROLL for (int i = 0; i < N; i++) {
            xt[i] = clampf(fma(-a, g[i], x[i]), lo[i], hi[i]);
            st[i] = xt[i] - x[i];
        }
        if (!(dot(st, st) <= delta * delta)) return false;  // ||s|| <= delta
        const double gts = dot(g, st);
        double hs[N];
        hmul(st, hs);
        const double q = fma(0.5, dot(st, hs), gts);
        return q <= kMu0 * gts;
    }

    // a below the largest breakpoint along -g: some finite bound i is not yet reached at
    // step a, i.e. a |g_i| < (distance to that bound), written without divisions; with no
    // finite breakpoint at all the bound is +inf
    MT_INLINE bool below_last_breakpoint(double a) const
    {
        bool any = false, below = false;
        MT_UNROLL for (int i = 0; i < N; i++) {
            const double d = -g[i];
            const bool up = d > 0.0 && isfinite(hi[i]);
            const bool dn = d < 0.0 && isfinite(lo[i]);
            any = any || up || dn;
            below = below || (up && a * d < hi[i] - x[i]) || (dn && a * d > lo[i] - x[i]);
        }
        return !any || below;
    }

    MT_INLINE void cauchy()
    {
        double a = alphac;
        double xt[N];
        if (cauchy_trial(a, xt)) {
            MT_UNROLL for (int i = 0; i < N; i++) xs[i] = xt[i];
            for (int t = 0; t < kCauchyMax; t++) {
                if (!below_last_breakpoint(a)) break;
                const double a2 = 10.0 * a;
                if (!cauchy_trial(a2, xt)) break;
                a = a2;
                MT_UNROLL for (int i = 0; i < N; i++) xs[i] = xt[i];
            }
        } else {
            for (int t = 0; t < kCauchyMax; t++) {
                a = 0.1 * a;
                if (cauchy_trial(a, xt)) break;
            }
            MT_UNROLL for (int i = 0; i < N; i++) xs[i] = xt[i];
        }
        alphac = a;
    }

    // Cholesky of the masked, shifted matrix: rows/columns outside fm are the identity.
    MT_INLINE bool chol(uint32_t fm, double alpha)
    {
        bool ok = true;
        MT_UNROLL for (int j = 0; j < N; j++) {
            const bool fj = (fm >> j) & 1u;
            double d = fam.H(j, j) + alpha;
            MT_UNROLL for (int k = 0; k < j; k++) d = fma(-L[tri(j, k)], L[tri(j, k)], d);
            ok = ok && (!fj || d > 0.0);
            const double r = fj ? rsqrt_pos(d) : 1.0;  // 1 / pivot
            L[tri(j, j)] = fj ? d * r : 1.0;        // pivot = d / sqrt(d)
            dinv[j] = r;
            MT_UNROLL for (int i = j + 1; i < N; i++) {
                double s = fam.H(i, j);
                MT_UNROLL for (int k = 0; k < j; k++) s = fma(-L[tri(i, k)], L[tri(j, k)], s);
                L[tri(i, j)] = (fj && ((fm >> i) & 1u)) ? s * r : 0.0;
            }
        }
        return ok;
    }

    // Returns the shift that succeeded, or -1 when the diagonal fallback was used.
    MT_INLINE double precond(uint32_t fm)
    {
        double dmn = 0.0, dmx = 0.0;
        bool first = true;
        MT_UNROLL for (int i = 0; i < N; i++) {
            if ((fm >> i) & 1u) {
                const double v = fam.H(i, i);
                dmn = (first || v < dmn) ? v : dmn;
                dmx = fabs(v) > dmx ? fabs(v) : dmx;
                first = false;
            }
        }
        const double beta = 1e-3 * (dmx > 1.0 ? dmx : 1.0);
        double alpha = dmn > 0.0 ? 0.0 : beta - dmn;
        for (int t = 0; t < kShiftTries; t++) {
            chol_tries++;
            if (chol(fm, alpha)) return alpha;
            alpha = 2.0 * alpha > beta ? 2.0 * alpha : beta;
        }
        MT_UNROLL for (int i = 0; i < N; i++) {
            MT_UNROLL for (int k = 0; k < i; k++) L[tri(i, k)] = 0.0;
            const double v = fabs(fam.H(i, i));
            const double piv = ((fm >> i) & 1u) ? sqrt(v > beta ? v : beta) : 1.0;
            L[tri(i, i)] = piv;
            dinv[i] = 1.0 / piv;
        }
        return -1.0;
    }

    // Steihaug CG in the preconditioned variable; result in sh (zero outside fm).
    // exact: L L^T is the unshifted block itself, so the preconditioned matrix is the
    // identity and its first CG step (section 3: one iteration when no shift is needed),
    // s_hat = r_hat cut at the radius, is the whole solve; the products that would only
    // reproduce p are not formed.
    MT_INLINE int pcg(uint32_t fm, int m, const double (&r)[N], double (&sh)[N], double cg_rtol, bool exact)
    {
        double rh[N], p[N];
        MT_UNROLL for (int i = 0; i < N; i++) {
            rh[i] = ((fm >> i) & 1u) ? -r[i] : 0.0;
            sh[i] = 0.0;
        }
        fwd(rh);
        MT_UNROLL for (int i = 0; i < N; i++) p[i] = rh[i];
        double rr = dot(rh, rh);
        if (rr == 0.0) return kCgConv;
        if (exact) {
            cg_iters++;
            if (rr >= delta * delta) {
                const double sig = trqsol(sh, p);
                MT_UNROLL for (int i = 0; i < N; i++) sh[i] = sig * p[i];
                return kCgBnd;
            }
            MT_UNROLL for (int i = 0; i < N; i++) sh[i] = p[i];
            return kCgConv;
        }
        const double tol2 = cg_rtol * cg_rtol * rr;  // (cg_rtol ||r0||)^2
        for (int j = 0; j < m; j++) {
            cg_iters++;
            double z[N], q[N];
            MT_UNROLL for (int i = 0; i < N; i++) z[i] = p[i];
            bwd(z);
            hmul(z, q);
            MT_UNROLL for (int i = 0; i < N; i++) q[i] = ((fm >> i) & 1u) ? q[i] : 0.0;
            fwd(q);
            const double kap = dot(p, q);
            if (!(kap > 0.0)) {
                const double sig = trqsol(sh, p);
                MT_UNROLL for (int i = 0; i < N; i++) sh[i] = fma(sig, p[i], sh[i]);
                return kCgNeg;
            }
            const double a = rr / kap;
            double tv[N];
            MT_UNROLL for (int i = 0; i < N; i++) tv[i] = fma(a, p[i], sh[i]);
            if (dot(tv, tv) >= delta * delta) {
                const double sig = trqsol(sh, p);
                MT_UNROLL for (int i = 0; i < N; i++) sh[i] = fma(sig, p[i], sh[i]);
                return kCgBnd;
            }
            MT_UNROLL for (int i = 0; i < N; i++) {
                sh[i] = tv[i];
                rh[i] = fma(-a, q[i], rh[i]);
            }
            const double rrn = dot(rh, rh);
            if (rrn <= tol2) return kCgConv;
            const double b = rrn / rr;
            MT_UNROLL for (int i = 0; i < N; i++) p[i] = fma(b, p[i], rh[i]);
            rr = rrn;
        }
        return kCgMaxit;
    }

    MT_INLINE uint32_t free_mask(const double (&v)[N]) const
    {
        uint32_t fm = 0;
        MT_UNROLL for (int i = 0; i < N; i++)
            if (lo[i] < v[i] && v[i] < hi[i]) fm |= 1u << i;
        return fm;
    }

    MT_INLINE void subspace(double cg_rtol)
    {
        lfm = 0u;
        for (int pass = 0; pass < N; pass++) {
            const uint32_t fm = free_mask(xs);
            if (fm == 0u) break;
            const int m = __builtin_popcount(fm);
            // model gradient r = g + H s at s = xs - x
            double s[N], r[N];
            MT_UNROLL for (int i = 0; i < N; i++) s[i] = xs[i] - x[i];
            hmul(s, r);
            MT_UNROLL for (int i = 0; i < N; i++) r[i] += g[i];
            lfm = fm;
            double w[N];
            const double shift = precond(fm);
            const int ex = pcg(fm, m, r, w, cg_rtol, shift == 0.0);
            bwd(w);  // w = L^-T s_hat (zero outside F)
            // projected search on the model
            double beta = 1.0;
            bool acc = false;
            double xt[N];
            for (int t = 0; t <= kSearchHalvings; t++) {
                search_trials++;
                double d[N], hd[N];
                MT_UNROLL for (int i = 0; i < N; i++) {
                    xt[i] = clampf(fma(beta, w[i], xs[i]), lo[i], hi[i]);
                    d[i] = xt[i] - xs[i];
                }
                hmul(d, hd);
                const double rd = dot(r, d);
                const double dq = fma(0.5, dot(d, hd), rd);
                if (dq <= kMu0 * rd) { acc = true; break; }
                beta *= 0.5;
            }
            if (acc) MT_UNROLL for (int i = 0; i < N; i++) xs[i] = xt[i];
            const bool newly_bound = (fm & ~free_mask(xs)) != 0u;
            if (!((ex == kCgConv || ex == kCgMaxit) && newly_bound)) break;
        }
    }

    // step length in the norm of the trust region that bounded it: ||L^T s|| with the last
    // factored pass's L (identity outside its free set), else ||s||_2
    MT_INLINE double step_norm(const double (&s)[N]) const
    {
        if (lfm == 0u) return sqrt(dot(s, s));
        double ss = 0.0;
        MT_UNROLL for (int i = 0; i < N; i++) {
            double t = 0.0;
            MT_UNROLL for (int k = i; k < N; k++) t = fma(L[tri(k, i)], s[k], t);
            ss = fma(t, t, ss);
        }
        return sqrt(ss);
    }

    MT_INLINE double radius_update(double rho, double ared, double gts, double snorm, bool fin) const
    {
        double astar;
        if (!fin) {
            astar = kSig1;
            rho = -__builtin_inf();
        } else {
            const double gam = -ared - gts;
            if (gam <= 0.0) astar = kSig3;
            else {
                astar = -0.5 * gts / gam;
                if (astar < kSig1) astar = kSig1;
            }
        }
        if (rho <= kEta0) return dmin((astar > kSig1 ? astar : kSig1) * snorm, kSig2 * delta);
        if (rho <= kEta1) return dmax(kSig1 * delta, dmin(astar * snorm, kSig2 * delta));
        if (rho < kEta2) return dmax(kSig1 * delta, dmin(astar * snorm, kSig3 * delta));
        return dmax(delta, dmin(astar * snorm, kSig3 * delta));
    }

    // Whole solve; lo, hi, x (= x0 on entry), fam loaded. Returns the status.
    MT_INLINE int32_t solve(const Options &o, double delta_in, double alphac_in)
    {
        iters = 0; cg_iters = 0; cauchy_trials = 0; search_trials = 0; chol_tries = 0;
        delta = 0.0;
        alphac = 1.0;
        f = __builtin_nan("");
        bool bad = false;
        MT_UNROLL for (int i = 0; i < N; i++) bad = bad || !(lo[i] <= hi[i]);
        if (bad) return kBadBounds;
        MT_UNROLL for (int i = 0; i < N; i++) x[i] = clampb(x[i], lo[i], hi[i]);
        f = fam.fg(x, g);
        bool fin = isfinite(f);
        MT_UNROLL for (int i = 0; i < N; i++) fin = fin && isfinite(g[i]);
        if (!fin) return kNonfinite;
        if (pg_inf() <= o.gtol) return kConverged;
        if (o.warm && delta_in > 0.0) delta = delta_in;
        else if (o.delta0 > 0.0) delta = o.delta0;
        else {
            delta = pg_nrm2();
            if (delta == 0.0) delta = 1.0;
        }
        if (o.warm && alphac_in > 0.0) alphac = alphac_in;
        fam.hess(x);
        int32_t status;
        for (;;) {
            cauchy();
            subspace(o.cg_rtol);
            double s[N], hs[N];
            MT_UNROLL for (int i = 0; i < N; i++) s[i] = xs[i] - x[i];
            const double snorm = step_norm(s);
            const double gts = dot(g, s);
            hmul(s, hs);
            const double pred = -fma(0.5, dot(s, hs), gts);
            iters++;
            if (!(pred > 0.0)) { status = kStalled; break; }
            double gt[N];
            const double ft = fam.fg(xs, gt);
            const bool tfin = isfinite(ft);
            double ared = f - ft;
            if (tfin && pred <= kAredSwitch * (fabs(f) > 1.0 ? fabs(f) : 1.0)) {
                double sg = 0.0;
                MT_UNROLL for (int i = 0; i < N; i++) sg = fma(g[i] + gt[i], s[i], sg);
                ared = -0.5 * sg;
            }
            const double rho = tfin ? ared / pred : -__builtin_inf();
            delta = radius_update(rho, ared, gts, snorm, tfin);
            const bool accept = rho > kEta0;
            if (accept) {
                MT_UNROLL for (int i = 0; i < N; i++) { x[i] = xs[i]; g[i] = gt[i]; }
                f = ft;
            }
            bool ok = isfinite(f);
            MT_UNROLL for (int i = 0; i < N; i++) ok = ok && isfinite(g[i]);
            if (!ok) { status = kNonfinite; break; }
            if (pg_inf() <= o.gtol) { status = kConverged; break; }
            if (iters >= o.max_iter) { status = kMaxIter; break; }
            const double tiny = kStallRel * (fabs(f) > 1.0 ? fabs(f) : 1.0);
            if (tfin && fabs(ared) <= tiny && pred <= tiny) { status = kStalled; break; }
            if (accept) fam.hess(x);
        }
        return status;
    }
};

}  // namespace mt
