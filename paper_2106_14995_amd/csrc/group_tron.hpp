// group_tron.hpp -- one trust-region Newton solve per group of G consecutive lanes
// (G = 2, 4, 8 or 16), for n <= N <= 16: the thread configuration of section 4.2 swept over
// the width of the group that shares one instance.
//
// Lane k of a group owns rows i = k + G r, r < R = ceil(N / G), of every vector, and the
// same rows of the Hessian (hrow), of the Cholesky factor (lrow, entries left of the
// diagonal, the pivot on it) and the same columns of the factor (lcol[r][j] = L[j][i], j > i),
// all in registers (indices are compile-time after unrolling; only comparisons with the
// lane's own row index are run-time). Component j lives in group lane j mod G, slot j / G,
// and reaches the other lanes of the group by one DPP broadcast (quad permutations for
// G <= 4, row broadcasts for 8 and 16); sums and maxima are DPP butterflies whose result has
// the same bits in every lane of the group, so every decision of the method is taken
// identically by the group's lanes and a group never diverges from itself. Groups of one
// wave may take different paths (their own exec masks); a group never leaves its 16-lane
// DPP row. When G does not divide N (n = 6 on 4 or 8 lanes) the last slot of some lanes lies
// past N: an identity row of the factor (reciprocal pivot 1, set before each factorisation)
// whose vector entries stay zero.
//
// The steps and readings are those of lane_tron.hpp (Algorithm 1 with the TRON ratio test,
// the step measured in the trust region's norm, the trapezoid reduction near rounding
// level). The factorisation runs right-looking over columns (each finished column is
// broadcast entry by entry and subtracted from the later columns), which performs the same
// operations in the same order as the left-looking form of the lane kernel, so the factor
// has the same bits; the substitutions run over columns (forward ascending, backward
// descending), each step one broadcast and one multiply-add per row.
#pragma once

#include "wave_tron.hpp"

namespace mt {

MT_INLINE long long d2ll(double v) { return __double_as_longlong(v); }
MT_INLINE double ll2d(long long v) { return __longlong_as_double(v); }

// Cross-lane operations inside aligned groups of G lanes.
template <int G>
struct Grp {
    static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group width");

    // the value of group lane S, in every lane of the group
    template <int S>
    static MT_INLINE double bcast(double v)
    {
        if constexpr (G == 1) {
            return v;
        } else if constexpr (G == 2) {
            return dpp_mov<S | (S << 2) | ((2 + S) << 4) | ((2 + S) << 6)>(v);
        } else if constexpr (G == 4) {
            return dpp_mov<S * 0x55>(v);
        } else if constexpr (G == 8) {
            // lanes 0..7 of each row take the row's lane S, lanes 8..15 its lane 8 + S
            const long long a = __builtin_amdgcn_update_dpp(0ll, d2ll(v), 0x150 + S, 0xF, 0x3, false);
            return ll2d(__builtin_amdgcn_update_dpp(a, d2ll(v), 0x158 + S, 0xF, 0xC, false));
        } else {
            return ll2d(__builtin_amdgcn_update_dpp(0ll, d2ll(v), 0x150 + S, 0xF, 0xF, false));
        }
    }

    // bcast with s in [0, G), a constant once the caller's loops are unrolled
    static MT_INLINE double from(double v, int s)
    {
#define MT_GRP_CASE(c) \
    case c:            \
        if constexpr (c < G) return bcast<c>(v); else return v;
        switch (s) {
            MT_GRP_CASE(0) MT_GRP_CASE(1) MT_GRP_CASE(2) MT_GRP_CASE(3)
            MT_GRP_CASE(4) MT_GRP_CASE(5) MT_GRP_CASE(6) MT_GRP_CASE(7)
            MT_GRP_CASE(8) MT_GRP_CASE(9) MT_GRP_CASE(10) MT_GRP_CASE(11)
            MT_GRP_CASE(12) MT_GRP_CASE(13) MT_GRP_CASE(14)
        default:
            if constexpr (G == 16) return bcast<15>(v); else return v;
        }
#undef MT_GRP_CASE
    }

    // butterfly over the group: partners combined commutatively at every step
    static MT_INLINE double sum(double v)
    {
        if constexpr (G >= 2) v += dpp_mov<kDppSwap1>(v);
        if constexpr (G >= 4) v += dpp_mov<kDppSwap2>(v);
        if constexpr (G >= 8) v += dpp_mov<kDppHalfMirror>(v);
        if constexpr (G >= 16) v += dpp_mov<kDppMirror>(v);
        return v;
    }
    static MT_INLINE double max(double v)
    {
        if constexpr (G >= 2) v = max_nan(v, dpp_mov<kDppSwap1>(v));
        if constexpr (G >= 4) v = max_nan(v, dpp_mov<kDppSwap2>(v));
        if constexpr (G >= 8) v = max_nan(v, dpp_mov<kDppHalfMirror>(v));
        if constexpr (G >= 16) v = max_nan(v, dpp_mov<kDppMirror>(v));
        return v;
    }
    // the group's bits of a wave ballot, lane k of the group at bit k
    static MT_INLINE uint32_t bits(bool p)
    {
        const uint64_t b = __ballot(p);
        const int base = (int)(threadIdx.x & 63) & ~(G - 1);
        return (uint32_t)(b >> base) & (G == 32 ? 0xFFFFFFFFu : ((1u << G) - 1u));
    }
    static MT_INLINE bool any(bool p) { return bits(p) != 0u; }
    static MT_INLINE bool all(bool p) { return bits(!p) == 0u; }
};

// ------------------------------------------------------------------------------------
// Families of the group solver. Each provides load(s, p, n), fg(s, v, va, g) -> f at the
// distributed point v (va: all of its components, in every lane; g: the gradient on the
// lane's rows), hess(s, v, va) (the Hessian at v), H(s, r, j) (its entry j of the lane's row
// slot r) and diag(r) (the diagonal entry of slot r). Comparisons with the lane's own row
// index go through s.eq / s.gt / s.ge, whose masks are opaque to the compiler: a chain of
// selects on "row == j" would otherwise be turned into an indexed array in scratch memory.
// ------------------------------------------------------------------------------------
template <int N, int G>
struct GQP4 {
    static constexpr int R = (N + G - 1) / G;
    static constexpr double pad = 0.0;
    double q[R][N];  // rows of Q on the lane's rows (zero outside the instance)
    double c[R];
    double hd[R];    // the Hessian's diagonal on the lane's rows (Q's diagonal + 12 kappa x^2)
    double kap;

    template <class S>
    MT_INLINE void load(const S &s, const double *__restrict__ p, int n)
    {
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = s.row(r);
            MT_UNROLL for (int j = 0; j < N; j++) {
                const bool in = i < n && j < n;
                q[r][j] = in ? p[in ? tri(i, j) : 0] : 0.0;
            }
        }
        const double *cp = p + n * (n + 1) / 2;
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = s.row(r);
            c[r] = i < n ? cp[i < n ? i : 0] : 0.0;
        }
        kap = cp[n];
    }
    template <class S>
    MT_INLINE double fg(const S &, const double (&v)[R], const double (&va)[N], double (&g)[R]) const
    {
        double acc = 0.0;
        const double k4 = 4.0 * kap;
        MT_UNROLL for (int r = 0; r < R; r++) {
            double y = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) y = fma(q[r][j], va[j], y);
            const double x2 = v[r] * v[r];
            g[r] = fma(k4 * x2, v[r], y + c[r]);
            acc = fma(v[r], fma(0.5, y, c[r]), acc);
            acc = fma(kap * x2, x2, acc);
        }
        return Grp<G>::sum(acc);
    }
    template <class S>
    MT_INLINE void hess(S &s, const double (&v)[R], const double (&)[N])
    {
        const double k12 = 12.0 * kap;
        MT_UNROLL for (int r = 0; r < R; r++) {
            double qd = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) qd = s.eq(r, j) ? q[r][j] : qd;
            hd[r] = fma(k12 * v[r], v[r], qd);
        }
    }
    // H[i][j] on the lane's row slot r (i its row)
    template <class S>
    MT_INLINE double H(const S &s, int r, int j) const { return s.eq(r, j) ? hd[r] : q[r][j]; }
    MT_INLINE double diag(int r) const { return hd[r]; }
};

// HS45M: f = 120 - prod x_k, products left to right with the excluded factors as 1.
template <int N, int G>
struct GHS45M {
    static constexpr int R = (N + G - 1) / G;
    static constexpr double pad = 1.0;
    double hrow[R][N];

    template <class S>
    MT_INLINE void load(const S &, const double *__restrict__, int) {}
    template <class S>
    MT_INLINE double fg(const S &s, const double (&)[R], const double (&va)[N], double (&g)[R]) const
    {
        double pr = 1.0;
        MT_UNROLL for (int k = 0; k < N; k++) pr *= va[k];
        MT_UNROLL for (int r = 0; r < R; r++) {
            double q = 1.0;
            MT_UNROLL for (int k = 0; k < N; k++) q *= s.eq(r, k) ? 1.0 : va[k];
            g[r] = -q;
        }
        return 120.0 - pr;
    }
    template <class S>
    MT_INLINE void hess(S &s, const double (&)[R], const double (&va)[N])
    {
        MT_UNROLL for (int r = 0; r < R; r++) {
            MT_UNROLL for (int j = 0; j < N; j++) {
                double q = 1.0;
                MT_UNROLL for (int k = 0; k < N; k++) q *= (s.eq(r, k) || k == j) ? 1.0 : va[k];
                hrow[r][j] = s.eq(r, j) ? 0.0 : -q;
            }
        }
    }
    template <class S>
    MT_INLINE double H(const S &, int r, int j) const { return hrow[r][j]; }
    MT_INLINE double diag(int) const { return 0.0; }
};

// BR6 (n = 6): every lane of the group evaluates the whole instance (the evaluation is a
// handful of flows around one sine and cosine) and keeps its own rows.
template <int G>
struct GBR6 {
    static constexpr int N = 6;
    static constexpr int R = (N + G - 1) / G;
    static constexpr double pad = 0.0;
    BR6R b6;
    double hrow[R][N];
    double hdg[R];

    template <class S>
    MT_INLINE void load(const S &, const double *__restrict__ p, int n) { b6.load(p, n); }
    template <class S>
    MT_INLINE double fg(const S &s, const double (&)[R], const double (&va)[N], double (&g)[R])
    {
        double gf[N];
        const double f = b6.fg(va, gf);
        MT_UNROLL for (int r = 0; r < R; r++) {
            double t = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) t = s.eq(r, j) ? gf[j] : t;
            g[r] = t;
        }
        return f;
    }
    template <class S>
    MT_INLINE void hess(S &s, const double (&)[R], const double (&va)[N])
    {
        b6.hess(va);
        MT_UNROLL for (int r = 0; r < R; r++) {
            double dg = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) {
                double t = 0.0;
                MT_UNROLL for (int ii = 0; ii < N; ii++) t = s.eq(r, ii) ? b6.H(ii, j) : t;
                hrow[r][j] = t;
                dg = s.eq(r, j) ? t : dg;
            }
            hdg[r] = dg;
        }
    }
    template <class S>
    MT_INLINE double H(const S &, int r, int j) const { return hrow[r][j]; }
    MT_INLINE double diag(int r) const { return hdg[r]; }
};

// ------------------------------------------------------------------------------------
// The solver for one group.
// ------------------------------------------------------------------------------------
template <class Fam, int N, int G>
struct GroupTron {
    static_assert(N >= 1 && N <= 16, "the group solver holds n <= 16");
    static constexpr int R = (N + G - 1) / G;
    using X = Grp<G>;
    Fam fam;
    int n;                 // the instance's size (<= N); rows at or past n are fixed padding
    int k;                 // lane within the group
    double lo[R], hi[R], x[R], g[R], xs[R], dinv[R];
    double lrow[R][N];     // factor rows: L[i][j] for j < i, the pivot at j = i
    double lcol[R][N];     // factor columns: L[j][i] for j > i
    uint32_t lfm;          // free set of the last factored pass (0: none this iteration)
    uint32_t ohm[R], ltm[R];  // per row slot: bit i (the row) and bits below i, opaque
    double f, delta, alphac;
    int32_t iters;

    MT_INLINE int row(int r) const { return k + G * r; }
    MT_INLINE bool bit(uint32_t m, int i) const { return (m >> i) & 1u; }
    // the slot's row equals / exceeds / is at least j (j a constant after unrolling)
    MT_INLINE bool eq(int r, int j) const { return (ohm[r] >> j) & 1u; }
    MT_INLINE bool gt(int r, int j) const { return (ltm[r] >> j) & 1u; }
    MT_INLINE bool ge(int r, int j) const { return ((ltm[r] | ohm[r]) >> j) & 1u; }
    MT_INLINE void set_lane(int lane_in_group)
    {
        k = lane_in_group;
        MT_UNROLL for (int r = 0; r < R; r++) {
            uint32_t o = 1u << row(r), l = (1u << row(r)) - 1u;
            asm volatile("" : "+v"(o), "+v"(l));
            ohm[r] = o;
            ltm[r] = l;
        }
    }

    // component j of a row-distributed vector, in every lane of the group
    MT_INLINE double comp(const double (&v)[R], int j) const
    {
        double t = v[j / G];
        asm volatile("" : "+v"(t));  // one broadcast per use: no common subexpression held live
        return X::from(t, j % G);
    }
    MT_INLINE void all(const double (&v)[R], double (&va)[N]) const
    {
        MT_UNROLL for (int j = 0; j < N; j++) va[j] = comp(v, j);
    }
    MT_INLINE double dot(const double (&a)[R], const double (&b)[R]) const
    {
        double s = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) s = fma(a[r], b[r], s);
        return X::sum(s);
    }
    MT_INLINE void hmul(const double (&v)[R], double (&out)[R]) const
    {
        double va[N];
        all(v, va);
        MT_UNROLL for (int r = 0; r < R; r++) {
            double s = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) s = fma(fam.H(*this, r, j), va[j], s);
            out[r] = s;
        }
    }
    MT_INLINE double fg(const double (&v)[R], double (&gr)[R])
    {
        double va[N];
        all(v, va);
        return fam.fg(*this, v, va, gr);
    }
    MT_INLINE void hess(const double (&v)[R])
    {
        double va[N];
        all(v, va);
        fam.hess(*this, v, va);
    }
    MT_INLINE double pg_inf() const
    {
        double m = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) m = fmax(m, fabs(pg_comp(x[r], lo[r], hi[r], g[r])));
        return X::max(m);
    }
    MT_INLINE double pg_nrm2() const
    {
        double s = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) {
            const double v = pg_comp(x[r], lo[r], hi[r], g[r]);
            s = fma(v, v, s);
        }
        return sqrt(X::sum(s));
    }
    // L y = b in place: step j broadcasts y_j (scaled in its owner) and every later row
    // subtracts it; rows keep their residual unscaled until the end
    MT_INLINE void fwd(double (&b)[R]) const
    {
        MT_UNROLL for (int j = 0; j < N; j++) {
            const double yj = X::from(b[j / G] * dinv[j / G], j % G);
            MT_UNROLL for (int r = 0; r < R; r++) {
                const double u = fma(-lrow[r][j], yj, b[r]);
                b[r] = gt(r, j) ? u : b[r];
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++) b[r] *= dinv[r];
    }
    // L^T y = b in place, steps from the last column down
    MT_INLINE void bwd(double (&b)[R]) const
    {
        MT_UNROLL for (int j = N - 1; j >= 0; j--) {
            const double yj = X::from(b[j / G] * dinv[j / G], j % G);
            MT_UNROLL for (int r = 0; r < R; r++) {
                const double u = fma(-lcol[r][j], yj, b[r]);
                b[r] = ge(r, j) ? b[r] : u;
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++) b[r] *= dinv[r];
    }
    MT_INLINE double trqsol(const double (&v)[R], const double (&p)[R]) const
    {
        const double ptx = dot(p, v), ptp = dot(p, p), xtx = dot(v, v);
        const double dsq = delta * delta;
        double disc = fma(ptx, ptx, ptp * (dsq - xtx));
        disc = disc < 0.0 ? 0.0 : disc;
        const double rad = sqrt(disc);
        const double sig = ptx >= 0.0 ? (dsq - xtx) / (ptx + rad) : (rad - ptx) / ptp;
        return sig > 0.0 ? sig : 0.0;
    }
    MT_INLINE bool cauchy_trial(double a, double (&xt)[R])
    {
        double st[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            xt[r] = clampf(fma(-a, g[r], x[r]), lo[r], hi[r]);
            st[r] = xt[r] - x[r];
        }
        if (!(dot(st, st) <= delta * delta)) return false;
        const double gts = dot(g, st);
        double hs[R];
        hmul(st, hs);
        const double q = fma(0.5, dot(st, hs), gts);
        return q <= kMu0 * gts;
    }
    MT_INLINE bool below_last_breakpoint(double a) const
    {
        bool any = false, below = false;
        MT_UNROLL for (int r = 0; r < R; r++) {
            const double d = -g[r];
            const bool up = d > 0.0 && isfinite(hi[r]);
            const bool dn = d < 0.0 && isfinite(lo[r]);
            any = any || up || dn;
            below = below || (up && a * d < hi[r] - x[r]) || (dn && a * d > lo[r] - x[r]);
        }
        return !X::any(any) || X::any(below);
    }
    MT_INLINE void cauchy()
    {
        double a = alphac;
        double xt[R];
        if (cauchy_trial(a, xt)) {
            MT_UNROLL for (int r = 0; r < R; r++) xs[r] = xt[r];
            for (int t = 0; t < kCauchyMax; t++) {
                if (!below_last_breakpoint(a)) break;
                const double a2 = 10.0 * a;
                if (!cauchy_trial(a2, xt)) break;
                a = a2;
                MT_UNROLL for (int r = 0; r < R; r++) xs[r] = xt[r];
            }
        } else {
            for (int t = 0; t < kCauchyMax; t++) {
                a = 0.1 * a;
                if (cauchy_trial(a, xt)) break;
            }
            MT_UNROLL for (int r = 0; r < R; r++) xs[r] = xt[r];
        }
        alphac = a;
    }
    MT_INLINE uint32_t free_mask(const double (&v)[R]) const
    {
        uint32_t m = 0u;
        MT_UNROLL for (int r = 0; r < R; r++) m |= X::bits(lo[r] < v[r] && v[r] < hi[r]) << (G * r);
        return N >= 32 ? m : (m & ((1u << N) - 1u));
    }

    // Factor of the masked, shifted matrix (rows and columns outside fm are the identity),
    // right-looking: column j is scaled by its pivot, then each of its entries L[c][j] is
    // broadcast and subtracted from column c of the later rows (and kept by column j's owner
    // in lcol).
    MT_INLINE bool chol(uint32_t fm, double alpha)
    {
        MT_UNROLL for (int r = 0; r < R; r++) {
            // the column loop below sets the reciprocal pivot of rows < N only; a slot past N
            // (G R > N, e.g. n = 6 on groups of 4 or 8) is an identity row of the factor, and
            // the substitutions scale every slot, so it needs its 1 here
            dinv[r] = 1.0;
            const bool fi = bit(fm, row(r));
            MT_UNROLL for (int j = 0; j < N; j++) {
                const double h = fam.H(*this, r, j);
                lrow[r][j] = eq(r, j) ? (fi ? h + alpha : 1.0) : ((fi && bit(fm, j)) ? h : 0.0);
            }
        }
        bool ok = true;
        MT_UNROLL for (int j = 0; j < N; j++) {
            const bool fj = bit(fm, j);
            const double d = X::from(lrow[j / G][j], j % G);
            ok = ok && (!fj || d > 0.0);
            const double rj = fj ? rsqrt_pos(fj ? d : 1.0) : 1.0;
            const double piv = fj ? d * rj : 1.0;
            MT_UNROLL for (int r = 0; r < R; r++) {
                const double l = (fj && bit(fm, row(r))) ? lrow[r][j] * rj : 0.0;
                lrow[r][j] = gt(r, j) ? l : (eq(r, j) ? piv : lrow[r][j]);
                dinv[r] = eq(r, j) ? rj : dinv[r];
            }
            const bool owner = k == j % G;
            MT_UNROLL for (int c = j + 1; c < N; c++) {
                const double lcj = X::from(lrow[c / G][j], c % G);
                MT_UNROLL for (int r = 0; r < R; r++) {
                    const double u = fma(-lrow[r][j], lcj, lrow[r][c]);
                    lrow[r][c] = ge(r, c) ? u : lrow[r][c];
                }
                lcol[j / G][c] = owner ? lcj : lcol[j / G][c];
            }
        }
        return ok;
    }
    // the shift that succeeded (the diagonal fallback after kShiftTries failures)
    MT_INLINE double precond(uint32_t fm)
    {
        double mn = __builtin_inf(), mx = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) {
            const double v = fam.diag(r);
            if (bit(fm, row(r))) {
                mn = v < mn ? v : mn;
                mx = fabs(v) > mx ? fabs(v) : mx;
            }
        }
        mn = -X::max(-mn);
        mx = X::max(mx);
        const double beta = 1e-3 * (mx > 1.0 ? mx : 1.0);
        double alpha = mn > 0.0 ? 0.0 : beta - mn;
        for (int t = 0; t < kShiftTries; t++) {
            if (chol(fm, alpha)) return alpha;
            alpha = 2.0 * alpha > beta ? 2.0 * alpha : beta;
        }
        MT_UNROLL for (int r = 0; r < R; r++) {
            const double v = fabs(fam.diag(r));
            const double piv = bit(fm, row(r)) ? sqrt(v > beta ? v : beta) : 1.0;
            MT_UNROLL for (int j = 0; j < N; j++) {
                lrow[r][j] = eq(r, j) ? piv : 0.0;
                lcol[r][j] = 0.0;
            }
            dinv[r] = 1.0 / piv;
        }
        return -1.0;
    }
    // exact: no shift was needed; the first CG step is the whole solve (see lane_tron.hpp)
    MT_INLINE int pcg(uint32_t fm, int m, const double (&rv)[R], double (&sh)[R], double cg_rtol, bool exact)
    {
        double rh[R], p[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            rh[r] = bit(fm, row(r)) ? -rv[r] : 0.0;
            sh[r] = 0.0;
        }
        fwd(rh);
        MT_UNROLL for (int r = 0; r < R; r++) p[r] = rh[r];
        double rr = dot(rh, rh);
        if (rr == 0.0) return kCgConv;
        if (exact) {
            if (rr >= delta * delta) {
                const double sig = trqsol(sh, p);
                MT_UNROLL for (int r = 0; r < R; r++) sh[r] = sig * p[r];
                return kCgBnd;
            }
            MT_UNROLL for (int r = 0; r < R; r++) sh[r] = p[r];
            return kCgConv;
        }
        const double tol2 = cg_rtol * cg_rtol * rr;
        for (int j = 0; j < m; j++) {
            double z[R], q[R];
            MT_UNROLL for (int r = 0; r < R; r++) z[r] = p[r];
            bwd(z);
            hmul(z, q);
            MT_UNROLL for (int r = 0; r < R; r++) q[r] = bit(fm, row(r)) ? q[r] : 0.0;
            fwd(q);
            const double kap = dot(p, q);
            if (!(kap > 0.0)) {
                const double sig = trqsol(sh, p);
                MT_UNROLL for (int r = 0; r < R; r++) sh[r] = fma(sig, p[r], sh[r]);
                return kCgNeg;
            }
            const double a = rr / kap;
            double tv[R];
            MT_UNROLL for (int r = 0; r < R; r++) tv[r] = fma(a, p[r], sh[r]);
            if (dot(tv, tv) >= delta * delta) {
                const double sig = trqsol(sh, p);
                MT_UNROLL for (int r = 0; r < R; r++) sh[r] = fma(sig, p[r], sh[r]);
                return kCgBnd;
            }
            MT_UNROLL for (int r = 0; r < R; r++) {
                sh[r] = tv[r];
                rh[r] = fma(-a, q[r], rh[r]);
            }
            const double rrn = dot(rh, rh);
            if (rrn <= tol2) return kCgConv;
            const double b = rrn / rr;
            MT_UNROLL for (int r = 0; r < R; r++) p[r] = fma(b, p[r], rh[r]);
            rr = rrn;
        }
        return kCgMaxit;
    }
    MT_INLINE void subspace(double cg_rtol)
    {
        lfm = 0u;
        for (int pass = 0; pass < N; pass++) {
            const uint32_t fm = free_mask(xs);
            if (fm == 0u) break;
            const int m = __builtin_popcount(fm);
            double s[R], rv[R];
            MT_UNROLL for (int r = 0; r < R; r++) s[r] = xs[r] - x[r];
            hmul(s, rv);
            MT_UNROLL for (int r = 0; r < R; r++) rv[r] += g[r];
            lfm = fm;
            const double shift = precond(fm);
            double w[R];
            const int ex = pcg(fm, m, rv, w, cg_rtol, shift == 0.0);
            bwd(w);
            double beta = 1.0;
            bool acc = false;
            double xt[R];
            for (int t = 0; t <= kSearchHalvings; t++) {
                double d[R], hd[R];
                MT_UNROLL for (int r = 0; r < R; r++) {
                    xt[r] = clampf(fma(beta, w[r], xs[r]), lo[r], hi[r]);
                    d[r] = xt[r] - xs[r];
                }
                hmul(d, hd);
                const double rd = dot(rv, d);
                const double dq = fma(0.5, dot(d, hd), rd);
                if (dq <= kMu0 * rd) { acc = true; break; }
                beta *= 0.5;
            }
            if (acc) MT_UNROLL for (int r = 0; r < R; r++) xs[r] = xt[r];
            const bool newly_bound = (fm & ~free_mask(xs)) != 0u;
            if (!((ex == kCgConv || ex == kCgMaxit) && newly_bound)) break;
        }
    }
    // ||L^T s|| on the last factored pass (L the identity outside its free set), else ||s||
    MT_INLINE double step_norm(const double (&s)[R]) const
    {
        if (lfm == 0u) return sqrt(dot(s, s));
        double sa[N];
        all(s, sa);
        double ss = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) {
            double t = 0.0;
            MT_UNROLL for (int j = 0; j < N; j++) {
                const double u = fma(eq(r, j) ? lrow[r][j] : lcol[r][j], sa[j], t);
                t = gt(r, j) ? t : u;
            }
            ss = fma(t, t, ss);
        }
        return sqrt(X::sum(ss));
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
    MT_INLINE bool finite_all(double fv, const double (&v)[R]) const
    {
        bool fin = true;
        MT_UNROLL for (int r = 0; r < R; r++) fin = fin && isfinite(v[r]);
        return isfinite(fv) && X::all(fin);
    }

    // Whole solve; lo, hi, x (= x0 on entry) and the family loaded. Returns the status.
    MT_INLINE int32_t solve(const Options &o, double delta_in, double alphac_in)
    {
        iters = 0;
        delta = 0.0;
        alphac = 1.0;
        f = __builtin_nan("");
        bool bad = false;
        MT_UNROLL for (int r = 0; r < R; r++) bad = bad || !(lo[r] <= hi[r]);
        if (X::any(bad)) return kBadBounds;
        MT_UNROLL for (int r = 0; r < R; r++) x[r] = clampb(x[r], lo[r], hi[r]);
        f = fg(x, g);
        if (!finite_all(f, g)) return kNonfinite;
        if (pg_inf() <= o.gtol) return kConverged;
        if (o.warm && delta_in > 0.0) delta = delta_in;
        else if (o.delta0 > 0.0) delta = o.delta0;
        else {
            delta = pg_nrm2();
            if (delta == 0.0) delta = 1.0;
        }
        if (o.warm && alphac_in > 0.0) alphac = alphac_in;
        hess(x);
        int32_t status;
        for (;;) {
            cauchy();
            subspace(o.cg_rtol);
            double s[R], hs[R];
            MT_UNROLL for (int r = 0; r < R; r++) s[r] = xs[r] - x[r];
            const double snorm = step_norm(s);
            const double gts = dot(g, s);
            hmul(s, hs);
            const double pred = -fma(0.5, dot(s, hs), gts);
            iters++;
            if (!(pred > 0.0)) { status = kStalled; break; }
            double gt[R];
            const double ft = fg(xs, gt);
            const bool tfin = isfinite(ft);
            double ared = f - ft;
            if (tfin && pred <= kAredSwitch * (fabs(f) > 1.0 ? fabs(f) : 1.0)) {
                double sg = 0.0;
                MT_UNROLL for (int r = 0; r < R; r++) sg = fma(g[r] + gt[r], s[r], sg);
                ared = -0.5 * X::sum(sg);
            }
            const double rho = tfin ? ared / pred : -__builtin_inf();
            delta = radius_update(rho, ared, gts, snorm, tfin);
            const bool accept = rho > kEta0;
            if (accept) {
                MT_UNROLL for (int r = 0; r < R; r++) { x[r] = xs[r]; g[r] = gt[r]; }
                f = ft;
            }
            if (!finite_all(f, g)) { status = kNonfinite; break; }
            if (pg_inf() <= o.gtol) { status = kConverged; break; }
            if (iters >= o.max_iter) { status = kMaxIter; break; }
            const double tiny = kStallRel * (fabs(f) > 1.0 ? fabs(f) : 1.0);
            if (tfin && fabs(ared) <= tiny && pred <= tiny) { status = kStalled; break; }
            if (accept) hess(x);
        }
        return status;
    }
};

}  // namespace mt
