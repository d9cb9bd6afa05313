// wave_tron.hpp -- one trust-region Newton solve per wavefront, for 8 < n <= 512.
//
// Lane l of the wave owns rows i = l + 64 r, r < R, of every vector (R = 1 up to n = 64, 2 up
// to 128, then 4 and 8 with the matrix array in global memory). The n x n Hessian and its
// Cholesky factor share one array (LDS up to n = 128) of n rows and odd
// row stride ld >= n + 1 (odd, so that both row and column walks touch distinct banks): the
// Hessian's upper triangle with its diagonal, the factor's strict lower triangle below it,
// and the factor's pivots in the spare column n. A Hessian-vector product then reads every
// H_kj from one address, min(j,k) ld + max(j,k) = min(j,k) (ld - 1) + j + k, with no
// special case on the diagonal.
// Every decision of the method is taken on wave-reduced, wave-uniform values (the free set
// is a 64-bit ballot), so the 64 lanes never diverge.
// Sums use a butterfly of lane swaps (every lane ends with the same bits); the pivots and
// solution components of the triangular solves are broadcast with readlane. The Cholesky
// factorisation is blocked in panels of 16 columns: FP64 matrix-core products form each
// panel from the columns before it, and the panel is factored in registers (chol_panels).
//
// The steps and readings are those of lane_tron.hpp (Algorithm 1 with the TRON ratio test,
// the step measured in the trust region's norm, and the trapezoid reduction near rounding
// level); only the data layout differs.
#pragma once

#include "lane_tron.hpp"

namespace mt {

// DPP lane permutation within 16-lane rows (VALU only, no LDS traffic)
template <int CTRL>
MT_INLINE double dpp_mov(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}
constexpr int kDppSwap1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int kDppSwap2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int kDppHalfMirror = 0x141; // lane i <- 7 - i within 8 lanes
constexpr int kDppMirror = 0x140;     // lane i <- 15 - i within 16 lanes

MT_INLINE double bcast(double v, int src);

// Sum over the 64 lanes; every lane returns the same bits: within each 16-lane row the
// partners of every step are combined commutatively, and the four row sums are read back
// and added in one fixed order.
MT_INLINE double wave_sum(double v)
{
    v += dpp_mov<kDppSwap1>(v);
    v += dpp_mov<kDppSwap2>(v);
    v += dpp_mov<kDppHalfMirror>(v);
    v += dpp_mov<kDppMirror>(v);
    return (bcast(v, 0) + bcast(v, 16)) + (bcast(v, 32) + bcast(v, 48));
}

// make a value the compiler treats as per-lane into a scalar (all lanes hold the same bits)
MT_INLINE double uni(double v)
{
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

MT_INLINE double bcast(double v, int src)
{
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
    return __hiloint2double(hi, lo);
}

MT_INLINE double max_nan(double a, double b) { return (b > a || b != b) ? b : a; }  // NaN propagates

MT_INLINE double wave_max(double v)
{
    v = max_nan(v, dpp_mov<kDppSwap1>(v));
    v = max_nan(v, dpp_mov<kDppSwap2>(v));
    v = max_nan(v, dpp_mov<kDppHalfMirror>(v));
    v = max_nan(v, dpp_mov<kDppMirror>(v));
    return max_nan(max_nan(bcast(v, 0), bcast(v, 16)), max_nan(bcast(v, 32), bcast(v, 48)));
}

// Objective families of the wave kernel. Each holds its own per-lane data and supplies
//   load(s, p)     read the instance's parameters (after the solver has read l, u, x0);
//   fg(s, v, g)    f(v) and its gradient on the lane's rows (0 on rows >= n);
//   hess(s)        the Hessian at s.x: its diagonal into s.hd, its strict upper triangle
//                  into the LDS array s.M when it depends on x.
// QP4: f = x'Qx/2 + c'x + kappa sum x_i^4 (Q packed lower by rows, then c, then kappa); the
// strict upper triangle of H is Q's and is written once at load.
template <int R_>
struct WaveFamQP4 {
    static constexpr int R = R_;
    double qd[R], c[R];  // Q's diagonal and c on the lane's rows
    double kap;

    template <class S>
    MT_INLINE void load(S &s, const double *__restrict__ p)
    {
        const int n = s.n;
        const double *cp = p + n * (n + 1) / 2;
        kap = cp[n];
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = s.row(r);
            const bool in = i < n;
            const int k = in ? i : 0;
            qd[r] = in ? p[k * (k + 1) / 2 + k] : 0.0;
            c[r] = in ? cp[k] : 0.0;
        }
        // strict upper part of Q (row i, column j > i = packed lower entry (j, i)); at each j
        // the lanes i < j read consecutive addresses
        for (int j = 1; j < n; j++) {
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = s.row(r);
                if (i < j) s.M[i * s.ld + j] = p[j * (j + 1) / 2 + i];
            }
        }
    }

    template <class S>
    MT_INLINE double fg(const S &s, const double (&v)[R], double (&gr)[R]) const
    {
        double y[R];
        s.amul(v, qd, y);
        double acc = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) {
            const double x2 = v[r] * v[r];
            gr[r] = s.valid(r) ? fma(4.0 * kap * x2, v[r], y[r] + c[r]) : 0.0;
            acc = fma(v[r], fma(0.5, y[r], c[r]), acc);
            acc = fma(kap * x2, x2, acc);
        }
        return uni(wave_sum(acc));
    }

    template <class S>
    MT_INLINE void hess(S &s) const
    {
        MT_UNROLL for (int r = 0; r < R; r++) {
            s.hd[r] = fma(12.0 * kap * s.x[r], s.x[r], qd[r]);
            if (s.valid(r)) s.M[s.row(r) * (s.ld + 1)] = s.hd[r];
        }
        s.sync();
    }
};

// HS45M: f = 120 - prod_k x_k (no parameters). Products run over k in ascending order with
// the excluded factors replaced by 1 (exact), so f and every gradient component carry the
// rounding of the plain left-to-right product.
template <int R_>
struct WaveFamHS45M {
    static constexpr int R = R_;

    template <class S>
    MT_INLINE void load(S &, const double *__restrict__) {}

    template <class S>
    MT_INLINE double fg(const S &s, const double (&v)[R], double (&gr)[R]) const
    {
        double pr = 1.0, q[R];
        MT_UNROLL for (int r = 0; r < R; r++) q[r] = 1.0;
        for (int k = 0; k < s.n; k++) {
            const double xk = s.comp(v, k);
            pr *= xk;
            MT_UNROLL for (int r = 0; r < R; r++) q[r] *= s.row(r) == k ? 1.0 : xk;
        }
        MT_UNROLL for (int r = 0; r < R; r++) gr[r] = s.valid(r) ? -q[r] : 0.0;
        return 120.0 - pr;
    }

    // H_ij = -prod_{k != i, j} x_k, H_ii = 0. Row i is the product of prefix and suffix
    // products of y = x with y_i = 1: H_ij = -(prod_{k < j} y_k)(prod_{k > j} y_k). The prefix
    // is stored in the strict upper row, then scaled by the suffix in a backward sweep.
    template <class S>
    MT_INLINE void hess(S &s) const
    {
        const int n = s.n, ld = s.ld;
        double pre[R];
        MT_UNROLL for (int r = 0; r < R; r++) pre[r] = 1.0;
        for (int j = 0; j < n; j++) {
            const double xj = s.comp(s.x, j);
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = s.row(r);
                if (i < j) s.M[i * ld + j] = pre[r];
                pre[r] *= i == j ? 1.0 : xj;
            }
        }
        double suf[R];
        MT_UNROLL for (int r = 0; r < R; r++) suf[r] = 1.0;
        for (int j = n - 1; j >= 0; j--) {
            const double xj = s.comp(s.x, j);
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = s.row(r);
                if (i < j) s.M[i * ld + j] = -(s.M[i * ld + j] * suf[r]);
                suf[r] *= i == j ? 1.0 : xj;
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++) {
            s.hd[r] = 0.0;
            if (s.valid(r)) s.M[s.row(r) * (ld + 1)] = 0.0;
        }
        s.sync();
    }
};

// One trust-region Newton solve per wave for the family Fam, Fam::R rows per lane
// (n <= 64 R).
// kGlobal: the matrix array M lives in global memory (a device workspace, for n > 128)
// instead of LDS; only the scope of the ordering between the lanes' writes and reads changes.
template <class Fam, bool kGlobal = false>
struct WaveTron {
    static constexpr int R = Fam::R;

    // order LDS writes before other lanes' LDS reads (the wave's LDS operations run in order)
    MT_INLINE void lds_sync() const
    {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }

    // make every lane's writes to M visible to every lane of the wave
    MT_INLINE void sync() const
    {
        if (kGlobal) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        } else {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
    }
    Fam fam;
    int n, ld, lane;
    double *M;                 // LDS: H upper with diagonal, L strict lower, pivots in column n
    double *P;                 // with M in global memory: LDS copy of a panel's 16 x 16 block
                               // of L (row stride 17), so that its columns meet at wave scope
    double *Q;                 // with M in global memory: kStage steps of each lane's entries of
                               // L, parked in LDS by the substitutions (slot (t R + r) 64 + lane)
    static constexpr int kStage = R >= 8 ? 4 : 8;  // 32 values in flight per lane
    double hd[R];              // H diagonal (own rows)
    double lo[R], hi[R], x[R], g[R], xs[R], dinv[R];
    uint64_t lfm[R];           // free set of the last factored pass
    bool has_l;
    double f, delta, alphac;
    int32_t iters;

    MT_INLINE int row(int r) const { return lane + 64 * r; }
    MT_INLINE bool valid(int r) const { return row(r) < n; }

    MT_INLINE double dot(const double (&a)[R], const double (&b)[R]) const
    {
        double s = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) s = fma(a[r], b[r], s);
        return uni(wave_sum(s));
    }

    // H_kj (upper triangle, diagonal included) sits at min(j,k) ld + max(j,k) = min(j,k)
    // (ld - 1) + j + k: with blk = M + k + j0 for a block of columns j = j0 + u (u a
    // constant after unrolling), the j0 + k part is the block's base, u an immediate offset,
    // and the rest one 24-bit multiply-add into a byte offset (indices stay far below 2^24);
    // ldb = 8 (ld - 1)
    MT_INLINE double hrd(const double *blk, unsigned ldb, int k, int j, int u) const
    {
        if constexpr (kGlobal) {
            // in global memory a 32-bit element index off the wave's uniform base keeps the
            // loads in their scalar-base form (a per-lane 64-bit base costs more than it saves)
            const int a = j < k ? j : k, b = j < k ? k : j;
            return M[(int)__umul24((unsigned)a, (unsigned)ld) + b];
        } else {
            const unsigned m = (unsigned)(j < k ? j : k);
            return *(const double *)((const char *)blk + __umul24(m, ldb) + 8 * u);
        }
    }

    // y = H v over the first n rows (H's diagonal read from LDS, as hess() stored it); rows
    // >= n give 0. Four independent accumulators per row; no lane-dependent branches.
    MT_INLINE void hmul(const double (&v)[R], double (&y)[R]) const
    {
        double acc[R][4];
        int kk[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;
            kk[r] = row(r) < n ? row(r) : 0;
        }
        const unsigned ldb = 8u * (unsigned)(ld - 1);
        MT_UNROLL for (int rr = 0; rr < R; rr++) {
            const int jend = n - 64 * rr < 64 ? n - 64 * rr : 64;
            int jj = 0;
            for (; jj + 4 <= jend; jj += 4) {
                double vj[4];
                MT_UNROLL for (int u = 0; u < 4; u++) vj[u] = bcast(v[rr], jj + u);
                MT_UNROLL for (int r = 0; r < R; r++) {
                    const double *blk = M + kk[r] + 64 * rr + jj;
                    MT_UNROLL for (int u = 0; u < 4; u++)
                        acc[r][u] = fma(hrd(blk, ldb, kk[r], 64 * rr + jj + u, u), vj[u], acc[r][u]);
                }
            }
            for (; jj < jend; jj++) {
                const double vj = bcast(v[rr], jj);
                MT_UNROLL for (int r = 0; r < R; r++)
                    acc[r][0] = fma(hrd(M + kk[r] + 64 * rr + jj, ldb, kk[r], 64 * rr + jj, 0), vj, acc[r][0]);
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++)
            y[r] = valid(r) ? (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]) : 0.0;
    }

    // y = A v over the first n rows, A = H's off-diagonal part with diagonal diag (QP4's f
    // and gradient use Q's diagonal); rows >= n give 0.
    MT_INLINE void amul(const double (&v)[R], const double (&diag)[R], double (&y)[R]) const
    {
        double acc[R][4];
        int kk[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;
            kk[r] = row(r) < n ? row(r) : 0;
        }
        const unsigned ldb = 8u * (unsigned)(ld - 1);
        MT_UNROLL for (int rr = 0; rr < R; rr++) {
            const int jend = n - 64 * rr < 64 ? n - 64 * rr : 64;
            int jj = 0;
            for (; jj + 4 <= jend; jj += 4) {
                double vj[4];
                MT_UNROLL for (int u = 0; u < 4; u++) vj[u] = bcast(v[rr], jj + u);
                MT_UNROLL for (int r = 0; r < R; r++) {
                    const double *blk = M + kk[r] + 64 * rr + jj;
                    MT_UNROLL for (int u = 0; u < 4; u++) {
                        const int j = 64 * rr + jj + u;
                        const double h = hrd(blk, ldb, kk[r], j, u);
                        acc[r][u] = fma(j == kk[r] ? diag[r] : h, vj[u], acc[r][u]);
                    }
                }
            }
            for (; jj < jend; jj++) {
                const double vj = bcast(v[rr], jj);
                MT_UNROLL for (int r = 0; r < R; r++) {
                    const int j = 64 * rr + jj;
                    const double h = hrd(M + kk[r] + j, ldb, kk[r], j, 0);
                    acc[r][0] = fma(j == kk[r] ? diag[r] : h, vj, acc[r][0]);
                }
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++)
            y[r] = valid(r) ? (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3]) : 0.0;
    }

    // component k (< n) of a row-distributed vector, the same in every lane
    MT_INLINE double comp(const double (&v)[R], int k) const
    {
        double t = v[0];
        MT_UNROLL for (int r = 1; r < R; r++) t = (k >> 6) == r ? v[r] : t;
        return bcast(t, k & 63);
    }

    MT_INLINE void load(const double *__restrict__ p, const double *__restrict__ lop,
                        const double *__restrict__ hip_, const double *__restrict__ x0p)
    {
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = row(r);
            const bool in = i < n;
            const int k = in ? i : 0;
            lo[r] = in ? lop[k] : 0.0;
            hi[r] = in ? hip_[k] : 0.0;
            x[r] = in ? x0p[k] : 0.0;
        }
        fam.load(*this, p);
    }

    MT_INLINE double fg(const double (&v)[R], double (&gr)[R]) const { return fam.fg(*this, v, gr); }

    MT_INLINE void hess() { fam.hess(*this); }

    MT_INLINE double pg_inf() const
    {
        double m = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) m = fmax(m, valid(r) ? fabs(pg_comp(x[r], lo[r], hi[r], g[r])) : 0.0);
        return uni(wave_max(m));
    }

    MT_INLINE double pg_nrm2() const
    {
        double s = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) {
            const double v = valid(r) ? pg_comp(x[r], lo[r], hi[r], g[r]) : 0.0;
            s = fma(v, v, s);
        }
        return sqrt(uni(wave_sum(s)));
    }

    // bit j of a row-distributed mask; a select chain rather than a runtime index, so the
    // mask stays in registers for every R
    MT_INLINE bool is_free(const uint64_t (&fm)[R], int j) const
    {
        uint64_t w = fm[0];
        MT_UNROLL for (int r = 1; r < R; r++) w = (j >> 6) == r ? fm[r] : w;
        return (w >> (j & 63)) & 1ull;
    }
    MT_INLINE bool own_free(const uint64_t (&fm)[R], int r) const { return (fm[r] >> lane) & 1ull; }

    // Cholesky factor of H_FF + alpha I with the identity outside F: the factor's strict lower
    // triangle into M's lower part, its pivots into column n, their reciprocals into dinv.
    // False when a pivot of a free column is not positive (the caller then raises alpha).
    MT_INLINE bool chol(const uint64_t (&fm)[R], double alpha)
    {
        return chol_panels(fm, alpha);
    }

    // Entry (k, j), k >= j, of H_FF + alpha I with the identity outside F, and 0 above the
    // diagonal and outside the first n rows and columns. k and j may differ between lanes.
    MT_INLINE double shifted(const uint64_t (&fm)[R], int k, int j, double alpha) const
    {
        const bool in = k < n && j < n && k >= j;
        // H_jk from the upper triangle; the address is clamped rather than branched on
        const double h = M[in ? (int)__umul24((unsigned)j, (unsigned)ld) + k : 0];
        const bool fj = is_free(fm, j);
        const double e = k == j ? (fj ? h + alpha : 1.0) : ((fj && is_free(fm, k)) ? h : 0.0);
        return in ? e : 0.0;
    }

    // Factor the 16 columns j0 .. j0 + 15 of S (left in the factor's slots, its diagonal in
    // column n), each lane holding its rows in registers, left-looking inside the panel and
    // pipelined by one column. The serial chain per column is kept to: the pivot lane's own
    // diagonal update, one readlane of the pivot, the reciprocal square root and the scale.
    // Beside it, the other rows subtract column c - 1 (its entry in row j0 + c read from the
    // pivot lane), and column c + 1 subtracts the panel's columns before c, reading row
    // j0 + c + 1 of the factor from LDS at one address in every lane (a broadcast read of
    // entries final since the last step). Each scaled entry goes straight to its slot in LDS
    // (one unconditional-path store per column, so the wait for the broadcast reads never
    // covers it); the pivots are stored once, after the panel.
    MT_INLINE bool panel_factor(const uint64_t (&fm)[R], int j0)
    {
        const int rp = j0 >> 6;  // register slot of the panel's rows
        double sv[R][16], pv[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = row(r);
            pv[r] = 1.0;
            MT_UNROLL for (int c = 0; c < 16; c++) {
                const int j = j0 + c;
                const bool in = i < n && i >= j;
                const double v = M[in ? (int)__umul24((unsigned)i, (unsigned)ld) + (i == j ? n : j) : 0];
                sv[r][c] = in ? v : 0.0;
            }
        }
        // A non-positive free pivot is remembered and reported once the panel is done. Column
        // c + 1 may lie past n (then it is prepared from row 0 and never used).
        bool bad = false;
        MT_UNROLL for (int c = 0; c < 16; c++) {
            const int j = j0 + c;
            if (j >= n) break;
            double pre[16];
            if (c + 1 < 16) {
                const int jn = j + 1 < n ? j + 1 : 0;
                const double *rn = M + __umul24((unsigned)jn, (unsigned)ld) + j0;
                MT_UNROLL for (int c1 = 0; c1 < c; c1++) pre[c1] = rn[c1];
            }
            double own = sv[0][c], prev = c > 0 ? sv[0][c - 1] : 0.0;
            MT_UNROLL for (int r = 1; r < R; r++) {
                own = rp == r ? sv[r][c] : own;
                prev = rp == r ? sv[r][c - (c > 0)] : prev;
            }
            if (c > 0) own = fma(-prev, prev, own);  // in the pivot lane: S_jj less L_j,j-1^2
            const double d = uni(bcast(own, j & 63));
            if (c > 0) {
                const double l = bcast(prev, j & 63);
                MT_UNROLL for (int r = 0; r < R; r++) sv[r][c] = fma(-sv[r][c - 1], l, sv[r][c]);
            }
            const bool fj = is_free(fm, j);
            bad = bad || (fj && !(d > 0.0));
            const double rinv = fj ? rsqrt_pos(fj ? d : 1.0) : 1.0;  // branch-free
            const double piv = fj ? d * rinv : 1.0;
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = row(r);
                sv[r][c] = (fj && own_free(fm, r)) ? sv[r][c] * rinv : 0.0;
                pv[r] = i == j ? piv : pv[r];
                dinv[r] = i == j ? rinv : dinv[r];
                if (i < n && i > j) M[__umul24((unsigned)i, (unsigned)ld) + j] = sv[r][c];
            }
            if (c + 1 < 16) {
                MT_UNROLL for (int r = 0; r < R; r++) {
                    double p0 = sv[r][c + 1], p1 = 0.0;
                    MT_UNROLL for (int c1 = 0; c1 < c; c1++) {
                        if (c1 & 1) p1 = fma(-sv[r][c1], pre[c1], p1);
                        else p0 = fma(-sv[r][c1], pre[c1], p0);
                    }
                    sv[r][c + 1] = p0 + p1;
                }
            }
            sync();
        }
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = row(r);
            if (i >= j0 && i < j0 + 16 && i < n) M[__umul24((unsigned)i, (unsigned)ld) + n] = pv[r];
        }
        sync();
        return !bad;
    }

    // The same panel step with M in global memory (4 or 8 rows per lane), in two passes that
    // keep 16 values per lane live instead of 16 per row slot. First the register slot that
    // holds the panel's rows, pipelined as above, with the panel's 16 x 16 block of L and its
    // pivot reciprocals mirrored in LDS (P, row stride 17, reciprocal in column 16) so that
    // its columns meet at wave scope; then every later slot by a triangular solve against
    // that block, its entries read from LDS at one address in every lane.
    MT_INLINE bool panel_factor_split(const uint64_t (&fm)[R], int j0)
    {
        const int rp = j0 >> 6;
        const int i = lane + 64 * rp;
        const bool ownf = i < n && is_free(fm, i);
        double sv[16], pv = 1.0, dv = 1.0;
        MT_UNROLL for (int c = 0; c < 16; c++) {
            const int j = j0 + c;
            const bool in = i < n && i >= j;
            const double v = M[in ? (int)__umul24((unsigned)i, (unsigned)ld) + (i == j ? n : j) : 0];
            sv[c] = in ? v : 0.0;
        }
        bool bad = false;
        MT_UNROLL for (int c = 0; c < 16; c++) {
            const int j = j0 + c;
            if (j >= n) break;
            double pre[16];
            if (c + 1 < 16) MT_UNROLL for (int c1 = 0; c1 < c; c1++) pre[c1] = P[(c + 1) * 17 + c1];
            double own = sv[c];
            if (c > 0) own = fma(-sv[c - 1], sv[c - 1], own);
            const double d = uni(bcast(own, j & 63));
            if (c > 0) {
                const double l = bcast(sv[c - 1], j & 63);
                sv[c] = fma(-sv[c - 1], l, sv[c]);
            }
            const bool fj = is_free(fm, j);
            bad = bad || (fj && !(d > 0.0));
            const double rinv = fj ? rsqrt_pos(fj ? d : 1.0) : 1.0;
            const double piv = fj ? d * rinv : 1.0;
            sv[c] = (fj && ownf) ? sv[c] * rinv : 0.0;
            pv = i == j ? piv : pv;
            dv = i == j ? rinv : dv;
            if (i < n && i > j) M[__umul24((unsigned)i, (unsigned)ld) + j] = sv[c];
            if (i > j && i < j0 + 16) P[(i - j0) * 17 + c] = sv[c];
            if (lane == 0) P[c * 17 + 16] = rinv;
            if (c + 1 < 16) {
                double p0 = sv[c + 1], p1 = 0.0;
                MT_UNROLL for (int c1 = 0; c1 < c; c1++) {
                    if (c1 & 1) p1 = fma(-sv[c1], pre[c1], p1);
                    else p0 = fma(-sv[c1], pre[c1], p0);
                }
                sv[c + 1] = p0 + p1;
            }
            lds_sync();
        }
        const bool inp = i >= j0 && i < j0 + 16 && i < n;
        if (inp) M[__umul24((unsigned)i, (unsigned)ld) + n] = pv;
        MT_UNROLL for (int r = 0; r < R; r++) dinv[r] = (r == rp && inp) ? dv : dinv[r];
        // rows of the later slots: L(i, j0 + c) = (S(i, j0 + c) - sum_{c1 < c} L(i, j0 + c1)
        // L(j0 + c, j0 + c1)) / L(j0 + c, j0 + c)
        for (int r2 = rp + 1; r2 < R && 64 * r2 < n; r2++) {
            const int i2 = lane + 64 * r2;
            const bool in2 = i2 < n;
            const bool f2 = in2 && is_free(fm, i2);
            const int base = (int)__umul24((unsigned)(in2 ? i2 : 0), (unsigned)ld) + j0;
            double t[16];
            MT_UNROLL for (int c = 0; c < 16; c++) {
                const double v = M[base + c];
                t[c] = in2 ? v : 0.0;
            }
            MT_UNROLL for (int c = 0; c < 16; c++) {
                if (j0 + c >= n) break;
                double p0 = t[c], p1 = 0.0;
                MT_UNROLL for (int c1 = 0; c1 < c; c1++) {
                    const double l = P[c * 17 + c1];
                    if (c1 & 1) p1 = fma(-t[c1], l, p1);
                    else p0 = fma(-t[c1], l, p0);
                }
                t[c] = (is_free(fm, j0 + c) && f2) ? (p0 + p1) * P[c * 17 + 16] : 0.0;
                if (in2) M[base + c] = t[c];
            }
        }
        sync();
        return !bad;
    }

    // Blocked left-looking factorisation in panels of 16 columns. For the panel starting at
    // column j0, the matrix cores form S = A[j0:n, panel] - L[j0:n, 0:j0] L[panel, 0:j0]^T,
    // 16 x 16 blocks by 16 x 16 x 4 FP64 products (operands read from LDS once, no
    // broadcasts); then each lane factors its rows of S in registers, column by column, with
    // the pivot and the panel's own factor entries broadcast by readlane. One wave barrier per
    // phase instead of one per column.
    // Lane layout of the 16 x 16 x 4 FP64 product: A(i, k) in lane i + 16 k, B(k, j) in lane
    // j + 16 k, C(i, j) in lane j + 16 (i mod 4), element i / 4 of the lane's four.
    MT_INLINE bool chol_panels(const uint64_t (&fm)[R], double alpha)
    {
        typedef double d4 __attribute__((ext_vector_type(4)));
        const int lr = lane & 15, lq = lane >> 4;
        for (int j0 = 0; j0 < n; j0 += 16) {
            const int jb = j0 + lr;  // this lane's panel column (B row, C column)
            const int jbk = jb < n ? jb : 0;
            for (int k0 = j0; k0 < n; k0 += 16) {
                const int ka = k0 + lr;  // this lane's A row
                const int kak = ka < n ? ka : 0;
                d4 acc0, acc1 = {0.0, 0.0, 0.0, 0.0};
                MT_UNROLL for (int v = 0; v < 4; v++) acc0[v] = shifted(fm, k0 + lq + 4 * v, jb, alpha);
                const double *ra = M + __umul24((unsigned)kak, (unsigned)ld) + lq;
                const double *rb = M + __umul24((unsigned)jbk, (unsigned)ld) + lq;
                // rows past n read row 0 (always present) and use 0
                const bool ain = ka < n, bin = jb < n;
                int q0 = 0;
                if constexpr (kGlobal) {
                    // operands from L2: eight chunks' loads in flight per round trip
                    for (; q0 + 32 <= j0; q0 += 32) {
                        double av[8], bv[8];
                        MT_UNROLL for (int u = 0; u < 8; u++) {
                            av[u] = ra[q0 + 4 * u];
                            bv[u] = rb[q0 + 4 * u];
                        }
                        MT_UNROLL for (int u = 0; u < 8; u += 2) {
                            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ain ? -av[u] : 0.0, bin ? bv[u] : 0.0, acc0, 0, 0, 0);
                            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ain ? -av[u + 1] : 0.0, bin ? bv[u + 1] : 0.0, acc1, 0, 0, 0);
                        }
                    }
                }
                for (; q0 + 8 <= j0; q0 += 8) {
                    const double a0 = ra[q0], b0 = rb[q0], a1 = ra[q0 + 4], b1 = rb[q0 + 4];
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ain ? -a0 : 0.0, bin ? b0 : 0.0, acc0, 0, 0, 0);
                    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ain ? -a1 : 0.0, bin ? b1 : 0.0, acc1, 0, 0, 0);
                }
                if (q0 < j0) {
                    const double a0 = ra[q0], b0 = rb[q0];
                    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ain ? -a0 : 0.0, bin ? b0 : 0.0, acc0, 0, 0, 0);
                }
                MT_UNROLL for (int v = 0; v < 4; v++) {
                    const int k = k0 + lq + 4 * v;
                    // S below the diagonal into the factor's slots, its diagonal into column n
                    if (k < n && jb < n && k >= jb)
                        M[__umul24((unsigned)k, (unsigned)ld) + (k == jb ? n : jb)] = acc0[v] + acc1[v];
                }
            }
            sync();
            if constexpr (kGlobal) {
                if (!panel_factor_split(fm, j0)) return false;
            } else {
                if (!panel_factor(fm, j0)) return false;
            }
        }
        return true;
    }

    // Returns the shift that succeeded, or -1 when the diagonal fallback was used.
    MT_INLINE double precond(const uint64_t (&fm)[R])
    {
        double mn = __builtin_inf(), mx = 0.0;
        MT_UNROLL for (int r = 0; r < R; r++) {
            if (valid(r) && own_free(fm, r)) {
                mn = hd[r] < mn ? hd[r] : mn;
                mx = fabs(hd[r]) > mx ? fabs(hd[r]) : mx;
            }
        }
        mn = -uni(wave_max(-mn));
        mx = uni(wave_max(mx));
        const double beta = 1e-3 * (mx > 1.0 ? mx : 1.0);
        double alpha = mn > 0.0 ? 0.0 : beta - mn;
        for (int t = 0; t < kShiftTries; t++) {
            if (chol(fm, alpha)) return alpha;
            alpha = 2.0 * alpha > beta ? 2.0 * alpha : beta;
        }
        for (int j = 0; j < n; j++) {
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = row(r);
                if (i < n && i > j) M[__umul24((unsigned)i, (unsigned)ld) + j] = 0.0;
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = row(r);
            if (i < n) {
                const double v = fabs(hd[r]);
                const double piv = own_free(fm, r) ? sqrt(v > beta ? v : beta) : 1.0;
                M[__umul24((unsigned)i, (unsigned)ld) + n] = piv;
                dinv[r] = 1.0 / piv;
            }
        }
        sync();
        return -1.0;
    }

    // component j of b * dinv, taken from its owner lane (wave-uniform result)
    MT_INLINE double owner_scaled(const double (&b)[R], int j) const
    {
        double v = b[0] * dinv[0];
        MT_UNROLL for (int r = 1; r < R; r++) v = (j >> 6) == r ? b[r] * dinv[r] : v;
        return bcast(v, j & 63);
    }

    // L y = b in place (b zero outside the factored set stays zero). Each row keeps its
    // residual unscaled while the substitution runs and is scaled by its reciprocal pivot once
    // at the end (the value its own step would have taken): the step's chain is then the
    // owner's scaling, the broadcast and one FMA, with no select on it. Rows not below the
    // step subtract an exact zero.
    MT_INLINE void fwd(double (&b)[R]) const
    {
        if constexpr (kGlobal) {
            // M in global memory: the lane's entries of L for kStage steps are loaded together
            // (one trip to L2 per kStage steps instead of one per step) and parked in the lane's
            // own LDS slots, which only it reads back
            for (int j0 = 0; j0 < n; j0 += kStage) {
                MT_UNROLL for (int t = 0; t < kStage; t++) {
                    MT_UNROLL for (int r = 0; r < R; r++) {
                        const int i = row(r);
                        const bool below = i > j0 + t && i < n && j0 + t < n;
                        const double v = M[below ? (int)__umul24((unsigned)i, (unsigned)ld) + j0 + t : 0];
                        Q[(t * R + r) * 64 + lane] = below ? v : 0.0;
                    }
                }
                MT_UNROLL for (int t = 0; t < kStage; t++) {
                    if (j0 + t >= n) break;
                    const double yj = owner_scaled(b, j0 + t);
                    MT_UNROLL for (int r = 0; r < R; r++) b[r] = fma(-Q[(t * R + r) * 64 + lane], yj, b[r]);
                }
            }
        } else {
            // the lane's row of L from column 0 (a row past n reads row 0, its update masked:
            // its index is taken as -1)
            const double *lr[R];
            int ii[R];
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = row(r);
                ii[r] = i < n ? i : -1;
                lr[r] = M + (int)__umul24((unsigned)(i < n ? i : 0), (unsigned)ld);
            }
            for (int j = 0; j < n; j++) {
                const double yj = owner_scaled(b, j);
                MT_UNROLL for (int r = 0; r < R; r++) {
                    const double l = lr[r][j];
                    b[r] = fma(-(j < ii[r] ? l : 0.0), yj, b[r]);
                }
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++) b[r] = valid(r) ? b[r] * dinv[r] : b[r];
    }

    // L^T y = b in place, the same way
    MT_INLINE void bwd(double (&b)[R]) const
    {
        if constexpr (kGlobal) {
            for (int j0 = ((n - 1) / kStage) * kStage; j0 >= 0; j0 -= kStage) {
                MT_UNROLL for (int t = 0; t < kStage; t++) {
                    MT_UNROLL for (int r = 0; r < R; r++) {
                        const int i = row(r);
                        const bool above = i < j0 + t && j0 + t < n;
                        const double v = M[above ? (int)__umul24((unsigned)(j0 + t), (unsigned)ld) + i : 0];
                        Q[(t * R + r) * 64 + lane] = above ? v : 0.0;
                    }
                }
                MT_UNROLL for (int t = kStage - 1; t >= 0; t--) {
                    if (j0 + t >= n) continue;
                    const double yj = owner_scaled(b, j0 + t);
                    MT_UNROLL for (int r = 0; r < R; r++) b[r] = fma(-Q[(t * R + r) * 64 + lane], yj, b[r]);
                }
            }
        } else {
            // the lane's column of L (entry j at j ld + i; a row past n reads column 0, and
            // is never above a step)
            const double *lc[R];
            MT_UNROLL for (int r = 0; r < R; r++) lc[r] = M + (row(r) < n ? row(r) : 0);
            const unsigned ldb = 8u * (unsigned)ld;
            for (int j = n - 1; j >= 0; j--) {
                const double yj = owner_scaled(b, j);
                MT_UNROLL for (int r = 0; r < R; r++) {
                    const double l = *(const double *)((const char *)lc[r] + (unsigned)j * ldb);
                    b[r] = fma(-(row(r) < j ? l : 0.0), yj, b[r]);
                }
            }
        }
        MT_UNROLL for (int r = 0; r < R; r++) b[r] = valid(r) ? b[r] * dinv[r] : b[r];
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
        double st[R], hs[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            xt[r] = clampf(fma(-a, g[r], x[r]), lo[r], hi[r]);
            st[r] = xt[r] - x[r];
        }
        if (!(dot(st, st) <= delta * delta)) return false;
        hmul(st, hs);
        double ss[R];
        MT_UNROLL for (int r = 0; r < R; r++) ss[r] = fma(0.5, hs[r], g[r]);
        const double gts = dot(g, st);
        const double q = dot(st, ss);  // g's + s'Hs/2
        return q <= kMu0 * gts;
    }

    MT_INLINE bool below_last_breakpoint(double a) const
    {
        bool any = false, below = false;
        MT_UNROLL for (int r = 0; r < R; r++) {
            const double d = -g[r];
            const bool up = valid(r) && d > 0.0 && isfinite(hi[r]);
            const bool dn = valid(r) && d < 0.0 && isfinite(lo[r]);
            any = any || up || dn;
            below = below || (up && a * d < hi[r] - x[r]) || (dn && a * d > lo[r] - x[r]);
        }
        const bool wany = __ballot(any) != 0ull, wbelow = __ballot(below) != 0ull;
        return !wany || wbelow;
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

    MT_INLINE void free_mask(const double (&v)[R], uint64_t (&fm)[R]) const
    {
        MT_UNROLL for (int r = 0; r < R; r++) fm[r] = __ballot(valid(r) && lo[r] < v[r] && v[r] < hi[r]);
    }

    // exact: no shift was needed, so the preconditioned matrix is the identity and the first
    // CG step, s_hat = r_hat cut at the radius, is the whole solve (see lane_tron.hpp)
    MT_INLINE int pcg(const uint64_t (&fm)[R], int m, const double (&rv)[R], double (&sh)[R],
                      double cg_rtol, bool exact)
    {
        double rh[R], p[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            rh[r] = own_free(fm, r) ? -rv[r] : 0.0;
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
            MT_UNROLL for (int r = 0; r < R; r++) q[r] = own_free(fm, r) ? q[r] : 0.0;
            fwd(q);
            const double kap_ = dot(p, q);
            if (!(kap_ > 0.0)) {
                const double sig = trqsol(sh, p);
                MT_UNROLL for (int r = 0; r < R; r++) sh[r] = fma(sig, p[r], sh[r]);
                return kCgNeg;
            }
            const double a = rr / kap_;
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
        has_l = false;
        for (int pass = 0; pass < n; pass++) {
            uint64_t fm[R];
            free_mask(xs, fm);
            int m = 0;
            MT_UNROLL for (int r = 0; r < R; r++) m += __builtin_popcountll(fm[r]);
            if (m == 0) break;
            double s[R], rv[R];
            MT_UNROLL for (int r = 0; r < R; r++) s[r] = xs[r] - x[r];
            hmul(s, rv);
            MT_UNROLL for (int r = 0; r < R; r++) rv[r] += g[r];
            const double shift = precond(fm);
            has_l = true;
            MT_UNROLL for (int r = 0; r < R; r++) lfm[r] = fm[r];
            double w[R];
            const int ex = pcg(fm, m, rv, w, cg_rtol, shift == 0.0);
            bwd(w);
            double beta = 1.0;
            bool acc = false;
            double xt[R];
            for (int t = 0; t <= kSearchHalvings; t++) {
                double d[R], hdv[R];
                MT_UNROLL for (int r = 0; r < R; r++) {
                    xt[r] = clampf(fma(beta, w[r], xs[r]), lo[r], hi[r]);
                    d[r] = xt[r] - xs[r];
                }
                hmul(d, hdv);
                double hh[R];
                MT_UNROLL for (int r = 0; r < R; r++) hh[r] = fma(0.5, hdv[r], rv[r]);
                const double rd = dot(rv, d);
                const double dq = dot(d, hh);  // r'd + d'Hd/2
                if (dq <= kMu0 * rd) { acc = true; break; }
                beta *= 0.5;
            }
            if (acc) MT_UNROLL for (int r = 0; r < R; r++) xs[r] = xt[r];
            uint64_t fm2[R];
            free_mask(xs, fm2);
            bool newly = false;
            MT_UNROLL for (int r = 0; r < R; r++) newly = newly || (fm[r] & ~fm2[r]) != 0ull;
            if (!((ex == kCgConv || ex == kCgMaxit) && newly)) break;
        }
    }

    MT_INLINE double step_norm(const double (&s)[R]) const
    {
        if (!has_l) return sqrt(dot(s, s));
        // t = L^T s: t_i = L_ii s_i + sum_{k > i} L_ki s_k (the pivot L_ii sits in column n), in
        // four independent partial sums, four broadcasts and loads at a time (entries of rows
        // not below i are read as exact zeros, no selects)
        double acc[R][4];
        MT_UNROLL for (int r = 0; r < R; r++) acc[r][0] = acc[r][1] = acc[r][2] = acc[r][3] = 0.0;
        int k = 0;
        for (; k + 4 <= n; k += 4) {
            double sk[4];
            MT_UNROLL for (int u = 0; u < 4; u++) sk[u] = comp(s, k + u);
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = row(r);
                MT_UNROLL for (int u = 0; u < 4; u++) {
                    const bool in = i < k + u;
                    const double l = M[in ? (int)__umul24((unsigned)(k + u), (unsigned)ld) + i : 0];
                    acc[r][u] = fma(in ? l : 0.0, sk[u], acc[r][u]);
                }
            }
        }
        for (; k < n; k++) {
            const double sk = comp(s, k);
            MT_UNROLL for (int r = 0; r < R; r++) {
                const int i = row(r);
                const bool in = i < k;
                const double l = M[in ? (int)__umul24((unsigned)k, (unsigned)ld) + i : 0];
                acc[r][0] = fma(in ? l : 0.0, sk, acc[r][0]);
            }
        }
        double t[R];
        MT_UNROLL for (int r = 0; r < R; r++) {
            const int i = row(r);
            const double piv = M[valid(r) ? (int)__umul24((unsigned)i, (unsigned)ld) + n : 0];
            t[r] = valid(r) ? fma(piv, s[r], (acc[r][0] + acc[r][1]) + (acc[r][2] + acc[r][3])) : 0.0;
        }
        return sqrt(dot(t, t));
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

    MT_INLINE int32_t solve(const Options &o, double delta_in, double alphac_in)
    {
        iters = 0;
        delta = 0.0;
        alphac = 1.0;
        f = __builtin_nan("");
        bool bad = false;
        MT_UNROLL for (int r = 0; r < R; r++) bad = bad || (valid(r) && !(lo[r] <= hi[r]));
        if (__ballot(bad) != 0ull) return kBadBounds;
        MT_UNROLL for (int r = 0; r < R; r++) x[r] = clampb(x[r], lo[r], hi[r]);
        sync();
        f = fg(x, g);
        bool fin = true;
        MT_UNROLL for (int r = 0; r < R; r++) fin = fin && isfinite(g[r]);
        fin = isfinite(f) && __ballot(!fin) == 0ull;
        if (!fin) return kNonfinite;
        if (pg_inf() <= o.gtol) return kConverged;
        if (o.warm && delta_in > 0.0) delta = delta_in;
        else if (o.delta0 > 0.0) delta = o.delta0;
        else {
            delta = pg_nrm2();
            if (delta == 0.0) delta = 1.0;
        }
        if (o.warm && alphac_in > 0.0) alphac = alphac_in;
        hess();
        int32_t status;
        for (;;) {
            cauchy();
            subspace(o.cg_rtol);
            double s[R], hs[R];
            MT_UNROLL for (int r = 0; r < R; r++) s[r] = xs[r] - x[r];
            const double snorm = step_norm(s);
            hmul(s, hs);
            double hh[R];
            MT_UNROLL for (int r = 0; r < R; r++) hh[r] = fma(0.5, hs[r], g[r]);
            const double gts = dot(g, s);
            const double pred = -dot(s, hh);
            iters++;
            if (!(pred > 0.0)) { status = kStalled; break; }
            double gt[R];
            const double ft = fg(xs, gt);
            const bool tfin = isfinite(ft);
            double ared = f - ft;
            if (tfin && pred <= kAredSwitch * (fabs(f) > 1.0 ? fabs(f) : 1.0)) {
                double sg[R];
                MT_UNROLL for (int r = 0; r < R; r++) sg[r] = g[r] + gt[r];
                ared = -0.5 * dot(sg, s);
            }
            const double rho = tfin ? ared / pred : -__builtin_inf();
            delta = radius_update(rho, ared, gts, snorm, tfin);
            const bool accept = rho > kEta0;
            if (accept) {
                MT_UNROLL for (int r = 0; r < R; r++) { x[r] = xs[r]; g[r] = gt[r]; }
                f = ft;
            }
            bool ok = true;
            MT_UNROLL for (int r = 0; r < R; r++) ok = ok && isfinite(g[r]);
            ok = isfinite(f) && __ballot(!ok) == 0ull;
            if (!ok) { status = kNonfinite; break; }
            if (pg_inf() <= o.gtol) { status = kConverged; break; }
            if (iters >= o.max_iter) { status = kMaxIter; break; }
            const double tiny = kStallRel * (fabs(f) > 1.0 ? fabs(f) : 1.0);
            if (tfin && fabs(ared) <= tiny && pred <= tiny) { status = kStalled; break; }
            if (accept) hess();
        }
        return status;
    }
};

}  // namespace mt
