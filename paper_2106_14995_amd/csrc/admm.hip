// admm.hip -- the component ADMM of the power-flow application (section 6.1) on the GPU.
//
// One iteration, in the order the paper gives (generators and branches, then buses, then
// multipliers), is two kernels on one stream:
//   branch     per branch (one lane each): its BR6 parameter block gathered from the state
//              into the workgroup's LDS, the batched branch solve warm-started in place
//              from the resident x, radius and Cauchy step length, then the branch
//              couplings y = (p_ij q_ij p_ji q_ji v_i^2 v_j^2 th_i th_j) at the new x;
//              one more workgroup reduces the previous iteration's residual parts
//   buses      per bus: weighted projection of the targets onto the two balance equations
//              (a 2 x 2 solve) giving new copies for its generators and branch ends, then
//              the multiplier steps of the couplings those copies belong to (each coupling
//              has its copy at exactly one bus), then the generator updates (closed form)
//              of the next iteration, whose inputs are all final at this point; per bus the
//              squared primal residuals and the squared changes of its copies
// The residual norms of an iteration sum the per-bus parts in a fixed order (deterministic);
// the last iteration of a call reduces them in a kernel of its own (reduce).
// The first iteration of each call updates the generators in a kernel of its own, so that
// the state between calls is the same as with the generator update at the top of every
// iteration. The state stays on the device in the flat layout of include/tron.h; the host
// only launches. The closed forms are the exact minimisers of the augmented Lagrangians of
// the generator and bus subproblems (the paper states only that they exist).
#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <vector>

#include "tron.h"
#include "tron_internal.hpp"

namespace {

struct Net {
    int32_t G, L, B, ref;
    double rho, base;
    const int32_t *br_from, *br_to, *gen_bus;
    const double *adm, *blo, *bhi, *cost, *glim, *load;
    const int32_t *bg_ptr, *bg_idx;   // generators of each bus (CSR, increasing index)
    const int32_t *be_ptr, *be_idx;   // branch ends of each bus (CSR, 2*l + side, increasing)
};

struct View {
    double *pg, *qg, *pgt, *qgt, *lpg, *lqg;
    double *x, *y, *yt, *lam, *mu, *del, *alp, *wt, *tht;
};

__host__ __device__ inline View split(double *s, int64_t G, int64_t L, int64_t B)
{
    View v;
    v.pg = s; v.qg = s + G; v.pgt = s + 2 * G; v.qgt = s + 3 * G; v.lpg = s + 4 * G; v.lqg = s + 5 * G;
    double *b = s + 6 * G;
    v.x = b; v.y = b + 6 * L; v.yt = b + 14 * L; v.lam = b + 18 * L; v.mu = b + 26 * L;
    v.del = b + 28 * L; v.alp = b + 29 * L; v.wt = b + 30 * L; v.tht = v.wt + B;
    (void)B;
    return v;
}

__device__ inline double clampd(double v, double lo, double hi) { return v < lo ? lo : (v > hi ? hi : v); }

// couplings of a branch at x (flows of eqs. pij..qji with w = v^2, wR = V cos, wI = V sin)
__device__ inline void couplings(const double *adm, const double *x, double *y)
{
    double s, c;
    sincos(x[2] - x[3], &s, &c);
    const double vi = x[0], vj = x[1], V = vi * vj;
    const double g0 = adm[0], b0 = adm[1], gc0 = adm[2], bc0 = adm[3];
    const double g1 = adm[4], b1 = adm[5], gc1 = adm[6], bc1 = adm[7];
    y[0] = gc0 * vi * vi + V * (b0 * s - g0 * c);
    y[1] = bc0 * vi * vi - V * (b0 * c + g0 * s);
    y[2] = gc1 * vj * vj - V * (g1 * c + b1 * s);
    y[3] = bc1 * vj * vj + V * (g1 * s - b1 * c);
    y[4] = vi * vi;
    y[5] = vj * vj;
    y[6] = x[2];
    y[7] = x[3];
}

// 64-lane workgroups: the ADMM kernels are a few thousand threads of scattered loads, and one
// wave per workgroup spreads them over four times as many CUs (and their load pipelines)
// as 256-lane workgroups would
constexpr int kBlock = 64;

__global__ __launch_bounds__(kBlock) void admm_init_kernel(Net n, double *s)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    View v = split(s, n.G, n.L, n.B);
    if (t < n.G) {
        const double *lim = n.glim + 4 * t;
        v.pg[t] = 0.5 * (lim[0] + lim[1]);
        v.qg[t] = 0.5 * (lim[2] + lim[3]);
        v.pgt[t] = v.pg[t];
        v.qgt[t] = v.qg[t];
        v.lpg[t] = 0.0;
        v.lqg[t] = 0.0;
    } else if (t < (int64_t)n.G + n.L) {
        const int64_t l = t - n.G;
        const double start[6] = {1.0, 1.0, 0.0, 0.0, 0.0, 0.0};
        double *x = v.x + 6 * l;
        for (int i = 0; i < 6; i++) x[i] = clampd(start[i], n.blo[6 * l + i], n.bhi[6 * l + i]);
        double y[8];
        couplings(n.adm + 8 * l, x, y);
        for (int k = 0; k < 8; k++) v.y[8 * l + k] = y[k];
        for (int k = 0; k < 4; k++) v.yt[4 * l + k] = y[k];
        for (int k = 0; k < 8; k++) v.lam[8 * l + k] = 0.0;
        v.mu[2 * l] = 0.0;
        v.mu[2 * l + 1] = 0.0;
        v.del[l] = 0.0;
        v.alp[l] = 0.0;
    } else if (t < (int64_t)n.G + n.L + n.B) {
        const int64_t b = t - n.G - n.L;
        v.wt[b] = 1.0;
        v.tht[b] = 0.0;
    }
}

// generator update (closed form) from its copies and multipliers
__device__ inline void gen_update(const Net &n, const View &v, int64_t t, double pgt, double qgt, double lpg,
                                  double lqg)
{
    const double rho = n.rho;
    const double c2 = n.base * n.base * n.cost[2 * t], c1 = n.base * n.cost[2 * t + 1];
    const double *lim = n.glim + 4 * t;
    const double p = (rho * pgt - lpg - c1) / (2.0 * c2 + rho);
    const double q = qgt - lqg / rho;
    v.pg[t] = clampd(p, lim[0], lim[1]);
    v.qg[t] = clampd(q, lim[2], lim[3]);
}

__global__ __launch_bounds__(kBlock) void gen_kernel(Net n, double *s)
{
    const int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (t >= n.G) return;
    const View v = split(s, n.G, n.L, n.B);
    gen_update(n, v, t, v.pgt[t], v.qgt[t], v.lpg[t], v.lqg[t]);
}

constexpr int kReduce = 1024;

// Residual norms from the parts: kReduce partial sums with fixed strides (sum over k = t,
// t + kReduce, ...) combined by a fixed halving tree, so the result is deterministic.
// reduce_kernel runs it with kReduce threads; reduce_parts64 with one 64-lane workgroup
// that takes the kReduce positions 64 at a time: the same additions in the same order.
__device__ void reduce_parts64(const double *part_primal, int64_t np, const double *part_dual, int64_t nd,
                               double rho, double *resid)
{
    __shared__ double sp[kReduce], sd[kReduce];
    const int t = threadIdx.x;
    for (int m = 0; m < kReduce / kBlock; m++) {
        const int tv = t + kBlock * m;
        double a = 0.0, b = 0.0;
        for (int64_t k = tv; k < np; k += kReduce) a += part_primal[k];
        for (int64_t k = tv; k < nd; k += kReduce) b += part_dual[k];
        sp[tv] = a;
        sd[tv] = b;
    }
    __syncthreads();
    for (int w = kReduce / 2; w > 0; w >>= 1) {
        for (int m = 0; m < kReduce / kBlock; m++) {
            const int tv = t + kBlock * m;
            if (tv < w) {
                sp[tv] += sp[tv + w];
                sd[tv] += sd[tv + w];
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        resid[0] = sqrt(sp[0]);
        resid[1] = rho * sqrt(sd[0]);
    }
}

// Branch l in the calling lane: its parameter block (in the order of include/tron.h: the
// admittances, the flow targets, the w and theta targets of both ends, the multipliers of
// the eight couplings and of the two flow copies, the penalty of each coupling) is formed
// from the previous copies and multipliers straight into the workgroup's LDS, where the BR6
// family keeps it; the solve is the batch API's BR6 lane solve, warm-started from the
// resident x, radius and Cauchy step length; the couplings at the new x follow.
// Outputs: x, radius and Cauchy step in the state, f, status and iterations per branch.
// With prev_resid, one workgroup past the branches' reduces the residual parts the previous
// iteration's bus kernel left (nothing writes them before this kernel ends).
__global__ __launch_bounds__(kBlock) void branch_kernel(Net n, double *s, mt::Options opt, double *fo,
                                                        int32_t *status, int32_t *iters,
                                                        const double *part_primal, const double *part_dual,
                                                        double *prev_resid)
{
    if (blockIdx.x == (n.L + kBlock - 1) / kBlock) {
        reduce_parts64(part_primal, n.B, part_dual, n.B, n.rho, prev_resid);
        return;
    }
    const int64_t l = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (l >= n.L) return;
    View v = split(s, n.G, n.L, n.B);
    const double rho = n.rho;
    const int i = n.br_from[l], j = n.br_to[l];
    double p[36];
    for (int k = 0; k < 8; k++) p[k] = n.adm[8 * l + k];
    for (int k = 0; k < 4; k++) p[8 + k] = v.yt[4 * l + k];
    p[12] = v.wt[i];
    p[13] = v.wt[j];
    p[14] = v.tht[i];
    p[15] = v.tht[j];
    for (int k = 0; k < 8; k++) p[16 + k] = v.lam[8 * l + k];
    p[24] = v.mu[2 * l];
    p[25] = v.mu[2 * l + 1];
    for (int k = 0; k < 10; k++) p[26 + k] = rho;
    mt::LaneTron<mt::BR6, 6> st;
    st.fam.load(p, 6);
    double *x = v.x + 6 * l;
    const double *lo = n.blo + 6 * l, *hi = n.bhi + 6 * l;
    MT_UNROLL for (int k = 0; k < 6; k++) {
        st.lo[k] = lo[k];
        st.hi[k] = hi[k];
        st.x[k] = x[k];
    }
    const int32_t rc = st.solve(opt, v.del[l], v.alp[l]);
    MT_UNROLL for (int k = 0; k < 6; k++) x[k] = st.x[k];
    fo[l] = st.f;
    status[l] = rc;
    iters[l] = st.iters;
    v.del[l] = st.delta;
    v.alp[l] = st.alphac;
    double y[8];
    couplings(n.adm + 8 * l, st.x, y);
    for (int k = 0; k < 8; k++) v.y[8 * l + k] = y[k];
}

// bus subproblem: minimise sum w_k/2 (yt_k - t_k)^2, t_k = y_k + lam_k / rho, over the bus
// copies (generator powers, branch-end flows, w shared by the ends, theta), subject to
// the two balance rows; yt = t - W^-1 A' (A W^-1 A')^-1 (A t - b)
// Then the multiplier steps of the couplings whose copies the bus holds (each coupling
// belongs to one bus: a generator's powers, a branch end's flows, w and theta, and the flow
// copy z of the end's p): lam += rho (y - yt), mu += rho (z - p); with gen_next, the
// generator update of the next iteration from the new copies and multipliers.
// Sixteen lanes per bus (one row of the wave's DPP rows): lane j takes the bus's generators
// and branch ends j, j + 16, ...; the sums over them are per-lane sums combined by a butterfly
// inside the row, which leaves the same bits in all sixteen lanes. The state was just written
// by kernels running on every XCD, so most loads miss this XCD's L2 and each round of
// dependent loads costs about a microsecond: a lane loads its first generator and first end
// in three rounds (the bus's CSR bounds; the neighbour indices; the neighbour values both
// passes use) and keeps them in registers; further ones (buses with more than sixteen) are
// read again in the second pass. Residual parts per bus: the squared primal residuals of its
// couplings and the squared changes of its copies.
constexpr int kBusLanes = 16;

template <int CTRL>
__device__ inline double dpp_row(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// sum over the 16 lanes of a DPP row, the same bits in each (every step adds two partners'
// values, commutatively): pairs, quads, half-rows, rows
__device__ inline double row_sum(double v)
{
    v += dpp_row<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp_row<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp_row<0x141>(v);  // row_half_mirror
    v += dpp_row<0x140>(v);  // row_mirror
    return v;
}

struct BusSums {
    double sgp = 0.0, sgq = 0.0, sep = 0.0, seq = 0.0, sw = 0.0, sth = 0.0;
};

struct BusSolve {
    double up, uq, wnew, tnew;
};

__device__ inline BusSolve bus_solve(const Net &n, int64_t b, const BusSums &t, int ng_, int ne_, const double *ld)
{
    const double rho = n.rho;
    const double ng = (double)ng_, deg = (double)ne_;
    const double pd = ld[0], qd = ld[1], gs = ld[2], bs = ld[3];
    const double tw = t.sw / deg, tth = t.sth / deg;
    const double ww = deg * rho;
    const double ep = t.sgp - t.sep - gs * tw - pd;
    const double eq = t.sgq - t.seq + bs * tw - qd;
    const double mpp = (ng + deg) / rho + gs * gs / ww;
    const double mqq = (ng + deg) / rho + bs * bs / ww;
    const double mpq = -gs * bs / ww;
    const double det = mpp * mqq - mpq * mpq;
    BusSolve r;
    r.up = (mqq * ep - mpq * eq) / det;
    r.uq = (mpp * eq - mpq * ep) / det;
    r.wnew = tw - (-gs * r.up + bs * r.uq) / ww;
    r.tnew = b == n.ref ? 0.0 : tth;
    return r;
}

// generator g of the bus after its new copies (np, nq): multipliers, primal residual part,
// and with gen_next its next update
__device__ inline void gen_duals(const Net &n, const View &v, int g, double pg, double qg, double lpg, double lqg,
                                 double np, double nq, int gen_next, double &p2)
{
    const double rho = n.rho;
    const double rp = pg - np, rq = qg - nq;
    const double lp = lpg + rho * rp, lq = lqg + rho * rq;
    v.lpg[g] = lp;
    v.lqg[g] = lq;
    p2 += rp * rp + rq * rq;
    if (gen_next) gen_update(n, v, g, np, nq, lp, lq);
}

// end e of branch l after the bus's new copies (np, nq, wnew, tnew): the multipliers of the
// end's four couplings (y: its p, q, w, theta; la: their multipliers), the flow copy's
// multiplier mu (z: the flow copy x[4 + e]), and the primal residual part
__device__ inline void end_duals(const Net &n, const View &v, int64_t l, int e, const double (&y)[4],
                                 const double (&la)[4], double z, double mu, double np, double nq, double wnew,
                                 double tnew, double &p2)
{
    const double rho = n.rho;
    const double r0 = y[0] - np, r1 = y[1] - nq, r2 = y[2] - wnew, r3 = y[3] - tnew;
    double *lam = v.lam + 8 * l;
    lam[2 * e] = la[0] + rho * r0;
    lam[2 * e + 1] = la[1] + rho * r1;
    lam[4 + e] = la[2] + rho * r2;
    lam[6 + e] = la[3] + rho * r3;
    v.mu[2 * l + e] = mu + rho * (z - y[0]);
    p2 += r0 * r0 + r1 * r1 + r2 * r2 + r3 * r3;
}

__global__ __launch_bounds__(kBlock) void bus_kernel(Net n, double *s, double *part_primal, double *part_dual,
                                                     int gen_next)
{
    const int64_t b = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kBusLanes;
    const int j = threadIdx.x & (kBusLanes - 1);
    // rows past the last bus compute on bus 0 and store nothing, so that every lane of a row
    // takes part in its sums
    const bool own = b < n.B;
    const int64_t bb = own ? b : 0;
    View v = split(s, n.G, n.L, n.B);
    const double rho = n.rho;
    const int g0 = n.bg_ptr[bb], g1 = n.bg_ptr[bb + 1];
    const int e0 = n.be_ptr[bb], e1 = n.be_ptr[bb + 1];
    double ld[4];
    MT_UNROLL for (int k = 0; k < 4; k++) ld[k] = n.load[4 * bb + k];
    const double wt0 = v.wt[bb], tht0 = v.tht[bb];
    const int ng = g1 - g0, ne = e1 - e0;
    // the lane's first generator and first branch end, kept in registers for both passes
    const bool hg = j < ng, he = j < ne;
    const int gi = hg ? n.bg_idx[g0 + j] : 0;
    const int code = he ? n.be_idx[e0 + j] : 0;
    const int64_t l = code >> 1;
    const int e = code & 1;
    double pg = 0.0, qg = 0.0, lpg = 0.0, lqg = 0.0, pgt = 0.0, qgt = 0.0;
    if (hg) {
        pg = v.pg[gi]; qg = v.qg[gi]; lpg = v.lpg[gi]; lqg = v.lqg[gi]; pgt = v.pgt[gi]; qgt = v.qgt[gi];
    }
    double ye[4] = {0.0, 0.0, 0.0, 0.0}, le[4] = {0.0, 0.0, 0.0, 0.0}, ot[2] = {0.0, 0.0}, z = 0.0, mu = 0.0;
    if (he) {
        const double *y = v.y + 8 * l, *la = v.lam + 8 * l, *yt = v.yt + 4 * l;
        ye[0] = y[2 * e]; ye[1] = y[2 * e + 1]; ye[2] = y[4 + e]; ye[3] = y[6 + e];
        le[0] = la[2 * e]; le[1] = la[2 * e + 1]; le[2] = la[4 + e]; le[3] = la[6 + e];
        ot[0] = yt[2 * e]; ot[1] = yt[2 * e + 1];
        z = v.x[6 * l + 4 + e]; mu = v.mu[2 * l + e];
    }
    BusSums t;
    if (hg) {
        t.sgp = pg + lpg / rho;
        t.sgq = qg + lqg / rho;
    }
    for (int k = g0 + j + kBusLanes; k < g1; k += kBusLanes) {
        const int g = n.bg_idx[k];
        t.sgp += v.pg[g] + v.lpg[g] / rho;
        t.sgq += v.qg[g] + v.lqg[g] / rho;
    }
    if (he) {
        t.sep = ye[0] + le[0] / rho;
        t.seq = ye[1] + le[1] / rho;
        t.sw = ye[2] + le[2] / rho;
        t.sth = ye[3] + le[3] / rho;
    }
    for (int k = e0 + j + kBusLanes; k < e1; k += kBusLanes) {
        const int c = n.be_idx[k];
        const int64_t lk = c >> 1;
        const int ek = c & 1;
        const double *y = v.y + 8 * lk, *la = v.lam + 8 * lk;
        t.sep += y[2 * ek] + la[2 * ek] / rho;
        t.seq += y[2 * ek + 1] + la[2 * ek + 1] / rho;
        t.sw += y[4 + ek] + la[4 + ek] / rho;
        t.sth += y[6 + ek] + la[6 + ek] / rho;
    }
    t.sgp = row_sum(t.sgp);
    t.sgq = row_sum(t.sgq);
    t.sep = row_sum(t.sep);
    t.seq = row_sum(t.seq);
    t.sw = row_sum(t.sw);
    t.sth = row_sum(t.sth);
    const BusSolve r = bus_solve(n, bb, t, ng, ne, ld);
    double d2 = 0.0, p2 = 0.0;
    if (hg && own) {
        const double np = pg + lpg / rho - r.up / rho;
        const double nq = qg + lqg / rho - r.uq / rho;
        d2 += (np - pgt) * (np - pgt) + (nq - qgt) * (nq - qgt);
        v.pgt[gi] = np;
        v.qgt[gi] = nq;
        gen_duals(n, v, gi, pg, qg, lpg, lqg, np, nq, gen_next, p2);
    }
    for (int k = g0 + j + kBusLanes; own && k < g1; k += kBusLanes) {
        const int g = n.bg_idx[k];
        const double pk = v.pg[g], qk = v.qg[g], lpk = v.lpg[g], lqk = v.lqg[g];
        const double np = pk + lpk / rho - r.up / rho;
        const double nq = qk + lqk / rho - r.uq / rho;
        d2 += (np - v.pgt[g]) * (np - v.pgt[g]) + (nq - v.qgt[g]) * (nq - v.qgt[g]);
        v.pgt[g] = np;
        v.qgt[g] = nq;
        gen_duals(n, v, g, pk, qk, lpk, lqk, np, nq, gen_next, p2);
    }
    const double dw = r.wnew - wt0, dt = r.tnew - tht0;
    if (he && own) {
        const double np = ye[0] + le[0] / rho + r.up / rho;
        const double nq = ye[1] + le[1] / rho + r.uq / rho;
        d2 += (np - ot[0]) * (np - ot[0]) + (nq - ot[1]) * (nq - ot[1]);
        d2 += dw * dw + dt * dt;
        double *yt = v.yt + 4 * l;
        yt[2 * e] = np;
        yt[2 * e + 1] = nq;
        end_duals(n, v, l, e, ye, le, z, mu, np, nq, r.wnew, r.tnew, p2);
    }
    for (int k = e0 + j + kBusLanes; own && k < e1; k += kBusLanes) {
        const int c = n.be_idx[k];
        const int64_t lk = c >> 1;
        const int ek = c & 1;
        const double *y = v.y + 8 * lk, *la = v.lam + 8 * lk;
        double *yt = v.yt + 4 * lk;
        const double yk[4] = {y[2 * ek], y[2 * ek + 1], y[4 + ek], y[6 + ek]};
        const double lk4[4] = {la[2 * ek], la[2 * ek + 1], la[4 + ek], la[6 + ek]};
        const double np = yk[0] + lk4[0] / rho + r.up / rho;
        const double nq = yk[1] + lk4[1] / rho + r.uq / rho;
        d2 += (np - yt[2 * ek]) * (np - yt[2 * ek]) + (nq - yt[2 * ek + 1]) * (nq - yt[2 * ek + 1]);
        d2 += dw * dw + dt * dt;
        yt[2 * ek] = np;
        yt[2 * ek + 1] = nq;
        end_duals(n, v, lk, ek, yk, lk4, v.x[6 * lk + 4 + ek], v.mu[2 * lk + ek], np, nq, r.wnew, r.tnew, p2);
    }
    d2 = row_sum(d2);
    p2 = row_sum(p2);
    if (own && j == 0) {
        v.wt[b] = r.wnew;
        v.tht[b] = r.tnew;
        part_primal[b] = p2;
        part_dual[b] = d2;
    }
}

// one workgroup of kReduce threads (see reduce_parts64)
__global__ __launch_bounds__(kReduce) void reduce_kernel(const double *part_primal, int64_t np,
                                                         const double *part_dual, int64_t nd,
                                                         double rho, double *resid)
{
    __shared__ double sp[kReduce], sd[kReduce];
    const int t = threadIdx.x;
    double a = 0.0, b = 0.0;
    for (int64_t k = t; k < np; k += kReduce) a += part_primal[k];
    for (int64_t k = t; k < nd; k += kReduce) b += part_dual[k];
    sp[t] = a;
    sd[t] = b;
    __syncthreads();
    for (int w = kReduce / 2; w > 0; w >>= 1) {
        if (t < w) {
            sp[t] += sp[t + w];
            sd[t] += sd[t + w];
        }
        __syncthreads();
    }
    if (t == 0 && resid) {
        resid[0] = sqrt(sp[0]);
        resid[1] = rho * sqrt(sd[0]);
    }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

struct admm {
    int device = 0;
    Net net{};
    tron_options opt{};
    int64_t state_size = 0;
    double *d_state = nullptr;
    double *d_f = nullptr, *d_part = nullptr;
    int32_t *d_status = nullptr, *d_iters = nullptr;
    std::vector<void *> owned;
};

static void free_admm(admm *a)
{
    if (!a) return;
    for (void *p : a->owned) (void)hipFree(p);
    delete a;
}

extern "C" int64_t admm_state_size(const admm_network *n)
{
    if (!n) return -1;
    return 6LL * n->ngen + 30LL * n->nbranch + 2LL * n->nbus;
}

template <class T>
static tron_err upload(admm *a, T **dst, const T *src, size_t count, hipStream_t st)
{
    *dst = nullptr;
    if (count == 0) return TRON_OK;
    if (hipMalloc((void **)dst, sizeof(T) * count) != hipSuccess)
        return mt_fail(TRON_ERR_NOMEM, "device allocation failed");
    a->owned.push_back(*dst);
    if (src) HIP_TRY(hipMemcpyAsync(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice, st));
    return TRON_OK;
}

extern "C" tron_err admm_create(admm **out, const admm_network *n, const tron_options *bopt,
                                void *stream)
{
    if (!out || !n) return mt_fail(TRON_ERR_INVALID, "null argument");
    *out = nullptr;
    if (n->nbus <= 0 || n->nbranch <= 0 || n->ngen < 0 || n->ref_bus < 0 || n->ref_bus >= n->nbus)
        return mt_fail(TRON_ERR_INVALID, "network sizes invalid");
    if (!n->br_from || !n->br_to || !n->br_adm || !n->br_lo || !n->br_hi || !n->bus_load ||
        (n->ngen > 0 && (!n->gen_bus || !n->gen_cost || !n->gen_lim)))
        return mt_fail(TRON_ERR_INVALID, "null network array");
    if (!(n->rho > 0.0)) return mt_fail(TRON_ERR_INVALID, "rho must be positive");
    const int G = n->ngen, L = n->nbranch, B = n->nbus;
    // adjacency in increasing index order
    std::vector<int32_t> gptr(B + 1, 0), eptr(B + 1, 0);
    for (int g = 0; g < G; g++) {
        if (n->gen_bus[g] < 0 || n->gen_bus[g] >= B) return mt_fail(TRON_ERR_INVALID, "generator bus out of range");
        gptr[n->gen_bus[g] + 1]++;
    }
    for (int l = 0; l < L; l++) {
        if (n->br_from[l] < 0 || n->br_from[l] >= B || n->br_to[l] < 0 || n->br_to[l] >= B ||
            n->br_from[l] == n->br_to[l])
            return mt_fail(TRON_ERR_INVALID, "branch %d ends invalid", l);
        eptr[n->br_from[l] + 1]++;
        eptr[n->br_to[l] + 1]++;
    }
    for (int b = 0; b < B; b++) {
        if (eptr[b + 1] == 0) return mt_fail(TRON_ERR_INVALID, "bus %d has no branch", b);
        gptr[b + 1] += gptr[b];
        eptr[b + 1] += eptr[b];
    }
    std::vector<int32_t> gidx(G), eidx(2 * (size_t)L), gfill(gptr.begin(), gptr.end() - 1),
        efill(eptr.begin(), eptr.end() - 1);
    for (int g = 0; g < G; g++) gidx[gfill[n->gen_bus[g]]++] = g;
    for (int l = 0; l < L; l++) {
        eidx[efill[n->br_from[l]]++] = 2 * l;
        eidx[efill[n->br_to[l]]++] = 2 * l + 1;
    }
    admm *a = new (std::nothrow) admm();
    if (!a) return mt_fail(TRON_ERR_NOMEM, "host allocation failed");
    (void)hipGetDevice(&a->device);
    tron_default_options(&a->opt);
    if (bopt) a->opt = *bopt;
    a->opt.flags |= TRON_FLAG_WARM;
    hipStream_t st = (hipStream_t)stream;
    Net &d = a->net;
    d.G = G; d.L = L; d.B = B; d.ref = n->ref_bus; d.rho = n->rho; d.base = n->base_mva;
    tron_err rc = TRON_OK;
    int32_t *p_from, *p_to, *p_gbus, *p_gptr, *p_gidx, *p_eptr, *p_eidx;
    double *p_adm, *p_lo, *p_hi, *p_cost, *p_lim, *p_load;
#define UP(dst, src, cnt) if ((rc = upload(a, &dst, src, cnt, st)) != TRON_OK) { free_admm(a); return rc; }
    UP(p_from, n->br_from, L);
    UP(p_to, n->br_to, L);
    UP(p_gbus, n->gen_bus, G);
    UP(p_adm, n->br_adm, 8 * (size_t)L);
    UP(p_lo, n->br_lo, 6 * (size_t)L);
    UP(p_hi, n->br_hi, 6 * (size_t)L);
    UP(p_cost, n->gen_cost, 2 * (size_t)G);
    UP(p_lim, n->gen_lim, 4 * (size_t)G);
    UP(p_load, n->bus_load, 4 * (size_t)B);
    UP(p_gptr, gptr.data(), B + 1);
    UP(p_gidx, gidx.data(), G);
    UP(p_eptr, eptr.data(), B + 1);
    UP(p_eidx, eidx.data(), 2 * (size_t)L);
    a->state_size = admm_state_size(n);
    UP(a->d_state, (const double *)nullptr, (size_t)a->state_size);
    UP(a->d_f, (const double *)nullptr, (size_t)L);
    UP(a->d_part, (const double *)nullptr, 2 * (size_t)B);
    UP(a->d_status, (const int32_t *)nullptr, (size_t)L);
    UP(a->d_iters, (const int32_t *)nullptr, (size_t)L);
#undef UP
    d.br_from = p_from; d.br_to = p_to; d.gen_bus = p_gbus; d.adm = p_adm; d.blo = p_lo;
    d.bhi = p_hi; d.cost = p_cost; d.glim = p_lim; d.load = p_load; d.bg_ptr = p_gptr;
    d.bg_idx = p_gidx; d.be_ptr = p_eptr; d.be_idx = p_eidx;
    hipLaunchKernelGGL(admm_init_kernel, dim3(grid_for((int64_t)G + L + B)), dim3(kBlock), 0, st, d, a->d_state);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) {
        free_admm(a);
        return mt_fail(TRON_ERR_DEVICE, "initialisation failed");
    }
    *out = a;
    return TRON_OK;
}

extern "C" tron_err admm_step(admm *a, int32_t iters, double *d_resid, void *stream)
{
    if (!a || iters < 0) return mt_fail(TRON_ERR_INVALID, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    const Net &n = a->net;
    mt::Options opt{};
    opt.gtol = a->opt.gtol;
    opt.cg_rtol = a->opt.cg_rtol;
    opt.delta0 = a->opt.delta0;
    opt.max_iter = a->opt.max_iter;
    opt.warm = 1;
    // branch lanes in 64-lane workgroups: a few thousand branches, one wave per workgroup,
    // spread over more CUs; each wave's parameter blocks take 36 x 64 doubles of LDS
    const size_t lds = sizeof(double) * mt::BR6::kLdsDoubles * kBlock;
    double *part_primal = a->d_part, *part_dual = a->d_part + n.B;
    for (int32_t it = 0; it < iters; it++) {
        if (it == 0 && n.G > 0)
            hipLaunchKernelGGL(gen_kernel, dim3(grid_for(n.G)), dim3(kBlock), 0, st, n, a->d_state);
        // the previous iteration's residuals are reduced by one more workgroup of this launch
        double *prev = (it > 0 && d_resid) ? d_resid + 2 * (int64_t)(it - 1) : nullptr;
        hipLaunchKernelGGL(branch_kernel, dim3(grid_for(n.L) + (prev ? 1u : 0u)), dim3(kBlock), lds, st, n,
                           a->d_state, opt, a->d_f, a->d_status, a->d_iters, (const double *)part_primal,
                           (const double *)part_dual, prev);
        hipLaunchKernelGGL(bus_kernel, dim3(grid_for((int64_t)n.B * kBusLanes)), dim3(kBlock), 0, st, n, a->d_state, part_primal,
                           part_dual, (int)(it + 1 < iters));
    }
    // the last iteration's residuals
    if (iters > 0 && d_resid)
        hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kReduce), 0, st, (const double *)part_primal,
                           (int64_t)n.B, (const double *)part_dual, (int64_t)n.B, n.rho,
                           d_resid + 2 * (int64_t)(iters - 1));
    HIP_TRY(hipGetLastError());
    return TRON_OK;
}

extern "C" tron_err admm_get_state(admm *a, double *d_buf, int64_t count, void *stream)
{
    if (!a || !d_buf || count != a->state_size) return mt_fail(TRON_ERR_INVALID, "bad argument");
    HIP_TRY(hipMemcpyAsync(d_buf, a->d_state, sizeof(double) * count, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return TRON_OK;
}

extern "C" tron_err admm_set_state(admm *a, const double *d_buf, int64_t count, void *stream)
{
    if (!a || !d_buf || count != a->state_size) return mt_fail(TRON_ERR_INVALID, "bad argument");
    HIP_TRY(hipMemcpyAsync(a->d_state, d_buf, sizeof(double) * count, hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return TRON_OK;
}

extern "C" tron_err admm_destroy(admm *a)
{
    free_admm(a);
    return TRON_OK;
}
