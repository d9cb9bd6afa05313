// lane_kernels.hpp -- the lane-per-instance solve kernel (n <= 8): one instance per lane of
// 64- or 256-lane workgroups, the solver state in registers (lane_tron.hpp).
#pragma once

#include "lane_tron.hpp"
#include "tron_internal.hpp"

// The largest workgroup a plan selects (64 is the default). The launch bound caps the size
// the kernel accepts; with one wave per SIMD either way, the register budget is the same.
constexpr int kLaneBlock = 256;

// Solve instance b in the calling lane.
template <class F, int N>
__device__ __forceinline__ void lane_solve(const LaneArgs &a, int64_t b)
{
    const int n = a.nper ? a.nper[b] : a.n_uniform;
    const int64_t po = a.poff ? a.poff[b] : b * (int64_t)a.psize;
    const int64_t vo = a.voff ? a.voff[b] : b * (int64_t)n;
    const int64_t t0 = a.ts ? (int64_t)wall_clock64() : 0;
    mt::LaneTron<F, N> s;
    s.fam.load(a.params + po, n);
    const double *lo = a.lo + vo, *hi = a.hi + vo, *x0 = a.x0 + vo;
    MT_UNROLL for (int i = 0; i < N; i++) {
        const bool in = i < n;
        const int k = in ? i : 0;
        s.lo[i] = in ? lo[k] : F::pad;
        s.hi[i] = in ? hi[k] : F::pad;
        s.x[i] = in ? x0[k] : F::pad;
    }
    const double din = a.opt.warm ? a.state[b] : 0.0;
    const double ain = a.opt.warm ? a.state[a.batch + b] : 0.0;
    const int32_t st = s.solve(a.opt, din, ain);
    double *xo = a.x + vo;
    MT_UNROLL for (int i = 0; i < N; i++)
        if (i < n) xo[i] = s.x[i];
    a.f[b] = s.f;
    a.status[b] = st;
    a.iters[b] = s.iters;
    a.state[b] = s.delta;
    a.state[a.batch + b] = s.alphac;
    if (a.ts) {
        a.ts[2 * b] = t0;
        a.ts[2 * b + 1] = (int64_t)wall_clock64();
    }
}

template <class F, int N>
__global__ __launch_bounds__(kLaneBlock) void lane_kernel(LaneArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.count) return;
    lane_solve<F, N>(a, a.index ? (int64_t)a.index[t] : t);
}

template <class F, int N>
static void launch_lane(const LaneArgs &a, hipStream_t st)
{
    const int blk = a.lane_block == 64 ? 64 : kLaneBlock;
    const unsigned grid = (unsigned)((a.count + blk - 1) / blk);
    const size_t lds = sizeof(double) * (size_t)F::kLdsDoubles * (size_t)blk;
    if (grid) hipLaunchKernelGGL((lane_kernel<F, N>), dim3(grid), dim3(blk), lds, st, a);
}
