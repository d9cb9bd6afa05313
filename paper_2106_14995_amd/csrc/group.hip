// group.hip -- kernels of the group solver (group_tron.hpp): one instance per group of G
// consecutive lanes, 64 / G instances per wavefront.
#include <hip/hip_runtime.h>

#include "group_tron.hpp"
#include "tron_internal.hpp"

template <class Fam, int N, int G>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void group_kernel(LaneArgs a)
{
    const int64_t t = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / G;
    if (t >= a.count) return;  // whole groups leave together
    const int64_t b = a.index ? (int64_t)a.index[t] : t;
    const int n = a.nper ? a.nper[b] : a.n_uniform;
    const int64_t po = a.poff ? a.poff[b] : b * (int64_t)a.psize;
    const int64_t vo = a.voff ? a.voff[b] : b * (int64_t)n;
    const int64_t t0 = a.ts ? (int64_t)wall_clock64() : 0;
    using S = mt::GroupTron<Fam, N, G>;
    S s;
    s.n = n;
    s.set_lane((int)(threadIdx.x & (G - 1)));
    s.fam.load(s, a.params + po, n);
    const double *lo = a.lo + vo, *hi = a.hi + vo, *x0 = a.x0 + vo;
    MT_UNROLL for (int r = 0; r < S::R; r++) {
        const int i = s.row(r);
        const bool in = i < n;
        const int k = in ? i : 0;
        s.lo[r] = in ? lo[k] : Fam::pad;
        s.hi[r] = in ? hi[k] : Fam::pad;
        s.x[r] = in ? x0[k] : Fam::pad;
    }
    const double din = a.opt.warm ? a.state[b] : 0.0;
    const double ain = a.opt.warm ? a.state[a.batch + b] : 0.0;
    const int32_t st = s.solve(a.opt, din, ain);
    double *xo = a.x + vo;
    MT_UNROLL for (int r = 0; r < S::R; r++)
        if (s.row(r) < n) xo[s.row(r)] = s.x[r];
    if (s.k == 0) {
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
}

template <class Fam, int N, int G>
static void launch_group(const LaneArgs &a, hipStream_t st)
{
    const int blk = a.lane_block == 64 ? 64 : 256;
    const int64_t threads = a.count * G;
    const unsigned grid = (unsigned)((threads + blk - 1) / blk);
    if (grid) hipLaunchKernelGGL((group_kernel<Fam, N, G>), dim3(grid), dim3(blk), 0, st, a);
}

lane_launch_fn mt_group_launcher(tron_family fam, int N, int G)
{
    using namespace mt;
    if (fam == TRON_FAMILY_BR6 && N == 6) {
        if (G == 2) return launch_group<GBR6<2>, 6, 2>;
        if (G == 4) return launch_group<GBR6<4>, 6, 4>;
        if (G == 8) return launch_group<GBR6<8>, 6, 8>;
    }
    if (fam == TRON_FAMILY_QP4) {
        if (N == 8 && G == 2) return launch_group<GQP4<8, 2>, 8, 2>;
        if (N == 8 && G == 4) return launch_group<GQP4<8, 4>, 8, 4>;
        if (N == 8 && G == 8) return launch_group<GQP4<8, 8>, 8, 8>;
        if (N == 16 && G == 4) return launch_group<GQP4<16, 4>, 16, 4>;
        if (N == 16 && G == 8) return launch_group<GQP4<16, 8>, 16, 8>;
        if (N == 16 && G == 16) return launch_group<GQP4<16, 16>, 16, 16>;
    }
    if (fam == TRON_FAMILY_HS45M) {
        if (N == 8 && G == 2) return launch_group<GHS45M<8, 2>, 8, 2>;
        if (N == 8 && G == 4) return launch_group<GHS45M<8, 4>, 8, 4>;
        if (N == 8 && G == 8) return launch_group<GHS45M<8, 8>, 8, 8>;
        if (N == 16 && G == 8) return launch_group<GHS45M<16, 8>, 16, 8>;
        if (N == 16 && G == 16) return launch_group<GHS45M<16, 16>, 16, 16>;
    }
    return nullptr;
}
