// tron_lib.hip -- kernels and C ABI of the MI355X batched TRON library (see include/tron.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lane_kernels.hpp"
#include "lane_tron.hpp"
#include "tron.h"
#include "tron_internal.hpp"
#include "wave_tron.hpp"

constexpr int kMaxSideStreams = 4;

// ------------------------------------------------------------------------------------
// error reporting
// ------------------------------------------------------------------------------------
static thread_local std::string g_err;

tron_err mt_fail(tron_err code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}


extern "C" const char *tron_last_error(void) { return g_err.c_str(); }

extern "C" void tron_default_options(tron_options *o)
{
    if (!o) return;
    o->gtol = 1e-6;
    o->max_iter = 500;
    o->flags = 0u;
    o->cg_rtol = 0.1;
    o->delta0 = 0.0;
}

extern "C" int64_t tron_param_size(tron_family fam, int32_t n)
{
    if (fam == TRON_FAMILY_QP4 && n >= 1 && n <= kMaxN) return (int64_t)n * (n + 1) / 2 + n + 1;
    if (fam == TRON_FAMILY_BR6 && n == 6) return 36;
    if (fam == TRON_FAMILY_HS45M && n >= 1 && n <= 128) return 0;
    if (fam == TRON_FAMILY_BR8L && n == 8) return 40;
    return -1;
}

// ------------------------------------------------------------------------------------
// lane-per-instance kernels (n <= 8)
// ------------------------------------------------------------------------------------
static lane_launch_fn lane_launcher(tron_family fam, int N)
{
    using namespace mt;
    if (fam == TRON_FAMILY_BR6) return N == 6 ? mt_launch_br6 : nullptr;
    if (fam == TRON_FAMILY_BR8L) return N == 8 ? launch_lane<BR8L, 8> : nullptr;
    if (fam == TRON_FAMILY_QP4) {
        switch (N) {
        case 1: return launch_lane<QP4<1>, 1>;
        case 2: return launch_lane<QP4<2>, 2>;
        case 3: return launch_lane<QP4<3>, 3>;
        case 4: return launch_lane<QP4<4>, 4>;
        case 5: return launch_lane<QP4<5>, 5>;
        case 6: return launch_lane<QP4<6>, 6>;
        case 7: return launch_lane<QP4<7>, 7>;
        case 8: return launch_lane<QP4<8>, 8>;
        }
    }
    if (fam == TRON_FAMILY_HS45M) {
        switch (N) {
        case 1: return launch_lane<HS45M<1>, 1>;
        case 2: return launch_lane<HS45M<2>, 2>;
        case 3: return launch_lane<HS45M<3>, 3>;
        case 4: return launch_lane<HS45M<4>, 4>;
        case 5: return launch_lane<HS45M<5>, 5>;
        case 6: return launch_lane<HS45M<6>, 6>;
        case 7: return launch_lane<HS45M<7>, 7>;
        case 8: return launch_lane<HS45M<8>, 8>;
        }
    }
    return nullptr;
}


// ------------------------------------------------------------------------------------
// augmented-Lagrangian loop for BR8L (section 1): each lane repeats the bound-constrained
// solve of its own instance and updates its multipliers and penalty in registers, so
// instances finish their outer loops independently and nothing returns to the host
// ------------------------------------------------------------------------------------
struct AlArgs {
    double *params;   // in/out: multipliers [37..38] and penalty [39] are updated
    int32_t *outer;
    double *viol;
    double ctol, rho_growth, decrease, rho_max;
    int32_t outer_max;
};

__global__ __launch_bounds__(kLaneBlock) void al_kernel(LaneArgs a, AlArgs al)
{
    constexpr int N = 8;
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.count) return;
    mt::LaneTron<mt::BR8L, N> s;
    double *prm = al.params + 40 * b;
    s.fam.load(prm, N);
    const double *lo = a.lo + N * b, *hi = a.hi + N * b, *x0 = a.x0 + N * b;
    MT_UNROLL for (int i = 0; i < N; i++) {
        s.lo[i] = lo[i];
        s.hi[i] = hi[i];
        s.x[i] = x0[i];
    }
    mt::Options o = a.opt;
    double din = o.warm ? a.state[b] : 0.0;
    double ain = o.warm ? a.state[a.batch + b] : 0.0;
    int32_t status = mt::kAlMaxOuter, total = 0, k = 0;
    double v = __builtin_inf(), vprev = __builtin_inf();
    while (k < al.outer_max) {
        const int32_t st = s.solve(o, din, ain);
        total += s.iters;
        k++;
        o.warm = 1;
        din = s.delta;
        ain = s.alphac;
        if (st != mt::kConverged) { status = st; break; }
        double hv[2];
        s.fam.limits(s.x, hv);
        v = fabs(hv[0]) > fabs(hv[1]) ? fabs(hv[0]) : fabs(hv[1]);
        if (!(v == v)) { status = mt::kNonfinite; break; }
        if (v <= al.ctol) { status = mt::kConverged; break; }
        s.fam.lam[0] += s.fam.rhoh * hv[0];
        s.fam.lam[1] += s.fam.rhoh * hv[1];
        if (v > al.decrease * vprev) s.fam.rhoh = mt::dmin(s.fam.rhoh * al.rho_growth, al.rho_max);
        vprev = v;
    }
    double *xo = a.x + N * b;
    MT_UNROLL for (int i = 0; i < N; i++) xo[i] = s.x[i];
    a.f[b] = s.f;
    a.status[b] = status;
    a.iters[b] = total;
    a.state[b] = s.delta;
    a.state[a.batch + b] = s.alphac;
    al.outer[b] = k;
    al.viol[b] = v;
    prm[37] = s.fam.lam[0];
    prm[38] = s.fam.lam[1];
    prm[39] = s.fam.rhoh;
}

// ------------------------------------------------------------------------------------
// wavefront-per-instance kernels (8 < n <= 128; QP4 and HS45M); one 64-lane workgroup per
// instance, so the hardware dispatcher hands the next instance to whichever CU frees up first
// ------------------------------------------------------------------------------------
// Solve instance b on one wavefront with its matrix array at M (scr: the LDS scratch of the
// global-memory form, unused otherwise).
template <class Fam, bool kGlobal>
__device__ __forceinline__ void wave_solve(const LaneArgs &a, int64_t b, double *M, double *scr)
{
    const int n = a.nper ? a.nper[b] : a.n_uniform;
    const int64_t po = a.poff ? a.poff[b] : b * (int64_t)a.psize;
    const int64_t vo = a.voff ? a.voff[b] : b * (int64_t)n;
    const int64_t t0 = a.ts ? (int64_t)wall_clock64() : 0;
    constexpr int R = Fam::R;
    const int lane = threadIdx.x & 63;
    mt::WaveTron<Fam, kGlobal> s;
    s.n = n;
    s.ld = (n + 1) | 1;  // odd and > n: column n holds the factor's pivots
    s.lane = lane;
    s.M = M;
    s.P = kGlobal ? scr : nullptr;
    s.Q = kGlobal ? scr + 16 * 17 : nullptr;
    s.load(a.params + po, a.lo + vo, a.hi + vo, a.x0 + vo);
    const double din = a.opt.warm ? a.state[b] : 0.0;
    const double ain = a.opt.warm ? a.state[a.batch + b] : 0.0;
    const int32_t st = s.solve(a.opt, din, ain);
    double *xo = a.x + vo;
    MT_UNROLL for (int r = 0; r < R; r++)
        if (s.valid(r)) xo[s.row(r)] = s.x[r];
    if (lane == 0) {
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

template <class Fam, bool kGlobal>
__device__ __forceinline__ void wave_body(const LaneArgs &a)
{
    extern __shared__ double smem[];
    const int64_t t = blockIdx.x;
    if (t >= a.count) return;
    const int64_t b = a.index ? (int64_t)a.index[t] : t;
    wave_solve<Fam, kGlobal>(a, b, kGlobal ? a.ws + t * a.ws_stride : smem, smem);
}

// Two builds of the same solver. Buckets of small n fit many instances per CU, so their
// kernel is held to three waves per SIMD's worth of registers. From n_max = kWaveBigN on,
// the LDS request already limits residency to about two waves per SIMD, so that build gets
// the registers it asks for.
constexpr int kWaveBigN = 48;

template <class Fam>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) void wave_kernel(LaneArgs a) { wave_body<Fam, false>(a); }

// n_max <= kWaveTinyN: the LDS request (8.4 KB at 32) allows four or more instances per SIMD,
// so this variant is held to four waves' worth of registers
constexpr int kWaveTinyN = 32;
template <class Fam>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void wave_kernel_tiny(LaneArgs a)
{
    wave_body<Fam, false>(a);
}

template <class Fam>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void wave_kernel_big(LaneArgs a)
{
    wave_body<Fam, false>(a);
}

// n > kLdsMaxN: the matrix array is the instance's slot of a global-memory workspace; the
// LDS holds one 16 x 16 block of the factor while its panel is factored
constexpr size_t kPanelScratchBytes = sizeof(double) * 16 * 17;
// and the substitutions park kStage steps of each lane's entries of L there (R rows each)
template <class Fam>
constexpr size_t global_lds_bytes()
{
    return kPanelScratchBytes + sizeof(double) * mt::WaveTron<Fam, true>::kStage * Fam::R * 64;
}

template <class Fam>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1, 2))) void wave_kernel_global(LaneArgs a)
{
    wave_body<Fam, true>(a);
}

static size_t wave_lds_bytes(int nmax) { return sizeof(double) * (size_t)nmax * (size_t)((nmax + 1) | 1); }

template <class Fam>
static void launch_wave(const LaneArgs &a, int nmax, hipStream_t st)
{
    if (a.count <= 0) return;
    const size_t lds = wave_lds_bytes(nmax);
    // two rows per lane means n_max > 64: always the low-occupancy build (the other is never
    // instantiated for it)
    if constexpr (Fam::R > 1) {
        hipLaunchKernelGGL((wave_kernel_big<Fam>), dim3((unsigned)a.count), dim3(64), lds, st, a);
    } else {
        if (nmax >= kWaveBigN)
            hipLaunchKernelGGL((wave_kernel_big<Fam>), dim3((unsigned)a.count), dim3(64), lds, st, a);
        else if (nmax > kWaveTinyN)
            hipLaunchKernelGGL((wave_kernel<Fam>), dim3((unsigned)a.count), dim3(64), lds, st, a);
        else
            hipLaunchKernelGGL((wave_kernel_tiny<Fam>), dim3((unsigned)a.count), dim3(64), lds, st, a);
    }
}

template <class Fam>
static void launch_wave_global(const LaneArgs &a, hipStream_t st)
{
    if (a.count <= 0) return;
    hipLaunchKernelGGL((wave_kernel_global<Fam>), dim3((unsigned)a.count), dim3(64), global_lds_bytes<Fam>(), st, a);
}

// the wave kernel of the family for instances with n <= nmax
static void launch_wave_fam(tron_family fam, const LaneArgs &a, int nmax, hipStream_t st)
{
    using namespace mt;
    if (a.ws && nmax <= kLdsMaxN && fam == TRON_FAMILY_QP4) {
        // the workspace form below the LDS limit (the plan's wave_global)
        if (nmax <= 64) launch_wave_global<WaveFamQP4<1>>(a, st);
        else launch_wave_global<WaveFamQP4<2>>(a, st);
        return;
    }
    if (fam == TRON_FAMILY_HS45M) {
        if (nmax <= 64) launch_wave<WaveFamHS45M<1>>(a, nmax, st);
        else launch_wave<WaveFamHS45M<2>>(a, nmax, st);
    } else {
        if (nmax <= 64) launch_wave<WaveFamQP4<1>>(a, nmax, st);
        else if (nmax <= kLdsMaxN) launch_wave<WaveFamQP4<2>>(a, nmax, st);
        else if (nmax <= 256) launch_wave_global<WaveFamQP4<4>>(a, st);
        else launch_wave_global<WaveFamQP4<8>>(a, st);
    }
}

static bool has_wave_kernel(tron_family fam) { return fam == TRON_FAMILY_QP4 || fam == TRON_FAMILY_HS45M; }

// ------------------------------------------------------------------------------------
// persistent size-bucketed launch: one launch for every wavefront instance of a mixed batch
// ------------------------------------------------------------------------------------
// A workgroup of kWaves wavefronts owns one CU's LDS as a pool of kPoolPage-byte pages. Each
// wave loops on its own: claim the next instance of the batch's list (the largest
// instances first, each followed by small ones to fill the waves beside it; see
// build_pool_plan), reserve the instance's matrix array (n ((n+1)|1) doubles) in the pool,
// solve it, release the pages.
// Instances of every size thus run side by side on every CU, packed by their actual LDS
// need, with no bucket waiting for a stream or a hardware queue.
constexpr int kPoolPage = 512;
constexpr int kPoolMaxPages = 320;  // 160 KB
constexpr int kPoolWords = kPoolMaxPages / 32;

struct PoolArgs {
    int32_t *counter;  // next list position to claim (set to 0 before each launch)
    int32_t pages;     // pool pages (the launch's dynamic LDS is pages x kPoolPage bytes)
};

struct PoolCtl {
    int lock;                    // held while a wave searches the page map
    uint32_t used[kPoolWords];   // page map; bits set and cleared by atomics
};

MT_INLINE uint32_t page_bits(int w, int first, int count)
{
    const int a0 = first > 32 * w ? first : 32 * w;
    const int a1 = first + count < 32 * w + 32 ? first + count : 32 * w + 32;
    if (a0 >= a1) return 0u;
    const int len = a1 - a0;
    return (len == 32 ? 0xFFFFFFFFu : ((1u << len) - 1u)) << (a0 - 32 * w);
}

// Reserve `need` consecutive free pages of the pool (wave-uniform result): lane 0 takes the
// lock, every lane tests the starts lane, lane + 64, ... against a snapshot of the map, the
// lowest start that fits is taken. Frees only clear bits, so a snapshot never offers a page
// that is in use. When nothing fits, the wave sleeps and retries: pages are only held by
// waves that are solving, and every solve ends.
MT_INLINE int pool_alloc(PoolCtl &ctl, int total, int need, int lane)
{
    for (;;) {
        int got = 0;
        if (lane == 0) got = atomicCAS(&ctl.lock, 0, 1) == 0;
        got = __builtin_amdgcn_readfirstlane(got);
        if (got) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            uint32_t u[kPoolWords];
            MT_UNROLL for (int w = 0; w < kPoolWords; w++) u[w] = __atomic_load_n(&ctl.used[w], __ATOMIC_RELAXED);
            int start = -1;
            for (int p0 = 0; p0 < total; p0 += 64) {
                const int p = p0 + lane;
                bool ok = p + need <= total;
                MT_UNROLL for (int w = 0; w < kPoolWords; w++) ok = ok && (u[w] & page_bits(w, p, need)) == 0u;
                const uint64_t bal = __ballot(ok);
                if (bal) {
                    start = p0 + (int)__builtin_ctzll(bal);
                    break;
                }
            }
            start = __builtin_amdgcn_readfirstlane(start);
            if (start >= 0 && lane == 0)
                MT_UNROLL for (int w = 0; w < kPoolWords; w++) {
                    const uint32_t m = page_bits(w, start, need);
                    if (m) atomicOr(&ctl.used[w], m);
                }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            if (lane == 0) atomicExch(&ctl.lock, 0);
            if (start >= 0) return start;
        }
        __builtin_amdgcn_s_sleep(4);
    }
}

MT_INLINE void pool_free(PoolCtl &ctl, int first, int need, int lane)
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");  // the solve's LDS accesses are done
    if (lane == 0)
        MT_UNROLL for (int w = 0; w < kPoolWords; w++) {
            const uint32_t m = page_bits(w, first, need);
            if (m) atomicAnd(&ctl.used[w], ~m);
        }
}

// Fam1: the one-row-per-lane solver (n <= 64); Fam2: two rows per lane (n <= 128), or Fam1
// again when the batch has no such instance.
template <class Fam1, class Fam2, int kWaves>
__global__ __launch_bounds__(64 * kWaves) void pool_kernel(LaneArgs a, PoolArgs p)
{
    extern __shared__ double smem[];
    __shared__ PoolCtl ctl;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x == 0) {
        ctl.lock = 0;
        for (int w = 0; w < kPoolWords; w++) ctl.used[w] = 0u;
    }
    __syncthreads();
    for (;;) {
        int item = 0;
        if (lane == 0) item = atomicAdd(p.counter, 1);
        item = __builtin_amdgcn_readfirstlane(item);
        if (item >= a.count) break;
        const int64_t b = a.index[item];
        const int n = a.nper ? a.nper[b] : a.n_uniform;
        const int need = (int)((mt_wave_matrix_doubles(n) * (int64_t)sizeof(double) + kPoolPage - 1) / kPoolPage);
        const int first = pool_alloc(ctl, p.pages, need, lane);
        double *M = smem + (size_t)first * (kPoolPage / sizeof(double));
        if (Fam2::R > 1 && n > 64) wave_solve<Fam2, false>(a, b, M, nullptr);
        else wave_solve<Fam1, false>(a, b, M, nullptr);
        pool_free(ctl, first, need, lane);
    }
}

__global__ void pool_reset_kernel(int32_t *counter) { *counter = 0; }

// The persistent launch: one workgroup per CU (the pool takes the CU's LDS), kWaves waves
// each. `pages` pool pages; nmax the batch's largest wave instance.
template <template <int> class FamT, int kWaves>
static void launch_pool_t(const LaneArgs &a, const PoolArgs &p, int nmax, int cus, hipStream_t st)
{
    const size_t lds = (size_t)p.pages * kPoolPage;
    if (nmax > 64)
        hipLaunchKernelGGL((pool_kernel<FamT<1>, FamT<2>, kWaves>), dim3(cus), dim3(64 * kWaves), lds, st, a, p);
    else
        hipLaunchKernelGGL((pool_kernel<FamT<1>, FamT<1>, kWaves>), dim3(cus), dim3(64 * kWaves), lds, st, a, p);
}

static void launch_pool(tron_family fam, const LaneArgs &a, const PoolArgs &p, int nmax, int waves, int cus,
                        hipStream_t st)
{
    using namespace mt;
    if (a.count <= 0) return;
    hipLaunchKernelGGL(pool_reset_kernel, dim3(1), dim3(1), 0, st, p.counter);
    if (fam == TRON_FAMILY_HS45M) {
        if (waves == 12) launch_pool_t<WaveFamHS45M, 12>(a, p, nmax, cus, st);
        else launch_pool_t<WaveFamHS45M, 8>(a, p, nmax, cus, st);
    } else {
        if (waves == 12) launch_pool_t<WaveFamQP4, 12>(a, p, nmax, cus, st);
        else launch_pool_t<WaveFamQP4, 8>(a, p, nmax, cus, st);
    }
}

// The pool kernels may take the whole LDS of a CU (once per process and device).
static void prepare_pool_kernels(int bytes)
{
    using namespace mt;
    const void *k[] = {(const void *)pool_kernel<WaveFamQP4<1>, WaveFamQP4<1>, 8>,
                       (const void *)pool_kernel<WaveFamQP4<1>, WaveFamQP4<2>, 8>,
                       (const void *)pool_kernel<WaveFamQP4<1>, WaveFamQP4<1>, 12>,
                       (const void *)pool_kernel<WaveFamQP4<1>, WaveFamQP4<2>, 12>,
                       (const void *)pool_kernel<WaveFamHS45M<1>, WaveFamHS45M<1>, 8>,
                       (const void *)pool_kernel<WaveFamHS45M<1>, WaveFamHS45M<2>, 8>,
                       (const void *)pool_kernel<WaveFamHS45M<1>, WaveFamHS45M<1>, 12>,
                       (const void *)pool_kernel<WaveFamHS45M<1>, WaveFamHS45M<2>, 12>};
    for (const void *f : k) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
}

// Lane packs: the instances with n <= 8 in packs of 64 of one size (a wave each; -1 pads a
// pack), every size in one launch. pack_n[k] is the size of pack k.
template <template <int> class FamT>
__global__ __launch_bounds__(64) void lane_pack_kernel(LaneArgs a, const int32_t *pack_n)
{
    const int64_t t = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const int32_t b = a.index[t];
    if (b < 0) return;
    switch (pack_n[blockIdx.x]) {
    case 1: lane_solve<FamT<1>, 1>(a, b); break;
    case 2: lane_solve<FamT<2>, 2>(a, b); break;
    case 3: lane_solve<FamT<3>, 3>(a, b); break;
    case 4: lane_solve<FamT<4>, 4>(a, b); break;
    case 5: lane_solve<FamT<5>, 5>(a, b); break;
    case 6: lane_solve<FamT<6>, 6>(a, b); break;
    case 7: lane_solve<FamT<7>, 7>(a, b); break;
    default: lane_solve<FamT<8>, 8>(a, b); break;
    }
}

static void launch_lane_packs(tron_family fam, const LaneArgs &a, const int32_t *pack_n, int64_t packs,
                              hipStream_t st)
{
    using namespace mt;
    if (packs <= 0) return;
    if (fam == TRON_FAMILY_HS45M)
        hipLaunchKernelGGL(lane_pack_kernel<HS45M>, dim3((unsigned)packs), dim3(64), 0, st, a, pack_n);
    else
        hipLaunchKernelGGL(lane_pack_kernel<QP4>, dim3((unsigned)packs), dim3(64), 0, st, a, pack_n);
}

// ------------------------------------------------------------------------------------
// batch handle
// ------------------------------------------------------------------------------------
struct Bucket {
    int32_t nmax;      // largest n the bucket's kernel holds
    int32_t lanes;     // lanes per instance (1: lane kernel, 64: wave kernel)
    int64_t count;     // instances in the bucket
    int32_t *d_index;  // instance list (null when the bucket is the whole batch in order)
    lane_launch_fn lane;
    double *d_ws;      // nmax > kLdsMaxN: count slots of mt_wave_matrix_doubles(nmax) doubles
};

// sizes above the LDS limit go to a global-memory bucket of 256 or kMaxN
static int global_edge(int n) { return n <= 256 ? 256 : kMaxN; }

lane_launch_fn mt_lane_launcher(tron_family fam, int N) { return lane_launcher(fam, N); }
void mt_launch_wave(tron_family fam, const LaneArgs &a, int nmax, hipStream_t st)
{
    launch_wave_fam(fam, a, nmax, st);
}
size_t mt_wave_lds_bytes(int nmax) { return wave_lds_bytes(nmax); }
void mt_prepare_wave_kernels()
{
    using namespace mt;
    const int big = (int)wave_lds_bytes(128), small = (int)wave_lds_bytes(64);
    const void *k64[] = {(const void *)wave_kernel<WaveFamQP4<1>>, (const void *)wave_kernel_big<WaveFamQP4<1>>,
                         (const void *)wave_kernel<WaveFamHS45M<1>>, (const void *)wave_kernel_big<WaveFamHS45M<1>>,
                         (const void *)wave_kernel_tiny<WaveFamQP4<1>>, (const void *)wave_kernel_tiny<WaveFamHS45M<1>>};
    const void *k128[] = {(const void *)wave_kernel_big<WaveFamQP4<2>>, (const void *)wave_kernel_big<WaveFamHS45M<2>>};
    for (const void *k : k64) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, small);
    for (const void *k : k128) (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    mt_prepare_br6();
}

static void launch_bucket(tron_family fam, const Bucket &b, const LaneArgs &a0, hipStream_t st)
{
    if (b.lanes < 64) {
        b.lane(a0, st);
        return;
    }
    LaneArgs a = a0;
    a.ws = b.d_ws;
    a.ws_stride = b.d_ws ? mt_wave_matrix_doubles(b.nmax) : 0;
    launch_wave_fam(fam, a, b.nmax, st);
}

// The default plan: the autotuner's usual choice on large uneven batches. Edges every 8 up to
// 64 keep each bucket's LDS request (n_max ((n_max+1)|1) x 8 B) close to what its instances
// need, so smaller instances are not held to the residency of the largest; 64-lane
// workgroups spread the lane kernels' few thousand lanes over more CUs.
static void default_spec(tron_plan_spec *p)
{
    constexpr int kN = 11;
    const int e[kN] = {16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128};
    p->lane_max_n = 8;
    p->nedges = kN;
    for (int i = 0; i < 16; i++) p->edges[i] = i < kN ? e[i] : 0;
    p->streams = kMaxSideStreams;
    p->lane_block = 64;
    p->pool_waves = 12;  // mixed batches: the persistent launch (uniform batches use buckets)
    p->lane_group = 0;
    p->group16 = 0;
    p->wave_global = 0;
}

static tron_err check_spec(const tron_plan_spec &p)
{
    if (p.lane_max_n < 0 || p.lane_max_n > 8 || p.nedges < 1 || p.nedges > 16 || p.streams < 1 ||
        p.streams > 8 || (p.lane_block != 64 && p.lane_block != 256) ||
        (p.pool_waves != 0 && p.pool_waves != 8 && p.pool_waves != 12) ||
        (p.lane_group != 0 && p.lane_group != 1 && p.lane_group != 2 && p.lane_group != 4 && p.lane_group != 8) ||
        (p.group16 != 0 && p.group16 != 8 && p.group16 != 16) || (p.wave_global != 0 && p.wave_global != 1))
        return mt_fail(TRON_ERR_INVALID, "invalid plan spec");
    for (int i = 0; i < p.nedges; i++)
        if (p.edges[i] < 1 || p.edges[i] > 128 || (i > 0 && p.edges[i] <= p.edges[i - 1]))
            return mt_fail(TRON_ERR_INVALID, "plan edges must increase within 1..128");
    return TRON_OK;
}

// wave bucket of size n under the spec: the first edge >= n (0 if none)
static int spec_edge(const tron_plan_spec &p, int n)
{
    for (int i = 0; i < p.nedges; i++)
        if (n <= p.edges[i]) return p.edges[i];
    return 0;
}


struct tron_batch {
    int device = 0;
    tron_plan_spec spec{};
    tron_family fam = TRON_FAMILY_QP4;
    int64_t batch = 0;
    int32_t n_uniform = 0;     // 0 when sizes differ
    int32_t nmax = 0;
    tron_options opt{};
    double *d_state = nullptr;
    int64_t *d_ts = nullptr;   // caller's timestamp buffer, or null
    int32_t *d_n = nullptr;
    int64_t *d_poff = nullptr, *d_voff = nullptr;
    std::vector<Bucket> buckets;
    // buckets run concurrently on side streams, forked from and joined to the caller's
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> ev;          // ev[0]: fork; ev[1 + k]: join of side stream k
    // captured solve (TRON_FLAG_GRAPH): replayed while the pointers stay the same
    hipGraphExec_t graph = nullptr;
    hipStream_t cap = nullptr;           // capture stream
    const void *graph_key[9] = {};
    // persistent form (spec.pool_waves > 0 on a mixed batch): the wavefront instances ordered
    // largest n first, their claim counter, and the lane instances in packs of 64 of one size
    bool pool = false;
    int64_t pool_count = 0, packs = 0;
    int32_t pool_nmax = 0, pool_pages = 0, cus = 0;
    int32_t *d_pool_index = nullptr, *d_counter = nullptr;
    int32_t *d_pack_index = nullptr, *d_pack_n = nullptr;
    std::vector<int64_t> pack_count;     // instances per lane size (1..8), for tron_batch_plan
};

static void drop_graph(tron_batch *h)
{
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    for (auto &k : h->graph_key) k = nullptr;
}

static mt::Options dev_options(const tron_options &o)
{
    mt::Options d;
    d.gtol = o.gtol;
    d.cg_rtol = o.cg_rtol;
    d.delta0 = o.delta0;
    d.max_iter = o.max_iter;
    d.warm = (o.flags & TRON_FLAG_WARM) ? 1 : 0;
    return d;
}

static void free_batch(tron_batch *h)
{
    if (!h) return;
    drop_graph(h);
    if (h->cap) (void)hipStreamDestroy(h->cap);
    for (hipStream_t q : h->side) (void)hipStreamDestroy(q);
    for (hipEvent_t e : h->ev) (void)hipEventDestroy(e);
    (void)hipFree(h->d_state);
    (void)hipFree(h->d_n);
    (void)hipFree(h->d_poff);
    (void)hipFree(h->d_voff);
    (void)hipFree(h->d_pool_index);
    (void)hipFree(h->d_counter);
    (void)hipFree(h->d_pack_index);
    (void)hipFree(h->d_pack_n);
    for (auto &b : h->buckets) {
        (void)hipFree(b.d_index);
        (void)hipFree(b.d_ws);
    }
    delete h;
}

static tron_err check_options(const tron_options &o)
{
    if (!(o.gtol >= 0.0) || o.max_iter < 0 || !(o.cg_rtol >= 0.0) || !(o.delta0 == o.delta0))
        return mt_fail(TRON_ERR_INVALID, "invalid options");
    return TRON_OK;
}

// The kernel of a bucket of instances of size n <= lane_max_n under the spec: the lane kernel
// of exactly that n, or the group kernel of width lane_group (null when the family has no
// such build); `lanes` receives the lanes per instance.
static lane_launch_fn small_launcher(tron_family fam, const tron_plan_spec &sp, int n, int *lanes)
{
    if (sp.lane_group > 1) {
        const int kn = fam == TRON_FAMILY_BR6 ? 6 : 8;
        lane_launch_fn f = n <= kn ? mt_group_launcher(fam, kn, sp.lane_group) : nullptr;
        if (f) {
            *lanes = sp.lane_group;
            return f;
        }
    }
    *lanes = 1;
    return lane_launcher(fam, n);
}

// The group kernel for lane_max_n < n <= 16 when the spec asks for one (else null).
static lane_launch_fn mid_launcher(tron_family fam, const tron_plan_spec &sp, int n)
{
    if (sp.group16 == 0 || n > 16 || n <= sp.lane_max_n) return nullptr;
    return mt_group_launcher(fam, 16, sp.group16);
}

// The persistent form: the wavefront instances sorted largest n first (within one n,
// instance order) and then interleaved from both ends (below), and the lane instances
// grouped by size into packs of 64 (the last pack of a size padded with -1).
static tron_err build_pool_plan(tron_batch *h, const std::vector<int32_t> &n, hipStream_t st)
{
    const tron_plan_spec &sp = h->spec;
    std::vector<int32_t> wave;
    std::vector<std::vector<int32_t>> lanes(9);
    for (int64_t i = 0; i < h->batch; i++) {
        const bool lane = n[i] <= sp.lane_max_n && lane_launcher(h->fam, n[i]) != nullptr;
        if (lane) lanes[n[i]].push_back((int32_t)i);
        else {
            if (!has_wave_kernel(h->fam)) return mt_fail(TRON_ERR_UNSUPPORTED, "n = %d has no kernel for this family", n[i]);
            wave.push_back((int32_t)i);
        }
    }
    std::stable_sort(wave.begin(), wave.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
    std::vector<int32_t> pidx, pn;
    h->pack_count.assign(9, 0);
    for (int k = 8; k >= 1; k--) {
        const auto &l = lanes[k];
        h->pack_count[k] = (int64_t)l.size();
        for (size_t i = 0; i < l.size(); i += 64) {
            for (size_t j = 0; j < 64; j++) pidx.push_back(i + j < l.size() ? l[i + j] : -1);
            pn.push_back(k);
        }
    }
    int dev = 0, cus = 0, lds = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    h->pool = true;
    h->cus = cus;
    // the pool takes what a workgroup may have, less the pool's own control block
    h->pool_pages = std::min(kPoolMaxPages, (int)((lds - (int)sizeof(PoolCtl)) / kPoolPage));
    h->pool_count = (int64_t)wave.size();
    h->packs = (int64_t)pn.size();
    h->pool_nmax = 0;
    for (int32_t i : wave) h->pool_nmax = std::max(h->pool_nmax, n[i]);
    if (h->pool_nmax > 0 &&
        (int64_t)h->pool_pages * kPoolPage < mt_wave_matrix_doubles(h->pool_nmax) * (int64_t)sizeof(double))
        return mt_fail(TRON_ERR_UNSUPPORTED, "n = %d does not fit the LDS pool", h->pool_nmax);
    // Claim order. Largest first keeps the costliest instances from ending the launch, but a
    // CU's pool holds only `fit` of the largest at once, and its other waves would sleep until
    // pages free up. So each of the largest is followed by enough of the smallest to fill the
    // CU's waves beside them (the two ends of the sorted list meet in the middle); when every
    // instance fits beside the others the order stays largest first.
    if (!wave.empty()) {
        const int64_t big = (mt_wave_matrix_doubles(h->pool_nmax) * (int64_t)sizeof(double) + kPoolPage - 1) / kPoolPage;
        const int fit = std::max(1, (int)(h->pool_pages / big));
        const int small_per_big = std::max(0, sp.pool_waves / fit - 1);
        if (small_per_big > 0) {
            std::vector<int32_t> o;
            o.reserve(wave.size());
            size_t f = 0, b = wave.size();
            while (f < b) {
                o.push_back(wave[f++]);
                for (int k = 0; k < small_per_big && f < b; k++) o.push_back(wave[--b]);
            }
            wave.swap(o);
        }
    }
    HIP_TRY(hipMalloc(&h->d_counter, sizeof(int32_t)));
    if (!wave.empty()) {
        HIP_TRY(hipMalloc(&h->d_pool_index, sizeof(int32_t) * wave.size()));
        HIP_TRY(hipMemcpyAsync(h->d_pool_index, wave.data(), sizeof(int32_t) * wave.size(), hipMemcpyHostToDevice, st));
    }
    if (!pn.empty()) {
        HIP_TRY(hipMalloc(&h->d_pack_index, sizeof(int32_t) * pidx.size()));
        HIP_TRY(hipMalloc(&h->d_pack_n, sizeof(int32_t) * pn.size()));
        HIP_TRY(hipMemcpyAsync(h->d_pack_index, pidx.data(), sizeof(int32_t) * pidx.size(), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(h->d_pack_n, pn.data(), sizeof(int32_t) * pn.size(), hipMemcpyHostToDevice, st));
    }
    prepare_pool_kernels(h->pool_pages * kPoolPage);
    HIP_TRY(hipStreamSynchronize(st));
    return TRON_OK;
}

// Buckets of the lane kernel: instances grouped by the smallest supported kernel size
// that holds them (sizes 1..8 each get their own kernel).
// Launch plan: n <= spec.lane_max_n goes to the lane kernel of exactly that n (one
// instance per lane); larger n to the wave kernel of the first spec edge >= n (one instance
// per wavefront, LDS sized for the edge), each bucket ordered largest first. Wave buckets
// (heaviest) are listed first so they start first.
static tron_err build_plan(tron_batch *h, const std::vector<int32_t> &n, hipStream_t st)
{
    if (h->batch == 0) return TRON_OK;
    const tron_plan_spec &sp = h->spec;
    auto lane_ok = [&](int k) { return k <= sp.lane_max_n && lane_launcher(h->fam, k) != nullptr; };
    if (h->n_uniform) {
        Bucket b{};
        b.count = h->batch;
        b.d_index = nullptr;
        if (lane_ok(h->n_uniform)) {
            b.nmax = h->n_uniform;
            // automatic group width: for a uniform quartic batch of n = 7 or 8 up to 16,384
            // instances, 8 lanes per instance shorten each solve's chain more than the extra
            // waves cost (measured 1.3-1.6x less time from 256 to 16,384 instances; at 65,536
            // the eight waves per SIMD take 2.2x longer than one lane per instance)
            tron_plan_spec eff = sp;
            if (eff.lane_group == 0)
                eff.lane_group = (h->fam == TRON_FAMILY_QP4 && h->n_uniform >= 7 && h->batch <= 16384) ? 8 : 1;
            b.lane = small_launcher(h->fam, eff, h->n_uniform, &b.lanes);
        } else if (lane_launch_fn m = mid_launcher(h->fam, sp, h->n_uniform)) {
            b.nmax = 16;
            b.lanes = sp.group16;
            b.lane = m;
        } else {
            if (!has_wave_kernel(h->fam)) return mt_fail(TRON_ERR_UNSUPPORTED, "this family has no wave kernel");
            b.nmax = h->n_uniform;
            b.lanes = 64;
            b.lane = nullptr;
            if ((b.nmax > kLdsMaxN || (sp.wave_global && h->fam == TRON_FAMILY_QP4)) &&
                hipMalloc(&b.d_ws, sizeof(double) * (size_t)mt_wave_matrix_doubles(b.nmax) * (size_t)b.count) != hipSuccess)
                return mt_fail(TRON_ERR_NOMEM, "matrix workspace allocation failed");
        }
        h->buckets.push_back(b);
        return TRON_OK;
    }
    if (sp.pool_waves > 0) {
        int nmax = 0;
        for (int64_t i = 0; i < h->batch; i++) nmax = std::max(nmax, n[i]);
        if (nmax <= kLdsMaxN) return build_pool_plan(h, n, st);
    }
    std::vector<std::vector<int32_t>> lane_lists(9);
    std::vector<int32_t> mid_list;                   // lane_max_n < n <= 16 on the group kernel
    std::map<int, std::vector<int32_t>> wave_lists;  // edge -> instances
    for (int64_t i = 0; i < h->batch; i++) {
        if (lane_ok(n[i])) lane_lists[n[i]].push_back((int32_t)i);
        else if (mid_launcher(h->fam, sp, n[i])) mid_list.push_back((int32_t)i);
        else {
            if (!has_wave_kernel(h->fam)) return mt_fail(TRON_ERR_UNSUPPORTED, "n = %d has no kernel for this family", n[i]);
            const int e = n[i] > kLdsMaxN ? global_edge(n[i]) : spec_edge(sp, n[i]);
            if (!e) return mt_fail(TRON_ERR_UNSUPPORTED, "n = %d above the largest plan edge", n[i]);
            wave_lists[e].push_back((int32_t)i);
        }
    }
    // lanes: 64 for the wavefront kernel, else the lanes per instance of `fn`
    auto add = [&](std::vector<int32_t> &list, int nmax, int lanes, lane_launch_fn fn) -> tron_err {
        // registered first, so that free_batch releases whatever the allocations below got
        h->buckets.push_back(Bucket{});
        Bucket &b = h->buckets.back();
        b.nmax = nmax;
        b.lanes = lanes;
        b.count = (int64_t)list.size();
        b.lane = fn;
        if (lanes == 64 && (nmax > kLdsMaxN || (sp.wave_global && h->fam == TRON_FAMILY_QP4)) &&
            hipMalloc(&b.d_ws, sizeof(double) * (size_t)mt_wave_matrix_doubles(nmax) * list.size()) != hipSuccess)
            return mt_fail(TRON_ERR_NOMEM, "matrix workspace allocation failed");
        HIP_TRY(hipMalloc(&b.d_index, sizeof(int32_t) * list.size()));
        HIP_TRY(hipMemcpyAsync(b.d_index, list.data(), sizeof(int32_t) * list.size(), hipMemcpyHostToDevice, st));
        return TRON_OK;
    };
    for (auto it = wave_lists.rbegin(); it != wave_lists.rend(); ++it) {
        auto &list = it->second;
        std::stable_sort(list.begin(), list.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
        tron_err rc = add(list, it->first, 64, nullptr);
        if (rc != TRON_OK) return rc;
    }
    if (!mid_list.empty()) {
        std::stable_sort(mid_list.begin(), mid_list.end(), [&](int32_t a, int32_t b) { return n[a] > n[b]; });
        tron_err rc = add(mid_list, 16, sp.group16, mid_launcher(h->fam, sp, n[mid_list[0]]));
        if (rc != TRON_OK) return rc;
    }
    for (int k = 8; k >= 1; k--) {
        if (lane_lists[k].empty()) continue;
        int lanes = 1;
        lane_launch_fn fn = small_launcher(h->fam, sp, k, &lanes);
        tron_err rc = add(lane_lists[k], k, lanes, fn);
        if (rc != TRON_OK) return rc;
    }
    // the device copies above read host vectors that die with this call
    HIP_TRY(hipStreamSynchronize(st));
    return TRON_OK;
}

extern "C" void tron_default_plan_spec(tron_plan_spec *spec)
{
    if (spec) default_spec(spec);
}

extern "C" tron_err tron_batch_create_ex(tron_batch **out, tron_family fam, int64_t batch,
                                         const int32_t *n_host, int32_t n_uniform,
                                         const tron_options *opt, const tron_plan_spec *spec,
                                         void *stream);

extern "C" tron_err tron_batch_create(tron_batch **out, tron_family fam, int64_t batch,
                                      const int32_t *n_host, int32_t n_uniform,
                                      const tron_options *opt, void *stream)
{
    return tron_batch_create_ex(out, fam, batch, n_host, n_uniform, opt, nullptr, stream);
}

extern "C" tron_err tron_batch_create_ex(tron_batch **out, tron_family fam, int64_t batch,
                                         const int32_t *n_host, int32_t n_uniform,
                                         const tron_options *opt, const tron_plan_spec *spec,
                                         void *stream)
{
    tron_plan_spec sp;
    default_spec(&sp);
    if (spec) {
        sp = *spec;
        if (check_spec(sp) != TRON_OK) return TRON_ERR_INVALID;
    }
    if (!out) return mt_fail(TRON_ERR_INVALID, "out is null");
    *out = nullptr;
    if (batch < 0 || batch > (int64_t)INT32_MAX) return mt_fail(TRON_ERR_INVALID, "batch out of range");
    if (fam != TRON_FAMILY_QP4 && fam != TRON_FAMILY_BR6 && fam != TRON_FAMILY_HS45M &&
        fam != TRON_FAMILY_BR8L)
        return mt_fail(TRON_ERR_INVALID, "unknown family");
    tron_options o;
    tron_default_options(&o);
    if (opt) o = *opt;
    if (check_options(o) != TRON_OK) return TRON_ERR_INVALID;
    hipStream_t st = (hipStream_t)stream;
    std::vector<int32_t> n;
    int32_t uni = 0;
    if (n_host) {
        n.assign(n_host, n_host + batch);
        uni = batch > 0 ? n[0] : 1;
        for (int64_t i = 0; i < batch; i++) {
            if (tron_param_size(fam, n[i]) < 0)
                return mt_fail(TRON_ERR_INVALID, "instance %lld: n = %d invalid for the family", (long long)i, n[i]);
            if (n[i] != uni) uni = 0;
        }
    } else {
        if (tron_param_size(fam, n_uniform) < 0)
            return mt_fail(TRON_ERR_INVALID, "n = %d invalid for the family", n_uniform);
        uni = n_uniform;
    }
    tron_batch *h = new (std::nothrow) tron_batch();
    if (!h) return mt_fail(TRON_ERR_NOMEM, "host allocation failed");
    (void)hipGetDevice(&h->device);
    h->fam = fam;
    h->spec = sp;
    h->batch = batch;
    h->n_uniform = uni;
    h->opt = o;
    tron_err rc = TRON_OK;
    auto bail = [&](tron_err e) { free_batch(h); return e; };
    if (batch > 0) {
        if (hipMalloc(&h->d_state, sizeof(double) * 2 * batch) != hipSuccess)
            return bail(mt_fail(TRON_ERR_NOMEM, "state allocation failed"));
        if (hipMemsetAsync(h->d_state, 0, sizeof(double) * 2 * batch, st) != hipSuccess)
            return bail(mt_fail(TRON_ERR_DEVICE, "state clear failed"));
    }
    if (!uni && batch > 0) {
        std::vector<int64_t> po(batch), vo(batch);
        int64_t pa = 0, va = 0;
        for (int64_t i = 0; i < batch; i++) {
            po[i] = pa;
            vo[i] = va;
            pa += tron_param_size(fam, n[i]);
            va += n[i];
        }
        if (hipMalloc(&h->d_n, sizeof(int32_t) * batch) != hipSuccess ||
            hipMalloc(&h->d_poff, sizeof(int64_t) * batch) != hipSuccess ||
            hipMalloc(&h->d_voff, sizeof(int64_t) * batch) != hipSuccess)
            return bail(mt_fail(TRON_ERR_NOMEM, "offset allocation failed"));
        if (hipMemcpyAsync(h->d_n, n.data(), sizeof(int32_t) * batch, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(h->d_poff, po.data(), sizeof(int64_t) * batch, hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(h->d_voff, vo.data(), sizeof(int64_t) * batch, hipMemcpyHostToDevice, st) != hipSuccess)
            return bail(mt_fail(TRON_ERR_DEVICE, "offset upload failed"));
        // the host vectors die here; make the copies complete first
        if (hipStreamSynchronize(st) != hipSuccess) return bail(mt_fail(TRON_ERR_DEVICE, "sync failed"));
    }
    rc = build_plan(h, n, st);
    if (rc != TRON_OK) return bail(rc);
    const size_t parts = h->pool ? (size_t)((h->pool_count > 0) + (h->packs > 0)) : h->buckets.size();
    if (parts > 1 && (h->pool || sp.streams > 1)) {
        const int k = h->pool ? 2 : (int)std::min<size_t>(h->buckets.size(), (size_t)sp.streams);
        for (int i = 0; i < k; i++) {
            hipStream_t q;
            if (hipStreamCreateWithFlags(&q, hipStreamNonBlocking) != hipSuccess)
                return bail(mt_fail(TRON_ERR_DEVICE, "stream creation failed"));
            h->side.push_back(q);
        }
        for (int i = 0; i <= k; i++) {
            hipEvent_t e;
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
                return bail(mt_fail(TRON_ERR_DEVICE, "event creation failed"));
            h->ev.push_back(e);
        }
    }
    mt_prepare_wave_kernels();
    if (hipStreamSynchronize(st) != hipSuccess) return bail(mt_fail(TRON_ERR_DEVICE, "sync failed"));
    *out = h;
    return TRON_OK;
}

extern "C" tron_err tron_batch_solve(tron_batch *h, const double *d_params, const double *d_lo,
                                     const double *d_hi, const double *d_x0, double *d_x,
                                     double *d_f, int32_t *d_status, int32_t *d_iters, void *stream)
{
    if (!h) return mt_fail(TRON_ERR_INVALID, "handle is null");
    if (h->batch == 0) return TRON_OK;
    if ((!d_params && h->fam != TRON_FAMILY_HS45M) || !d_lo || !d_hi || !d_x0 || !d_x || !d_f ||
        !d_status || !d_iters)
        return mt_fail(TRON_ERR_INVALID, "null device pointer");
    hipStream_t st = (hipStream_t)stream;
    LaneArgs a{};
    a.params = d_params;
    a.lo = d_lo;
    a.hi = d_hi;
    a.x0 = d_x0;
    a.x = d_x;
    a.f = d_f;
    a.status = d_status;
    a.iters = d_iters;
    a.state = h->d_state;
    a.ts = h->d_ts;
    a.nper = h->n_uniform ? nullptr : h->d_n;
    a.poff = h->n_uniform ? nullptr : h->d_poff;
    a.voff = h->n_uniform ? nullptr : h->d_voff;
    a.batch = h->batch;
    a.n_uniform = h->n_uniform;
    a.psize = h->n_uniform ? (int32_t)tron_param_size(h->fam, h->n_uniform) : 0;
    a.opt = dev_options(h->opt);
    a.lane_block = h->spec.lane_block;
    const bool use_graph = (h->opt.flags & TRON_FLAG_GRAPH) != 0u;
    const void *key[9] = {d_params, d_lo, d_hi, d_x0, d_x, d_f, d_status, d_iters, h->d_ts};
    if (use_graph && h->graph && std::equal(key, key + 9, h->graph_key)) {
        HIP_TRY(hipGraphLaunch(h->graph, st));
        return TRON_OK;
    }
    hipStream_t cs = st;  // where the launch sequence is enqueued (or captured)
    if (use_graph) {
        // capture on the handle's own stream (the caller's may be the null stream, which
        // cannot be captured); the graph is then launched on the caller's stream
        drop_graph(h);
        if (!h->cap) HIP_TRY(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
        cs = h->cap;
        HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    }
    tron_err rc = TRON_OK;
    if (h->pool) {
        // the lane packs and the persistent launch, side by side when both exist
        LaneArgs ap = a, al = a;
        ap.index = h->d_pool_index;
        ap.count = h->pool_count;
        al.index = h->d_pack_index;
        al.count = h->packs * 64;
        const PoolArgs pa{h->d_counter, h->pool_pages};
        const int waves = h->spec.pool_waves;
        if (h->side.empty()) {
            launch_pool(h->fam, ap, pa, h->pool_nmax, waves, h->cus, cs);
            launch_lane_packs(h->fam, al, h->d_pack_n, h->packs, cs);
        } else {
            if (hipEventRecord(h->ev[0], cs) != hipSuccess) rc = mt_fail(TRON_ERR_DEVICE, "event record failed");
            for (int i = 0; i < 2 && rc == TRON_OK; i++)
                if (hipStreamWaitEvent(h->side[i], h->ev[0], 0) != hipSuccess)
                    rc = mt_fail(TRON_ERR_DEVICE, "stream wait failed");
            if (rc == TRON_OK) {
                launch_pool(h->fam, ap, pa, h->pool_nmax, waves, h->cus, h->side[0]);
                launch_lane_packs(h->fam, al, h->d_pack_n, h->packs, h->side[1]);
            }
            for (int i = 0; i < 2 && rc == TRON_OK; i++)
                if (hipEventRecord(h->ev[1 + i], h->side[i]) != hipSuccess ||
                    hipStreamWaitEvent(cs, h->ev[1 + i], 0) != hipSuccess)
                    rc = mt_fail(TRON_ERR_DEVICE, "join failed");
        }
    } else if (h->side.empty()) {
        for (const Bucket &b : h->buckets) {
            a.index = b.d_index;
            a.count = b.count;
            launch_bucket(h->fam, b, a, cs);
        }
    } else {
        // fork: every side stream waits for the caller's stream; buckets are dealt to the
        // side streams heaviest first; join: the caller's stream waits for all of them
        const int k = (int)h->side.size();
        if (hipEventRecord(h->ev[0], cs) != hipSuccess) rc = mt_fail(TRON_ERR_DEVICE, "event record failed");
        for (int i = 0; i < k && rc == TRON_OK; i++)
            if (hipStreamWaitEvent(h->side[i], h->ev[0], 0) != hipSuccess)
                rc = mt_fail(TRON_ERR_DEVICE, "stream wait failed");
        for (size_t i = 0; i < h->buckets.size() && rc == TRON_OK; i++) {
            const Bucket &b = h->buckets[i];
            a.index = b.d_index;
            a.count = b.count;
            launch_bucket(h->fam, b, a, h->side[i % k]);
        }
        for (int i = 0; i < k && rc == TRON_OK; i++) {
            if (hipEventRecord(h->ev[1 + i], h->side[i]) != hipSuccess ||
                hipStreamWaitEvent(cs, h->ev[1 + i], 0) != hipSuccess)
                rc = mt_fail(TRON_ERR_DEVICE, "join failed");
        }
    }
    if (use_graph) {
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (rc == TRON_OK && e != hipSuccess) rc = mt_fail(TRON_ERR_DEVICE, "capture failed: %s", hipGetErrorString(e));
        if (rc == TRON_OK) {
            e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = mt_fail(TRON_ERR_DEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
        }
        if (g) (void)hipGraphDestroy(g);
        if (rc != TRON_OK) {
            drop_graph(h);
            return rc;
        }
        std::copy(key, key + 9, h->graph_key);
        HIP_TRY(hipGraphLaunch(h->graph, st));
        return TRON_OK;
    }
    if (rc != TRON_OK) return rc;
    HIP_TRY(hipGetLastError());
    return TRON_OK;
}

extern "C" void tron_default_al_options(tron_al_options *o)
{
    if (!o) return;
    o->ctol = 1e-6;
    o->outer_max = 50;
    o->rho_growth = 10.0;
    o->decrease = 0.25;
    o->rho_max = 1e6;
}

extern "C" tron_err tron_al_solve(tron_batch *h, const tron_al_options *opt, double *d_params,
                                  const double *d_lo, const double *d_hi, const double *d_x0,
                                  double *d_x, double *d_f, int32_t *d_status, int32_t *d_iters,
                                  int32_t *d_outer, double *d_viol, void *stream)
{
    if (!h) return mt_fail(TRON_ERR_INVALID, "handle is null");
    if (h->fam != TRON_FAMILY_BR8L) return mt_fail(TRON_ERR_UNSUPPORTED, "the multiplier loop needs a BR8L batch");
    tron_al_options o;
    tron_default_al_options(&o);
    if (opt) o = *opt;
    if (!(o.ctol >= 0.0) || o.outer_max < 1 || !(o.rho_growth >= 1.0) || !(o.decrease >= 0.0) ||
        !(o.rho_max > 0.0))
        return mt_fail(TRON_ERR_INVALID, "invalid multiplier-loop options");
    if (h->batch == 0) return TRON_OK;
    if (!d_params || !d_lo || !d_hi || !d_x0 || !d_x || !d_f || !d_status || !d_iters || !d_outer || !d_viol)
        return mt_fail(TRON_ERR_INVALID, "null device pointer");
    LaneArgs a{};
    a.lo = d_lo;
    a.hi = d_hi;
    a.x0 = d_x0;
    a.x = d_x;
    a.f = d_f;
    a.status = d_status;
    a.iters = d_iters;
    a.state = h->d_state;
    a.count = h->batch;
    a.batch = h->batch;
    a.n_uniform = 8;
    a.psize = 40;
    a.opt = dev_options(h->opt);
    AlArgs al{d_params, d_outer, d_viol, o.ctol, o.rho_growth, o.decrease, o.rho_max, o.outer_max};
    const unsigned grid = (unsigned)((h->batch + kLaneBlock - 1) / kLaneBlock);
    hipLaunchKernelGGL(al_kernel, dim3(grid), dim3(kLaneBlock), 0, (hipStream_t)stream, a, al);
    HIP_TRY(hipGetLastError());
    return TRON_OK;
}

extern "C" tron_err tron_batch_get_state(tron_batch *h, double *d_state, void *stream)
{
    if (!h || (!d_state && h->batch)) return mt_fail(TRON_ERR_INVALID, "null argument");
    if (h->batch)
        HIP_TRY(hipMemcpyAsync(d_state, h->d_state, sizeof(double) * 2 * h->batch,
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return TRON_OK;
}

extern "C" tron_err tron_batch_set_state(tron_batch *h, const double *d_state, void *stream)
{
    if (!h || (!d_state && h->batch)) return mt_fail(TRON_ERR_INVALID, "null argument");
    if (h->batch)
        HIP_TRY(hipMemcpyAsync(h->d_state, d_state, sizeof(double) * 2 * h->batch,
                               hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return TRON_OK;
}

extern "C" tron_err tron_batch_set_options(tron_batch *h, const tron_options *opt)
{
    if (!h || !opt) return mt_fail(TRON_ERR_INVALID, "null argument");
    if (check_options(*opt) != TRON_OK) return TRON_ERR_INVALID;
    h->opt = *opt;
    drop_graph(h);
    return TRON_OK;
}

extern "C" tron_err tron_batch_plan(const tron_batch *h, int32_t *nbuckets, int32_t *desc,
                                    int32_t max_buckets)
{
    if (!h || !nbuckets) return mt_fail(TRON_ERR_INVALID, "null argument");
    if (h->pool) {
        // the persistent launch as one entry (largest n, 64 lanes, its instances), then one
        // entry per lane size
        std::vector<int32_t> d;
        if (h->pool_count) d.insert(d.end(), {h->pool_nmax, 64, (int32_t)h->pool_count});
        for (int k = 8; k >= 1; k--)
            if (h->pack_count.size() > (size_t)k && h->pack_count[k]) d.insert(d.end(), {k, 1, (int32_t)h->pack_count[k]});
        *nbuckets = (int32_t)(d.size() / 3);
        for (int32_t i = 0; desc && i < max_buckets && i < *nbuckets; i++)
            for (int c = 0; c < 3; c++) desc[3 * i + c] = d[3 * i + c];
        return TRON_OK;
    }
    *nbuckets = (int32_t)h->buckets.size();
    for (int32_t i = 0; desc && i < max_buckets && i < (int32_t)h->buckets.size(); i++) {
        desc[3 * i] = h->buckets[i].nmax;
        desc[3 * i + 1] = h->buckets[i].lanes;
        desc[3 * i + 2] = (int32_t)h->buckets[i].count;
    }
    return TRON_OK;
}

extern "C" tron_err tron_batch_set_timestamps(tron_batch *h, int64_t *d_ts)
{
    if (!h) return mt_fail(TRON_ERR_INVALID, "handle is null");
    h->d_ts = d_ts;
    drop_graph(h);
    return TRON_OK;
}

extern "C" int64_t tron_clock_rate_hz(void)
{
    int dev = 0, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) return 0;
    return (int64_t)khz * 1000;
}

extern "C" tron_err tron_batch_destroy(tron_batch *h)
{
    free_batch(h);
    return TRON_OK;
}

// ------------------------------------------------------------------------------------
// autotuner
// ------------------------------------------------------------------------------------
static std::string tune_key(tron_family fam, int64_t batch, const int32_t *n)
{
    // family, batch, and the share of instances per size class (exact n <= 8, then octaves)
    int64_t cls[13] = {0};
    for (int64_t i = 0; i < batch; i++) {
        const int k = n[i];
        const int c = k <= 8 ? k : k <= 16 ? 9 : k <= 32 ? 10 : k <= 64 ? 11 : 12;
        cls[c]++;
    }
    std::ostringstream o;
    o << "fam=" << (int)fam << " batch=" << batch << " hist=";
    for (int c = 1; c <= 12; c++) o << (c > 1 ? "," : "") << (batch ? (100 * cls[c] + batch / 2) / batch : 0);
    return o.str();
}

static std::string spec_str(const tron_plan_spec &p)
{
    std::ostringstream o;
    o << p.lane_max_n << " " << p.streams << " " << p.lane_block << " " << p.nedges;
    for (int i = 0; i < p.nedges; i++) o << " " << p.edges[i];
    o << " " << p.pool_waves << " " << p.lane_group << " " << p.group16 << " " << p.wave_global;
    return o.str();
}

static bool spec_parse(const std::string &t, tron_plan_spec *p)
{
    std::istringstream in(t);
    tron_plan_spec q{};
    if (!(in >> q.lane_max_n >> q.streams >> q.lane_block >> q.nedges)) return false;
    if (q.nedges < 1 || q.nedges > 16) return false;
    for (int i = 0; i < q.nedges; i++)
        if (!(in >> q.edges[i])) return false;
    if (!(in >> q.pool_waves)) q.pool_waves = 0;
    if (!(in >> q.lane_group)) q.lane_group = 1;
    if (!(in >> q.group16)) q.group16 = 0;
    if (!(in >> q.wave_global)) q.wave_global = 0;
    if (check_spec(q) != TRON_OK) return false;
    *p = q;
    return true;
}

extern "C" tron_err tron_autotune(tron_family fam, int64_t batch, const int32_t *n_host,
                                  const double *d_params, const double *d_lo, const double *d_hi,
                                  const double *d_x0, double *d_x, double *d_f, int32_t *d_status,
                                  int32_t *d_iters, int32_t reps, const char *cache_path,
                                  tron_plan_spec *best, double *best_ms, void *stream)
{
    if (!n_host || !best || batch <= 0 || reps < 1) return mt_fail(TRON_ERR_INVALID, "bad argument");
    hipStream_t st = (hipStream_t)stream;
    const std::string key = tune_key(fam, batch, n_host);
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (std::getline(in, line)) {
            const size_t bar = line.find('|');
            if (bar != std::string::npos && line.substr(0, bar) == key && spec_parse(line.substr(bar + 1), best)) {
                if (best_ms) *best_ms = -1.0;
                return TRON_OK;
            }
        }
    }
    int nmax = 0;
    for (int64_t i = 0; i < batch; i++) nmax = std::max(nmax, n_host[i]);
    const std::vector<std::vector<int>> edge_sets = {
        {16, 32, 64, 128}, {32, 64, 128}, {12, 16, 24, 32, 48, 64, 96, 128},
        {16, 24, 32, 40, 48, 56, 64, 80, 96, 112, 128}};
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // candidates are timed as captured graphs: the device time of the plan, without the
    // host's launch overhead, which differs between plans of 2 and of 12 launches
    tron_options gopt;
    tron_default_options(&gopt);
    gopt.flags |= TRON_FLAG_GRAPH;
    auto time_once = [&](const tron_plan_spec &sp, double *ms) -> tron_err {
        tron_batch *h = nullptr;
        tron_err rc = tron_batch_create_ex(&h, fam, batch, n_host, 0, &gopt, &sp, stream);
        if (rc != TRON_OK) return rc;
        rc = tron_batch_solve(h, d_params, d_lo, d_hi, d_x0, d_x, d_f, d_status, d_iters, stream);
        float best_t = 1e30f;
        for (int r = 0; r < reps && rc == TRON_OK; r++) {
            if (hipEventRecord(e0, st) != hipSuccess) rc = mt_fail(TRON_ERR_DEVICE, "event");
            if (rc == TRON_OK) rc = tron_batch_solve(h, d_params, d_lo, d_hi, d_x0, d_x, d_f, d_status, d_iters, stream);
            if (rc == TRON_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                rc = mt_fail(TRON_ERR_DEVICE, "event");
            float t = 0.0f;
            if (rc == TRON_OK && hipEventElapsedTime(&t, e0, e1) == hipSuccess) best_t = std::min(best_t, t);
        }
        tron_batch_destroy(h);
        *ms = best_t;
        return rc;
    };
    // every timed candidate, for the confirmation round at the end
    std::vector<std::pair<double, tron_plan_spec>> seen;
    auto time_spec = [&](const tron_plan_spec &sp, double *ms) -> tron_err {
        const tron_err r = time_once(sp, ms);
        if (r == TRON_OK) seen.emplace_back(*ms, sp);
        return r;
    };
    tron_plan_spec cur;
    default_spec(&cur);
    cur.pool_waves = 0;  // stages 1-3 tune the bucketed form, stage 4 the persistent one
    double cur_ms = 1e30;
    tron_err rc = TRON_OK;
    // stage 1: bucket edges x streams
    for (const auto &es : edge_sets) {
        for (int streams : {1, 4}) {
            tron_plan_spec sp;
            default_spec(&sp);
            sp.pool_waves = 0;
            sp.nedges = (int)es.size();
            for (int i = 0; i < sp.nedges; i++) sp.edges[i] = es[i];
            sp.streams = streams;
            if (spec_edge(sp, nmax) == 0 && nmax > sp.lane_max_n) continue;
            double ms = 0.0;
            rc = time_spec(sp, &ms);
            if (rc != TRON_OK) break;
            if (ms < cur_ms) { cur_ms = ms; cur = sp; }
        }
        if (rc != TRON_OK) break;
    }
    // stage 2: lane/wave split and lane workgroup size on the best edges
    for (int lane_max : {4, 6, 8}) {
        for (int blk : {64, 256}) {
            if (rc != TRON_OK) break;
            tron_plan_spec sp = cur;
            sp.lane_max_n = lane_max;
            sp.lane_block = blk;
            if (lane_max == cur.lane_max_n && blk == cur.lane_block) continue;
            double ms = 0.0;
            rc = time_spec(sp, &ms);
            if (rc == TRON_OK && ms < cur_ms) { cur_ms = ms; cur = sp; }
        }
    }
    // stage 3: group widths for the lane sizes and for 8 < n <= 16
    for (int lg : {2, 4, 8}) {
        if (rc != TRON_OK) break;
        tron_plan_spec sp = cur;
        sp.lane_group = lg;
        double ms = 0.0;
        rc = time_spec(sp, &ms);
        if (rc == TRON_OK && ms < cur_ms) { cur_ms = ms; cur = sp; }
    }
    if (has_wave_kernel(fam) && nmax > cur.lane_max_n) {
        for (int g16 : {8, 16}) {
            if (rc != TRON_OK) break;
            tron_plan_spec sp = cur;
            sp.group16 = g16;
            double ms = 0.0;
            rc = time_spec(sp, &ms);
            if (rc == TRON_OK && ms < cur_ms) { cur_ms = ms; cur = sp; }
        }
    }
    // stage 4: the persistent form (wave instances up to 128 only) with the best lane split so
    // far, the default split (n <= 8 on lane kernels) and no lane kernels
    if (nmax <= kLdsMaxN && has_wave_kernel(fam)) {
        const tron_plan_spec base = cur;
        std::vector<int> splits;
        for (int lm : {base.lane_max_n, 8, 0})
            if (std::find(splits.begin(), splits.end(), lm) == splits.end()) splits.push_back(lm);
        for (int waves : {8, 12}) {
            for (int lane_max : splits) {
                if (rc != TRON_OK) break;
                tron_plan_spec sp = base;
                sp.pool_waves = waves;
                sp.lane_max_n = lane_max;
                if (lane_max != base.lane_max_n) sp.lane_group = 1;
                double ms = 0.0;
                rc = time_spec(sp, &ms);
                if (rc == TRON_OK && ms < cur_ms) { cur_ms = ms; cur = sp; }
            }
        }
    }
    // Confirmation: one timing per candidate can rank plans within a few per cent of each
    // other by noise, so the four fastest distinct candidates are timed again in three
    // interleaved rounds and the lowest median wins.
    if (rc == TRON_OK && seen.size() > 1) {
        std::stable_sort(seen.begin(), seen.end(),
                         [](const std::pair<double, tron_plan_spec> &a, const std::pair<double, tron_plan_spec> &b) {
                             return a.first < b.first;
                         });
        std::vector<tron_plan_spec> fin;
        std::vector<std::string> keys;
        for (const auto &c : seen) {
            const std::string k = spec_str(c.second);
            if (std::find(keys.begin(), keys.end(), k) != keys.end()) continue;
            keys.push_back(k);
            fin.push_back(c.second);
            if (fin.size() == 4) break;
        }
        std::vector<std::vector<double>> t(fin.size());
        for (int round = 0; round < 3 && rc == TRON_OK; round++)
            for (size_t i = 0; i < fin.size() && rc == TRON_OK; i++) {
                const size_t k = round % 2 ? fin.size() - 1 - i : i;
                double ms = 0.0;
                rc = time_once(fin[k], &ms);
                t[k].push_back(ms);
            }
        if (rc == TRON_OK) {
            double best_med = 1e30;
            for (size_t i = 0; i < fin.size(); i++) {
                std::sort(t[i].begin(), t[i].end());
                const double med = t[i][t[i].size() / 2];
                if (med < best_med) { best_med = med; cur = fin[i]; cur_ms = med; }
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != TRON_OK) return rc;
    *best = cur;
    if (best_ms) *best_ms = cur_ms;
    if (cache_path) {
        std::ofstream out(cache_path, std::ios::app);
        if (out) out << key << "|" << spec_str(cur) << "\n";
    }
    return TRON_OK;
}

// ------------------------------------------------------------------------------------
// allocation-free solve: the working memory of one uniform-n solve (per-instance radius and
// Cauchy step length, and for n > 128 the matrix workspace) lives in one fixed device array
// instead of handle allocations
// ------------------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kScratchMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kScratchMaxDevices];  // device address of `scratch`, per device

// The device address of this device's copy of `scratch` (the host-side name is only a
// stand-in); looked up once per device, with that device current.
static tron_err scratch_address(double **out)
{
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kScratchMaxDevices)
        return mt_fail(TRON_ERR_UNSUPPORTED, "device %d: the allocation-free solve supports devices 0..%d", dev,
                       kScratchMaxDevices - 1);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return mt_fail(TRON_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        mt_prepare_wave_kernels();
        g_scratch_dev[dev] = (double *)p;
    }
    *out = g_scratch_dev[dev];
    return TRON_OK;
}

extern "C" int64_t tron_noalloc_scratch_bytes(void) { return (int64_t)kScratchBytes; }

extern "C" tron_err tron_solve_noalloc(tron_family fam, int64_t batch, int32_t n, const tron_options *opt,
                                       const double *d_params, const double *d_lo, const double *d_hi,
                                       const double *d_x0, double *d_x, double *d_f, int32_t *d_status,
                                       int32_t *d_iters, void *stream)
{
    if (fam != TRON_FAMILY_QP4 && fam != TRON_FAMILY_BR6 && fam != TRON_FAMILY_HS45M && fam != TRON_FAMILY_BR8L)
        return mt_fail(TRON_ERR_INVALID, "unknown family");
    if (batch < 0 || batch > (int64_t)INT32_MAX) return mt_fail(TRON_ERR_INVALID, "batch out of range");
    const int64_t psize = tron_param_size(fam, n);
    if (psize < 0) return mt_fail(TRON_ERR_INVALID, "n = %d invalid for the family", n);
    tron_options o;
    tron_default_options(&o);
    if (opt) o = *opt;
    if (check_options(o) != TRON_OK) return TRON_ERR_INVALID;
    if (o.flags != 0u) return mt_fail(TRON_ERR_INVALID, "the allocation-free solve takes no flags (cold start, no graph)");
    if (batch == 0) return TRON_OK;
    if ((!d_params && fam != TRON_FAMILY_HS45M) || !d_lo || !d_hi || !d_x0 || !d_x || !d_f || !d_status || !d_iters)
        return mt_fail(TRON_ERR_INVALID, "null device pointer");
    const bool lane = n <= 8 && lane_launcher(fam, n) != nullptr;
    if (!lane && !has_wave_kernel(fam)) return mt_fail(TRON_ERR_UNSUPPORTED, "this family has no wave kernel");
    // scratch layout: radii [batch], Cauchy steps [batch], then (n > 128) the matrix slots,
    // 256-byte aligned
    const int64_t state_doubles = (2 * batch + 31) / 32 * 32;
    const int64_t ws_stride = (!lane && n > kLdsMaxN) ? mt_wave_matrix_doubles(n) : 0;
    const int64_t need = state_doubles + ws_stride * batch;
    if (need > (int64_t)(kScratchBytes / sizeof(double)))
        return mt_fail(TRON_ERR_INVALID,
                       "%lld instances of n = %d need %lld bytes of working memory; the allocation-free solve "
                       "holds %lld",
                       (long long)batch, n, (long long)(need * (int64_t)sizeof(double)), (long long)kScratchBytes);
    double *sp = nullptr;
    tron_err rc = scratch_address(&sp);
    if (rc != TRON_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    LaneArgs a{};
    a.params = d_params;
    a.lo = d_lo;
    a.hi = d_hi;
    a.x0 = d_x0;
    a.x = d_x;
    a.f = d_f;
    a.status = d_status;
    a.iters = d_iters;
    a.state = sp;  // written, not read (cold start)
    a.count = batch;
    a.batch = batch;
    a.n_uniform = n;
    a.psize = (int32_t)psize;
    a.opt = dev_options(o);
    a.lane_block = 64;
    if (lane) {
        lane_launcher(fam, n)(a, st);
    } else {
        a.ws = ws_stride ? sp + state_doubles : nullptr;
        a.ws_stride = ws_stride;
        launch_wave_fam(fam, a, n, st);
    }
    HIP_TRY(hipGetLastError());
    return TRON_OK;
}
