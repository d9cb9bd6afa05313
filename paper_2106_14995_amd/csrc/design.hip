// design.hip -- the kernel-design alternatives of section 4 (Tables 1-3) as batched kernels,
// one wavefront per problem, lane i owning row i (see include/tron_design.h).
#include <hip/hip_runtime.h>

#include "tron_design.h"
#include "tron_internal.hpp"
#include "wave_tron.hpp"

namespace {

using mt::bcast;

MT_INLINE void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// the same for a workspace in global memory: the acquire side is taken at device scope so
// that no lane reads a stale vector-L1 line that another lane has just written through
MT_INLINE void wave_sync_global()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Lower triangle of problem p's n x n row-major block into W (row stride ld); coalesced
// over the flat index, the strict upper part of W is left alone.
MT_INLINE void stage_lower(double *W, int ld, const double *__restrict__ src, int n)
{
    for (int e = threadIdx.x; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        if (c <= r) W[r * ld + c] = src[e];
    }
}

// L (lower part of W, row stride ld) out to dst as a dense row-major block, zero above.
MT_INLINE void write_lower(double *__restrict__ dst, const double *W, int ld, int n)
{
    for (int e = threadIdx.x; e < n * n; e += 64) {
        const int r = e / n, c = e - r * n;
        dst[e] = c <= r ? W[r * ld + c] : 0.0;
    }
}

// Left-looking (lazy update): column j gathers the contributions of columns 0..j-1 just
// before it is scaled (the paper's choice, Table 1). W may be LDS or global memory.
template <bool kGlobal>
MT_INLINE int chol_left(double *W, int ld, int n)
{
    const int i = threadIdx.x;
    for (int j = 0; j < n; j++) {
        double s = 0.0;
        if (i < n && i >= j) {
            const double *ri = W + i * ld, *rj = W + j * ld;
            double p[4] = {ri[j], 0.0, 0.0, 0.0};
            int k = 0;
            for (; k + 4 <= j; k += 4)
                MT_UNROLL for (int u = 0; u < 4; u++) p[u] = fma(-ri[k + u], rj[k + u], p[u]);
            for (; k < j; k++) p[0] = fma(-ri[k], rj[k], p[0]);
            s = (p[0] + p[1]) + (p[2] + p[3]);
        }
        const double d = bcast(s, j);
        if (!(d > 0.0)) return j + 1;
        const double piv = sqrt(d);
        if (i == j) W[j * ld + j] = piv;
        if (i > j && i < n) W[i * ld + j] = s / piv;
        if (kGlobal) wave_sync_global();
        else wave_sync();
    }
    return 0;
}

// Right-looking (eager update): after column j is scaled, every row below updates its
// trailing entries at once.
MT_INLINE int chol_right(double *W, int ld, int n)
{
    const int i = threadIdx.x;
    for (int j = 0; j < n; j++) {
        const double d = W[j * ld + j];  // same address in every lane: an LDS broadcast
        if (!(d > 0.0)) return j + 1;
        const double piv = sqrt(d);
        double lij = 0.0;
        if (i > j && i < n) {
            lij = W[i * ld + j] / piv;
            W[i * ld + j] = lij;
        }
        if (i == j) W[j * ld + j] = piv;
        wave_sync();
        if (i > j && i < n) {
            double *ri = W + i * ld;
            for (int k = j + 1; k <= i; k++) ri[k] = fma(-lij, W[k * ld + j], ri[k]);
        }
        wave_sync();
    }
    return 0;
}

__global__ __launch_bounds__(64) void chol_kernel(int variant, int64_t count, int n, const double *a,
                                                  double *l, int32_t *info)
{
    extern __shared__ double sm[];
    const int64_t p = blockIdx.x;
    if (p >= count) return;
    const double *A = a + p * n * n;
    double *Lp = l + p * n * n;
    int rc;
    if (variant == TRON_CHOL_BLOCKED_MFMA) {
        // the solver's layout: the matrix's upper triangle with its diagonal at row stride
        // (n + 1) | 1, the factor's strict lower triangle below it, its pivots in column n
        mt::WaveTron<mt::WaveFamQP4<1>, false> s;
        s.n = n;
        s.ld = (n + 1) | 1;
        s.lane = threadIdx.x;
        s.M = sm;
        for (int e = threadIdx.x; e < n * n; e += 64) {
            const int r = e / n, c = e - r * n;
            if (c >= r) sm[r * s.ld + c] = A[e];
        }
        wave_sync();
        const uint64_t fm[1] = {n == 64 ? ~0ull : (1ull << n) - 1ull};
        const bool ok = s.chol(fm, 0.0);
        wave_sync();
        for (int e = threadIdx.x; e < n * n; e += 64) {
            const int r = e / n, c = e - r * n;
            Lp[e] = c < r ? sm[r * s.ld + c] : (c == r ? sm[r * s.ld + n] : 0.0);
        }
        // the first pivot that is not positive: every pivot before it was
        const int i = threadIdx.x;
        const uint64_t badp = __ballot(i < n && !(sm[(i < n ? i : 0) * s.ld + n] > 0.0));
        rc = ok ? 0 : (badp ? __builtin_ctzll(badp) + 1 : 1);
    } else if (variant == TRON_CHOL_LEFT_GLOBAL) {
        stage_lower(Lp, n, A, n);
        wave_sync_global();
        rc = chol_left<true>(Lp, n, n);
        wave_sync_global();
        for (int e = threadIdx.x; e < n * n; e += 64) {
            const int r = e / n, c = e - r * n;
            if (c > r) Lp[e] = 0.0;
        }
    } else {
        const int ld = n | 1;
        stage_lower(sm, ld, A, n);
        wave_sync();
        rc = variant == TRON_CHOL_LEFT_LDS ? chol_left<false>(sm, ld, n) : chol_right(sm, ld, n);
        wave_sync();
        write_lower(Lp, sm, ld, n);
    }
    if (threadIdx.x == 0) info[p] = rc;
}

// Forward substitution L y = b, column by column: at step j lane j finishes y_j and every
// lane below subtracts its multiple. Lane i reads L_ij at W[i ld + j] (a column walk), or,
// with lt, L^T's row j at W[j ld + i] (a row walk through the explicit copy).
MT_INLINE double fwd(const double *W, int ld, int n, double b, bool lt)
{
    const int i = threadIdx.x;
    for (int j = 0; j < n; j++) {
        const double yj = bcast(i == j ? b / W[j * ld + j] : 0.0, j);
        if (i == j) b = yj;
        if (i > j && i < n) b = fma(-(lt ? W[j * ld + i] : W[i * ld + j]), yj, b);
    }
    return b;
}

// Backward substitution L^T x = y: at step j lane j finishes x_j and every lane above
// subtracts L_ji x_j, reading row j of L (W[j ld + i]).
MT_INLINE double bwd(const double *W, int ld, int n, double y)
{
    const int i = threadIdx.x;
    for (int j = n - 1; j >= 0; j--) {
        const double xj = bcast(i == j ? y / W[j * ld + j] : 0.0, j);
        if (i == j) y = xj;
        if (i < j) y = fma(-W[j * ld + i], xj, y);
    }
    return y;
}

__global__ __launch_bounds__(64) void trsv_kernel(int variant, int64_t count, int n, const double *l,
                                                  const double *b, double *x, int reps)
{
    extern __shared__ double sm[];
    const int64_t p = blockIdx.x;
    if (p >= count) return;
    const int i = threadIdx.x;
    const double *Lp = l + p * n * n;
    const double bi = i < n ? b[p * n + i] : 0.0;
    const double *W = sm;
    int ld = n;
    bool lt = false;
    if (variant == TRON_TRSV_GLOBAL) {
        W = Lp;
    } else {
        ld = variant == TRON_TRSV_PADDED ? (n | 1) : n;
        stage_lower(sm, ld, Lp, n);
        wave_sync();
        if (variant == TRON_TRSV_EXPLICIT) {
            // L^T into the strict upper triangle: element (j, i) above the diagonal = L_ij
            for (int e = threadIdx.x; e < n * n; e += 64) {
                const int r = e / n, c = e - r * n;
                if (c > r) sm[r * ld + c] = sm[c * ld + r];
            }
            wave_sync();
            lt = true;
        }
    }
    double out = 0.0;
    for (int rep = 0; rep < reps; rep++) {
        out = bwd(W, ld, n, fwd(W, ld, n, bi, lt));
        wave_sync();  // keeps the repetitions from being merged
    }
    if (i < n) x[p * n + i] = out;
}

// Eight independent FMA chains per lane: enough independent work per wave to cover the
// FP64 pipeline's latency, so that the launch measures issue rate, not dependency stalls.
__global__ __launch_bounds__(256) void fma_peak_kernel(int32_t iters, double a, double b, double *sink)
{
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double x[8];
    MT_UNROLL for (int c = 0; c < 8; c++) x[c] = 1.0 + (double)(c + (int)(t & 7) + 1) * 0x1p-10;
    for (int k = 0; k < iters; k++) {
        MT_UNROLL for (int c = 0; c < 8; c++) x[c] = fma(x[c], a, b);
    }
    double s = 0.0;
    MT_UNROLL for (int c = 0; c < 8; c++) s += x[c];
    sink[t] = s;
}

}  // namespace

extern "C" tron_err tron_design_fma_peak(int64_t blocks, int32_t iters, double *d_sink, void *stream)
{
    if (!d_sink || blocks < 1 || blocks > INT32_MAX || iters < 1)
        return mt_fail(TRON_ERR_INVALID, "invalid FMA-rate benchmark arguments");
    hipLaunchKernelGGL(fma_peak_kernel, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (int)iters,
                       1.0 - 0x1p-20, 0x1p-20, d_sink);
    HIP_TRY(hipGetLastError());
    return TRON_OK;
}

extern "C" tron_err tron_design_chol(int32_t variant, int64_t count, int32_t n, const double *d_a,
                                     double *d_l, int32_t *d_info, void *stream)
{
    if (variant < TRON_CHOL_LEFT_LDS || variant > TRON_CHOL_BLOCKED_MFMA || count < 0 || n < 1 || n > 64)
        return mt_fail(TRON_ERR_INVALID, "invalid Cholesky benchmark arguments");
    if (count == 0) return TRON_OK;
    if (!d_a || !d_l || !d_info) return mt_fail(TRON_ERR_INVALID, "null device pointer");
    const size_t stride = variant == TRON_CHOL_BLOCKED_MFMA ? (size_t)((n + 1) | 1) : (size_t)(n | 1);
    const size_t lds = variant == TRON_CHOL_LEFT_GLOBAL ? 0 : sizeof(double) * (size_t)n * stride;
    hipLaunchKernelGGL(chol_kernel, dim3((unsigned)count), dim3(64), lds, (hipStream_t)stream, (int)variant,
                       count, (int)n, d_a, d_l, d_info);
    HIP_TRY(hipGetLastError());
    return TRON_OK;
}

extern "C" tron_err tron_design_trsv(int32_t variant, int64_t count, int32_t n, const double *d_l,
                                     const double *d_b, double *d_x, int32_t reps, void *stream)
{
    if (variant < TRON_TRSV_IMPLICIT || variant > TRON_TRSV_GLOBAL || count < 0 || n < 1 || n > 64 || reps < 1)
        return mt_fail(TRON_ERR_INVALID, "invalid triangular-solve benchmark arguments");
    if (count == 0) return TRON_OK;
    if (!d_l || !d_b || !d_x) return mt_fail(TRON_ERR_INVALID, "null device pointer");
    const int ld = variant == TRON_TRSV_PADDED ? (n | 1) : n;
    const size_t lds = variant == TRON_TRSV_GLOBAL ? 0 : sizeof(double) * (size_t)n * (size_t)ld;
    hipLaunchKernelGGL(trsv_kernel, dim3((unsigned)count), dim3(64), lds, (hipStream_t)stream, (int)variant,
                       count, (int)n, d_l, d_b, d_x, (int)reps);
    HIP_TRY(hipGetLastError());
    return TRON_OK;
}
