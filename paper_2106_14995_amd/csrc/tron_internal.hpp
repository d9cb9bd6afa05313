// tron_internal.hpp -- declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lane_tron.hpp"
#include "tron.h"

// Arguments of the lane-per-instance solve kernels.
struct LaneArgs {
    const double *params, *lo, *hi, *x0;
    double *x, *f;
    int32_t *status, *iters;
    double *state;           // radius [batch], Cauchy step [batch]
    const int32_t *index;    // instance list of this bucket, or null (all, in order)
    const int32_t *nper;     // per-instance n, or null (n_uniform)
    const int64_t *poff, *voff;
    int64_t *ts;             // optional: per-instance start / end device clock (2 per instance)
    int64_t count, batch;
    int32_t n_uniform, psize;
    int32_t lane_block;      // workgroup size of the lane kernels (64 or 256; 0 means 256)
    mt::Options opt;
    double *ws;              // n > 128: per-instance matrix workspace in global memory
    int64_t ws_stride;       // doubles per instance in ws (bucket slot t uses ws + t stride)
};

// Largest n of any family with a wave kernel; n in (kLdsMaxN, kMaxN] keeps its matrices in a
// global-memory workspace instead of LDS.
constexpr int kLdsMaxN = 128;
constexpr int kMaxN = 512;
// doubles of one instance's matrix array for bucket size nmax (n rows, odd stride > n)
__host__ __device__ inline int64_t mt_wave_matrix_doubles(int nmax) { return (int64_t)nmax * (int64_t)((nmax + 1) | 1); }

typedef void (*lane_launch_fn)(const LaneArgs &, hipStream_t);

// Launch the BR6 lane kernel (n = 6) over a.count instances.
void mt_launch_br6(const LaneArgs &a, hipStream_t st);
// Let the BR6 lane kernel take the LDS of its largest workgroup (once per process and device).
void mt_prepare_br6();
// The lane kernel for (family, N <= 8), or null when unsupported.
lane_launch_fn mt_lane_launcher(tron_family fam, int N);
// The wavefront-per-instance kernel of the family (QP4 or HS45M) for instances with
// n <= nmax (nmax <= kLdsMaxN: LDS sized for nmax; larger nmax: a.ws must hold a.count
// slots of a.ws_stride >= mt_wave_matrix_doubles(nmax) doubles).
void mt_launch_wave(tron_family fam, const LaneArgs &a, int nmax, hipStream_t st);
// LDS bytes the wave kernel uses for one instance of size n (its bucket's footprint).
size_t mt_wave_lds_bytes(int nmax);
// Make the wave kernels and the BR6 lane kernel accept their largest LDS request (once per
// process and device).
void mt_prepare_wave_kernels();

// Record an error message for tron_last_error() and return `code`.
tron_err mt_fail(tron_err code, const char *fmt, ...);

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return mt_fail(TRON_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));   \
    } while (0)

// The group-solver kernel for (family, N, G): one instance per G lanes, n <= N; null when
// that build does not exist (group.hip).
lane_launch_fn mt_group_launcher(tron_family fam, int N, int G);
