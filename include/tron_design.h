/*
 * tron_design.h -- batched building blocks of the trust-region solver in the alternative
 * forms the paper compares when it designs its kernels (section 4: Table 1, left- against
 * right-looking Cholesky; Table 2, the backward substitution with L^T read in place against
 * an explicit copy; Table 3, workspace in on-chip shared memory against global memory).
 * They exist to measure those choices on gfx950, where the trade-offs differ, and to feed
 * the layout the solver kernels use; the solver itself does not call them.
 *
 * Every call works on `count` independent problems of the same size n (1 <= n <= 64), one
 * 64-lane wavefront per problem, lane i owning row i. Matrices are dense, row-major, n x n
 * per problem, packed back to back; vectors are n doubles per problem. All pointers are
 * caller-owned device memory; calls are asynchronous on `stream` (a hipStream_t, or null)
 * and return TRON_ERR_INVALID for a null pointer, count < 0, n outside 1..64 or an unknown
 * variant, TRON_ERR_DEVICE when the launch fails, TRON_OK otherwise.
 */
#ifndef TRON_DESIGN_H
#define TRON_DESIGN_H

#include <stdint.h>

#include "tron.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Cholesky variants (section 4.3, Table 1, and the solver's own form). */
enum {
    TRON_CHOL_LEFT_LDS = 0,     /* left-looking: column j gathers the updates of columns < j */
    TRON_CHOL_RIGHT_LDS = 1,    /* right-looking: column j updates the trailing submatrix    */
    TRON_CHOL_LEFT_GLOBAL = 2,  /* left-looking, working in global memory (no LDS)          */
    TRON_CHOL_BLOCKED_MFMA = 3  /* the solver's factorisation: 16-column panels, each formed
                                   by FP64 matrix-core products from the columns before it
                                   and factored in registers (LDS, the solver's layout)      */
};

/* A = L L^T for each SPD block of d_a (read only). d_l receives L (lower triangle with the
 * diagonal; the strict upper triangle is zeroed). d_info[p] = 0, or j + 1 when pivot j of
 * problem p is not positive or not a number (then L holds the columns before j; with
 * TRON_CHOL_BLOCKED_MFMA only those before j's panel of 16 are meaningful). The LDS
 * variants stage the matrix with an odd row stride (n | 1, and (n + 1) | 1 for the blocked
 * variant, whose spare column n holds the pivots). */
tron_err tron_design_chol(int32_t variant, int64_t count, int32_t n, const double *d_a,
                          double *d_l, int32_t *d_info, void *stream);

/* Triangular-solve variants (section 4.4, Table 2). */
enum {
    TRON_TRSV_IMPLICIT = 0,    /* L in LDS with row stride n; L^T read in place              */
    TRON_TRSV_PADDED = 1,      /* L in LDS with odd row stride n | 1; L^T read in place      */
    TRON_TRSV_EXPLICIT = 2,    /* L^T also written into the upper triangle (stride n)        */
    TRON_TRSV_GLOBAL = 3       /* L read from global memory                                 */
};

/* Solve L L^T x = b for each problem, as the conjugate-gradient step uses the factor: the
 * forward substitution L y = b, then the backward substitution L^T x = y. d_l holds L
 * (lower triangle read; the diagonal must be non-zero), d_b the right-hand sides; d_x
 * receives x (it may equal d_b). `reps` > 1 repeats the pair of solves on the same data
 * inside the kernel (x is re-solved from b each time) so that the solves outweigh the load
 * of L; results are those of one solve. */
tron_err tron_design_trsv(int32_t variant, int64_t count, int32_t n, const double *d_l,
                          const double *d_b, double *d_x, int32_t reps, void *stream);

/* Achievable FP64 vector rate on this device, the measured reference for the roofline (not a
 * step of the method). `blocks` workgroups of 256 lanes; each lane runs 8 independent chains
 * of `iters` fused multiply-adds x <- x a + b with a = 1 - 2^-20 and b = 2^-20, whose fixed
 * point is 1, from x0 = 1 + (c + (lane mod 8) + 1) 2^-10 for chain c, so every value stays
 * in [1, 2]; the lane's sum of its 8 chains goes to d_sink[global lane index] (blocks x 256
 * doubles, caller-owned device memory) so that no chain is dropped. FP64 flops issued =
 * blocks x 256 x 8 x iters x 2; the caller times the launch. Asynchronous on `stream`.
 * TRON_ERR_INVALID for a null sink, blocks < 1 or iters < 1. */
tron_err tron_design_fma_peak(int64_t blocks, int32_t iters, double *d_sink, void *stream);

#ifdef __cplusplus
}
#endif
#endif
