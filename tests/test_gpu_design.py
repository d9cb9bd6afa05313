"""GPU tests of the kernel-design variants (include/tron_design.h): every Cholesky variant
against the oracle's left-looking factorisation, every triangular-solve variant against the
oracle's substitutions, failure reporting on indefinite blocks, and repetition invariance.

Tolerances: the blocks are A = M'M + n I (condition number below ~5), so the factor and the
solution are determined to a few units of rounding; different summation orders (the oracle
sums left to right without FMA, the kernels in partial sums with FMA or in the matrix
cores' 16 x 16 x 4 products) then differ by at most ~n eps relative. The bar is 1e-12 relative, with the residual ||L L' - A|| below
1e-13 ||A||."""
import numpy as np
import pytest

import oracle
from paper_2106_14995_amd import workloads as W

pytestmark = pytest.mark.gpu
SIZES = [1, 2, 3, 7, 8, 15, 16, 17, 31, 32, 33, 47, 48, 49, 63, 64]


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_2106_14995_amd import tron
    tron.lib()
    return tron


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("n", SIZES)
def test_cholesky_variants_match_the_oracle(T, n):
    import torch
    A, _ = W.spd_blocks(200, n)
    ref = np.zeros_like(A)
    for p in range(A.shape[0]):
        rc, ref[p] = oracle.ccf(A[p])
        assert rc == 0
    for variant in (T.CHOL_LEFT_LDS, T.CHOL_RIGHT_LDS, T.CHOL_LEFT_GLOBAL, T.CHOL_BLOCKED_MFMA):
        L, info = T.design_chol(variant, dev(A))
        torch.cuda.synchronize()
        L, info = L.cpu().numpy(), info.cpu().numpy()
        assert np.all(info == 0), variant
        assert np.all(np.triu(L, 1) == 0.0), variant
        scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
        assert np.abs(L - ref).max() <= 1e-12 * scale.max(), (variant, np.abs(L - ref).max())
        res = np.abs(L @ np.transpose(L, (0, 2, 1)) - A).max(axis=(1, 2))
        assert np.all(res <= 1e-13 * np.abs(A).max(axis=(1, 2))), variant


@pytest.mark.parametrize("n", [4, 9, 32])
def test_cholesky_reports_the_failing_pivot(T, n):
    import torch
    A, _ = W.spd_blocks(40, n, config_id=81)
    rng = np.random.default_rng(2)
    for p in range(A.shape[0]):
        j = int(rng.integers(0, n))
        A[p, j, j] = -1.0 - A[p, j, j]       # column j's pivot becomes negative
    want = [oracle.ccf(A[p])[0] for p in range(A.shape[0])]
    for variant in (T.CHOL_LEFT_LDS, T.CHOL_RIGHT_LDS, T.CHOL_LEFT_GLOBAL, T.CHOL_BLOCKED_MFMA):
        _, info = T.design_chol(variant, dev(A))
        torch.cuda.synchronize()
        assert list(info.cpu().numpy()) == want, variant


@pytest.mark.parametrize("n", SIZES)
def test_triangular_solve_variants_match_the_oracle(T, n):
    import torch
    A, B = W.spd_blocks(200, n, config_id=82)
    Ls = np.linalg.cholesky(A)
    ref = np.array([oracle.trsv_lower_t(Ls[p], oracle.trsv_lower(Ls[p], B[p])) for p in range(A.shape[0])])
    Ld, Bd = dev(Ls), dev(B)
    for variant in (T.TRSV_IMPLICIT, T.TRSV_PADDED, T.TRSV_EXPLICIT, T.TRSV_GLOBAL):
        x = T.design_trsv(variant, Ld, Bd)
        x4 = T.design_trsv(variant, Ld, Bd, reps=4)
        torch.cuda.synchronize()
        x, x4 = x.cpu().numpy(), x4.cpu().numpy()
        assert np.array_equal(x, x4), variant
        err = np.abs(x - ref).max(axis=1) / np.maximum(np.abs(ref).max(axis=1), 1e-300)
        assert err.max() <= 1e-12, (variant, err.max())


def test_fma_rate_kernel_computes_its_chains(T):
    """The FP64 FMA-rate kernel (the measured reference of the roofline) does the work it is
    charged for: each lane's sum of its 8 chains x <- x a + b, a = 1 - 2^-20, b = 2^-20, from
    x0 = 1 + (c + lane mod 8 + 1) 2^-10, equals the closed form 8 + 2^-10 a^k sum_c (c + lane
    mod 8 + 1) after k steps (the fixed point is exactly 1), to the rounding of k FMAs."""
    import torch
    blocks, iters = 3, 1000
    s = T.design_fma_peak(blocks, iters)
    torch.cuda.synchronize()
    got = s.cpu().numpy()
    lane = np.arange(blocks * 256)
    a = 1.0 - 2.0 ** -20
    want = 8.0 + 2.0 ** -10 * a ** iters * np.array([sum(c + (t % 8) + 1 for c in range(8)) for t in lane])
    assert got.shape == (blocks * 256,)
    assert np.abs(got - want).max() <= 1e-12 * 8.0
