"""Pins of the oracle's core operations (figure "Core operations") against library
routines, closed forms and hand-worked cases."""
import math

import numpy as np
import pytest
import scipy.linalg as sla

INF = math.inf


def spd(rng, m, shift=0.5):
    a = rng.standard_normal((m, m))
    return a @ a.T + shift * np.eye(m)


@pytest.mark.parametrize("m", [1, 2, 5, 8, 17, 33])
def test_ccf_matches_numpy_cholesky(orc, m):
    rng = np.random.default_rng(m)
    a = spd(rng, m)
    rc, l = orc.ccf(a, 0.0)
    assert rc == 0
    ref = np.linalg.cholesky(a)
    assert np.allclose(l, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    assert np.all(np.triu(l, 1) == 0.0)
    # with a shift: L L^T = A + alpha I (ccfs then ccf)
    rc, l2 = orc.ccf(a, 0.75)
    assert rc == 0
    assert np.linalg.norm(l2 @ l2.T - (a + 0.75 * np.eye(m))) <= 1e-13 * np.linalg.norm(a) * m


def test_ccf_reports_first_bad_pivot(orc):
    # leading 2x2 block positive definite, 3x3 indefinite: pivot of column 3 fails
    a = np.array([[4.0, 2.0, 0.0], [2.0, 5.0, 3.0], [0.0, 3.0, 1.0]])
    rc, _ = orc.ccf(a, 0.0)
    assert rc == 3
    # a zero pivot counts as failure
    rc, _ = orc.ccf(np.zeros((2, 2)), 0.0)
    assert rc == 1
    # the shift makes it succeed
    rc, l = orc.ccf(a, 3.0)
    assert rc == 0 and np.allclose(l @ l.T, a + 3.0 * np.eye(3))


@pytest.mark.parametrize("m", [1, 3, 8, 20])
def test_trsv_matches_scipy(orc, m):
    rng = np.random.default_rng(100 + m)
    l = np.tril(rng.standard_normal((m, m))) + 3.0 * np.eye(m)
    b = rng.standard_normal(m)
    y = orc.trsv_lower(l, b)
    assert np.allclose(y, sla.solve_triangular(l, b, lower=True), rtol=1e-13, atol=1e-13)
    z = orc.trsv_lower_t(l, b)
    assert np.allclose(z, sla.solve_triangular(l, b, lower=True, trans="T"), rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("seed", range(6))
def test_trqsol_hits_radius(orc, seed):
    rng = np.random.default_rng(seed)
    m = 5
    p = rng.standard_normal(m)
    x = rng.standard_normal(m)
    x *= 0.3 / np.linalg.norm(x)
    if seed % 2:
        p = -np.sign(p @ x) * p if p @ x != 0 else p  # make p'x < 0 on odd seeds
    delta = 1.7
    sig = orc.trqsol(x, p, delta)
    assert sig >= 0
    assert abs(np.linalg.norm(x + sig * p) - delta) <= 1e-14 * delta * 10


def test_trqsol_from_origin(orc):
    p = np.array([3.0, 4.0])
    assert orc.trqsol(np.zeros(2), p, 10.0) == pytest.approx(2.0, rel=1e-15)


def test_breakpt_hand_cases(orc):
    x = np.array([0.0, 1.0, 0.5, 0.0, 0.0])
    lo = np.array([-1.0, 0.0, -INF, -2.0, 0.0])
    hi = np.array([2.0, 3.0, INF, 2.0, 1.0])
    w = np.array([1.0, -0.5, 1.0, 0.0, -1.0])
    # i0: (2-0)/1 = 2 ; i1: (0-1)/-0.5 = 2 ; i2: no bound ; i3: w = 0 ; i4: (0-0)/-1 = 0
    nb, bmin, bmax = orc.breakpt(x, lo, hi, w)
    assert nb == 3 and bmin == 0.0 and bmax == 2.0
    nb, bmin, bmax = orc.breakpt(x[2:4], lo[2:4], hi[2:4], w[2:4])
    assert nb == 0 and bmax == INF


def test_gpstep_hand_cases(orc):
    x = np.array([0.0, 1.0, 0.5, -1.0])
    lo = np.array([-1.0, 0.0, -INF, -1.0])
    hi = np.array([2.0, 3.0, INF, 1.0])
    w = np.array([4.0, -4.0, 10.0, -1.0])
    s = orc.gpstep(x, lo, hi, 0.5, w)  # P(x + w/2) - x
    assert np.array_equal(s, np.array([2.0, -1.0, 5.0, 0.0]))


def test_projgrad_definition(orc):
    lo = np.array([0.0, 0.0, 0.0, 0.0, 0.0, 1.0])
    hi = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0])
    x = np.array([0.0, 0.0, 1.0, 1.0, 0.5, 1.0])
    g = np.array([2.0, -3.0, -4.0, 5.0, -0.5, 9.0])
    # at lower: only negative g counts; at upper: only positive; fixed: 0
    assert orc.projgrad_inf(x, lo, hi, g) == 5.0
    g2 = np.array([2.0, -0.25, -4.0, 0.1, -0.5, 9.0])
    assert orc.projgrad_inf(x, lo, hi, g2) == 0.5


@pytest.mark.parametrize("m", [1, 4, 7])
def test_cg_spd_one_iteration_newton(orc, m):
    """With A positive definite the shift is 0, L L^T = A, the preconditioned matrix is the
    identity and CG ends after one iteration at the Newton step (section 4.3)."""
    rng = np.random.default_rng(7 * m)
    a = spd(rng, m)
    r = rng.standard_normal(m)
    res = orc.subspace_cg(a, r, delta=1e6, cg_rtol=0.1)
    assert res["shift"] == 0.0
    assert res["iters"] == 1
    assert res["exit"] == 0
    assert np.allclose(res["w"], -np.linalg.solve(a, r), rtol=1e-10, atol=1e-12)


def test_cg_boundary_and_cap(orc):
    rng = np.random.default_rng(3)
    a = spd(rng, 6)
    r = 100.0 * rng.standard_normal(6)
    res = orc.subspace_cg(a, r, delta=1e-3)
    assert res["exit"] == 3
    assert abs(np.linalg.norm(res["shat"]) - 1e-3) <= 1e-15
    assert res["iters"] <= 6


def test_cg_indefinite_shift_and_curvature(orc):
    """Indefinite A: a positive shift is used, CG takes at most |F| iterations and ends on
    negative curvature or at the trust boundary with ||s_hat|| = delta."""
    rng = np.random.default_rng(11)
    q, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    a = q @ np.diag([-3.0, -1.0, 0.5, 1.0, 2.0, 4.0]) @ q.T
    r = rng.standard_normal(6)
    res = orc.subspace_cg(a, r, delta=0.7)
    assert res["shift"] > 0.0
    assert res["iters"] <= 6
    assert res["exit"] in (2, 3)
    assert abs(np.linalg.norm(res["shat"]) - 0.7) <= 1e-14
    # the step is a descent direction of the model r's + s'As/2
    w = res["w"]
    assert r @ w + 0.5 * w @ a @ w < 0
