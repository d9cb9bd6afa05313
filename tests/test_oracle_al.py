"""Pins of the oracle's augmented-Lagrangian loop (section 1: general constraints through a
sequence of bound-constrained solves) on branch subproblems with line limits (family BR8L):
finite-difference derivatives, the reduction to BR6 without the limit terms, the limit terms
rebuilt from the complex-power form of the flows, the BR6 solution when no limit binds, an
independent SQP solve (SciPy's SLSQP) of the constrained problem when limits bind, and the
sign and complementarity of the final multipliers."""
import numpy as np
import pytest

from paper_2106_14995_amd import workloads as W

BR6, BR8L = W.BR6, W.BR8L


def fd_grad(f, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x); e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


def inside(rng, lo, hi):
    return lo + (hi - lo) * rng.uniform(0.2, 0.8, lo.size)


def limit_terms(p, x):
    """h_lm = |S_lm|^2 + sigma_lm - smax^2 from the complex-power flows."""
    pq = W.complex_flows(p[0], p[1], x[0], x[1], x[2], x[3])
    return np.array([pq[0] ** 2 + pq[1] ** 2 + x[6] - p[36], pq[2] ** 2 + pq[3] ** 2 + x[7] - p[36]])


def test_br8l_derivatives_match_finite_differences(orc):
    bt = W.br8l_batch(12, config_id=50)
    rng = np.random.default_rng(3)
    for b in range(bt.batch):
        n, p, lo, hi, _ = bt.instance(b)
        p = p.copy()
        p[37:39] = rng.standard_normal(2)  # non-zero multipliers
        x = inside(rng, lo, np.minimum(hi, lo + 1.0))
        g = orc.eval_g(BR8L, 8, p, x)
        gfd = fd_grad(lambda v: orc.eval_f(BR8L, 8, p, v), x)
        assert np.allclose(g, gfd, rtol=1e-6, atol=1e-5 * max(1.0, np.abs(g).max()))
        H = orc.eval_h(BR8L, 8, p, x)
        Hfd = np.array([fd_grad(lambda v: orc.eval_g(BR8L, 8, p, v)[i], x) for i in range(8)])
        assert np.allclose(H, H.T, rtol=0, atol=1e-9 * max(1.0, np.abs(H).max()))
        assert np.allclose(H, Hfd, rtol=1e-5, atol=1e-5 * max(1.0, np.abs(H).max()))


def test_br8l_without_limit_terms_is_br6(orc):
    bt = W.br8l_batch(8, config_id=51)
    rng = np.random.default_rng(4)
    for b in range(bt.batch):
        _, p, lo, hi, _ = bt.instance(b)
        p = p.copy()
        p[37:40] = 0.0
        x = inside(rng, lo, np.minimum(hi, lo + 1.0))
        assert orc.eval_f(BR8L, 8, p, x) == orc.eval_f(BR6, 6, p[:36], x[:6])
        g8, g6 = orc.eval_g(BR8L, 8, p, x), orc.eval_g(BR6, 6, p[:36], x[:6])
        assert np.array_equal(g8[:6], g6) and np.all(g8[6:] == 0.0)
        H8, H6 = orc.eval_h(BR8L, 8, p, x), orc.eval_h(BR6, 6, p[:36], x[:6])
        assert np.array_equal(H8[:6, :6], H6) and np.all(H8[6:, :] == 0.0)


def test_br8l_limit_terms_from_complex_power(orc):
    bt = W.br8l_batch(20, config_id=52)
    rng = np.random.default_rng(5)
    for b in range(bt.batch):
        _, p, lo, hi, _ = bt.instance(b)
        p = p.copy()
        p[37:39] = rng.standard_normal(2)
        p[39] = rng.uniform(0.5, 50.0)
        x = inside(rng, lo, np.minimum(hi, lo + 1.0))
        h = limit_terms(p, x)
        extra = float(np.sum(p[37:39] * h + 0.5 * p[39] * h * h))
        diff = orc.eval_f(BR8L, 8, p, x) - orc.eval_f(BR6, 6, p[:36], x[:6])
        assert diff == pytest.approx(extra, rel=1e-10, abs=1e-9)


def test_al_with_loose_limits_returns_the_br6_solution(orc):
    """With every limit far above the flows the slacks absorb h = 0, so the first
    bound-constrained solve is the BR6 problem: one outer iteration, the BR6 minimiser."""
    bt = W.br8l_batch(60, config_id=53)
    po = bt.poff()
    vo = bt.voff()
    for b in range(bt.batch):
        smax2 = 100.0 * bt.params[po[b] + 36]
        bt.params[po[b] + 36] = smax2
        bt.hi[vo[b] + 6:vo[b] + 8] = smax2
        _, p, _, _, x0 = bt.instance(b)
        pq = W.complex_flows(p[0], p[1], x0[0], x0[1], x0[2], x0[3])
        bt.x0[vo[b] + 6] = smax2 - (pq[0] ** 2 + pq[1] ** 2)
        bt.x0[vo[b] + 7] = smax2 - (pq[2] ** 2 + pq[3] ** 2)
    # (gtol 1e-8: with smax^2 in the thousands, h rounds at ~1e-13 and the limit terms put
    # gradient noise of ~1e-9 on the angles)
    r = orc.al_solve(bt, ctol=1e-8, gtol=1e-8)
    assert np.all(r["status"] == 0) and np.all(r["outer"] == 1)
    six = W.Batch(BR6, np.full(bt.batch, 6, dtype=np.int32),
                  np.concatenate([bt.params[po[b]:po[b] + 36] for b in range(bt.batch)]),
                  bt.lo.reshape(-1, 8)[:, :6].ravel(), bt.hi.reshape(-1, 8)[:, :6].ravel(),
                  bt.x0.reshape(-1, 8)[:, :6].ravel())
    r6 = orc.solve(six, gtol=1e-9)
    assert np.all(r6["status"] == 0)
    x8 = r["x"].reshape(-1, 8)
    assert np.abs(x8[:, :6] - r6["x"].reshape(-1, 6)).max() <= 1e-5
    for b in range(bt.batch):
        f6 = orc.eval_f(BR6, 6, six.params[36 * b:36 * b + 36], x8[b, :6])
        assert f6 == pytest.approx(r6["f"][b], rel=1e-10, abs=1e-10)


def test_al_matches_an_sqp_solve_when_limits_bind(orc):
    """Binding limits: the AL result against SciPy's SLSQP on min f_BR6 subject to
    |S_ij|^2, |S_ji|^2 <= smax^2 and the BR6 bounds, from the same start."""
    from scipy.optimize import minimize
    bt = W.br8l_batch(160, config_id=54)
    r = orc.al_solve(bt, ctol=1e-8, gtol=1e-7)
    assert np.mean(r["status"] == 0) >= 0.95
    x8 = r["x"].reshape(-1, 8)
    binding = np.where((x8[:, 6:] <= 1e-12).any(axis=1) & (r["status"] == 0))[0]
    assert binding.size >= 30
    checked = 0
    for b in binding[:40]:
        _, p, lo, hi, x0 = bt.instance(b)
        p6 = p[:36]
        cons = [{"type": "ineq", "fun": (lambda v, k=k: p[36] - (W.complex_flows(p[0], p[1], *v[:4])[2 * k] ** 2 +
                                                                   W.complex_flows(p[0], p[1], *v[:4])[2 * k + 1] ** 2))}
                for k in range(2)]
        res = minimize(lambda v: orc.eval_f(BR6, 6, p6, v), x0[:6], jac=lambda v: orc.eval_g(BR6, 6, p6, v),
                       bounds=list(zip(lo[:6], hi[:6])), constraints=cons, method="SLSQP",
                       options={"ftol": 1e-12, "maxiter": 500})
        if not res.success:
            continue
        f_al = orc.eval_f(BR6, 6, p6, x8[b, :6])
        assert f_al == pytest.approx(res.fun, rel=1e-6, abs=1e-6), b
        assert np.abs(x8[b, :6] - res.x).max() <= 1e-5, b
        checked += 1
    assert checked >= 20


def test_al_multipliers_sign_and_complementarity(orc):
    """At the end: |h| <= ctol; a limit with a positive slack has a multiplier estimate
    lambda + rho h near 0 (the slack's gradient vanishes inside its bounds); a binding limit
    (slack 0) has a non-negative estimate."""
    bt = W.br8l_batch(300, config_id=55)
    ctol, gtol = 1e-7, 1e-7
    r = orc.al_solve(bt, ctol=ctol, gtol=gtol)
    ok = r["status"] == 0
    assert np.mean(ok) >= 0.98
    assert r["viol"][ok].max() <= ctol
    p = r["params"].reshape(-1, 40)
    x = r["x"].reshape(-1, 8)
    for b in np.where(ok)[0]:
        h = limit_terms(p[b], x[b])
        assert np.abs(h).max() <= 1.01 * ctol
        est = p[b, 37:39] + p[b, 39] * h
        for k in range(2):
            if x[b, 6 + k] > 1e-10:
                assert abs(est[k]) <= gtol * 1.01
            else:
                assert est[k] >= -gtol * 1.01
    # some limits bind and carry a clearly positive price
    assert np.sum(p[:, 37:39] > 1e-3) >= 30
