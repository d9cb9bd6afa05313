"""Pins of the oracle's problem families: the branch flows against the complex-power form
of the same physics, special cases of the augmented-Lagrangian objective, identities of the
quartic family, and finite-difference derivatives of all families."""
import math

import numpy as np
import pytest

from paper_2106_14995_amd import workloads as W


def fd_grad(f, x, h=1e-6):
    g = np.zeros_like(x)
    for i in range(x.size):
        e = np.zeros_like(x); e[i] = h
        g[i] = (f(x + e) - f(x - e)) / (2 * h)
    return g


def fd_hess(gfun, x, h=1e-6):
    n = x.size
    H = np.zeros((n, n))
    for i in range(n):
        e = np.zeros_like(x); e[i] = h
        H[:, i] = (gfun(x + e) - gfun(x - e)) / (2 * h)
    return H


def test_br6_flows_match_complex_power(orc):
    rng = np.random.default_rng(5)
    for _ in range(50):
        g, b = rng.uniform(0.5, 5), rng.uniform(-20, -1)
        x = np.array([rng.uniform(0.9, 1.1), rng.uniform(0.9, 1.1), rng.uniform(-3, 3),
                      rng.uniform(-3, 3), 0.0, 0.0])
        p = np.zeros(36)
        p[:8] = [g, b, g, b, g, b, g, b]
        got = orc.br6_flows(p, x)
        ref = W.complex_flows(g, b, x[0], x[1], x[2], x[3])
        assert np.allclose(got, ref, rtol=1e-12, atol=1e-12)
        # physics: the real and reactive losses are g |V_i - V_j|^2 and b |V_i - V_j|^2
        dv = abs(x[0] * np.exp(1j * x[2]) - x[1] * np.exp(1j * x[3])) ** 2
        assert got[0] + got[2] == pytest.approx(g * dv, abs=1e-11)
        assert got[1] + got[3] == pytest.approx(b * dv, abs=1e-11)


def test_br6_flows_each_admittance_slot(orc):
    """Each of the eight admittance slots enters the flow it belongs to (eqs. pij..qji)."""
    x = np.array([1.03, 0.97, 0.3, -0.1, 0.0, 0.0])
    vi, vj, d = x[0], x[1], x[2] - x[3]
    V, c, s = vi * vj, math.cos(d), math.sin(d)
    expect = {  # slot -> (flow index, derivative of that flow w.r.t. the slot)
        0: (0, -V * c), 1: (0, V * s), 2: (0, vi * vi),
        4: (2, -V * c), 5: (2, -V * s), 6: (2, vj * vj),
    }
    for slot, (k, dval) in expect.items():
        p = np.zeros(36); p[slot] = 1.0
        assert orc.br6_flows(p, x)[k] == pytest.approx(dval, abs=1e-14)
    # reactive flows: slots 1 (b_ij), 3 (bc_ij), 0 (g_ij) in q_ij; 5, 7, 4 in q_ji
    for slot, k, dval in [(1, 1, -V * c), (3, 1, vi * vi), (0, 1, -V * s),
                          (5, 3, -V * c), (7, 3, vj * vj), (4, 3, V * s)]:
        p = np.zeros(36); p[slot] = 1.0
        assert orc.br6_flows(p, x)[k] == pytest.approx(dval, abs=1e-14)


def test_br6_objective_special_cases(orc):
    """With every penalty 0 and one multiplier 1 the objective is that coupling's residual;
    with one penalty 2 and no multipliers it is the squared residual (eq. exp-branch)."""
    rng = np.random.default_rng(9)
    g, b = 2.0, -7.0
    x = np.array([1.02, 0.98, 0.15, -0.05, 0.4, -0.3])
    flows = W.complex_flows(g, b, x[0], x[1], x[2], x[3])
    y = np.array([*flows, x[0] ** 2, x[1] ** 2, x[2], x[3]])
    t = rng.standard_normal(8)
    base = np.zeros(36)
    base[:8] = [g, b, g, b, g, b, g, b]
    base[8:16] = t
    for k in range(8):
        p = base.copy(); p[16 + k] = 1.0
        assert orc.eval_f(1, 6, p, x) == pytest.approx(y[k] - t[k], abs=1e-12)
        p = base.copy(); p[26 + k] = 2.0
        assert orc.eval_f(1, 6, p, x) == pytest.approx((y[k] - t[k]) ** 2, abs=1e-12)
    for s, (zi, fk) in enumerate([(4, 0), (5, 2)]):
        p = base.copy(); p[24 + s] = 1.0
        assert orc.eval_f(1, 6, p, x) == pytest.approx(x[zi] - flows[fk], abs=1e-12)
        p = base.copy(); p[34 + s] = 2.0
        assert orc.eval_f(1, 6, p, x) == pytest.approx((x[zi] - flows[fk]) ** 2, abs=1e-12)


def test_qp4_identities(orc):
    """f(0) = 0, f(e_i) = Q_ii/2 + c_i + kappa, and the mixed difference
    f(e_i+e_j) - f(e_i) - f(e_j) + f(0) = Q_ij (the quartic is separable)."""
    n = 5
    bt = W.qp4_batch(1, n, config_id=50)
    _, p, _, _, _ = bt.instance(0)
    rng = np.random.default_rng(0)
    a = rng.standard_normal((n, n))
    Q = a.T @ a + 0.1 * np.eye(n)
    c = rng.standard_normal(n)
    kap = 0.37
    p = np.concatenate([Q[np.tril_indices(n)], c, [kap]])
    f = lambda x: orc.eval_f(0, n, p, x)
    assert f(np.zeros(n)) == 0.0
    E = np.eye(n)
    for i in range(n):
        assert f(E[i]) == pytest.approx(0.5 * Q[i, i] + c[i] + kap, rel=1e-14)
        for j in range(n):
            if i != j:
                mixed = f(E[i] + E[j]) - f(E[i]) - f(E[j]) + f(np.zeros(n))
                assert mixed == pytest.approx(Q[i, j], abs=1e-12)


@pytest.mark.parametrize("family,n", [(0, 8), (0, 3), (1, 6), (2, 5)])
def test_derivatives_finite_differences(orc, family, n):
    rng = np.random.default_rng(family * 10 + n)
    if family == 0:
        bt = W.qp4_batch(3, n, config_id=51)
    elif family == 1:
        bt = W.br6_batch(3, config_id=52)
    else:
        bt = W.hs45m_batch(3, n)
    for b in range(3):
        _, p, lo, hi, x0 = bt.instance(b)
        x = np.clip(x0 + 0.05 * rng.standard_normal(n), lo, hi)
        f = lambda z: orc.eval_f(family, n, p, z)
        gf = lambda z: orc.eval_g(family, n, p, z)
        g = gf(x)
        gfd = fd_grad(f, x)
        scale = max(1.0, np.abs(g).max())
        assert np.abs(g - gfd).max() <= 1e-6 * scale
        H = orc.eval_h(family, n, p, x)
        assert np.allclose(H, H.T, atol=1e-10 * max(1.0, np.abs(H).max()))
        Hfd = fd_hess(gf, x)
        assert np.abs(H - Hfd).max() <= 1e-6 * max(1.0, np.abs(H).max())


def test_hs45m_values(orc):
    n = 4
    x = np.array([1.0, 2.0, 3.0, 4.0])
    assert orc.eval_f(2, n, np.zeros(0), x) == 120.0 - 24.0
    g = orc.eval_g(2, n, np.zeros(0), x)
    assert np.allclose(g, -24.0 / x)
