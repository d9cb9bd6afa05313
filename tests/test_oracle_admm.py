"""Pins of the oracle's component-ADMM updates (section "Distributed control of ACOPF"):
the generator update against a bounded 1-D minimisation, the bus update against a generic
equality-constrained least-squares KKT solve of the balance equations, and the multiplier
update as an identity."""
import numpy as np
import pytest
import scipy.optimize as so

from paper_2106_14995_amd import workloads as W


@pytest.fixture(scope="module")
def small(orc):
    net = W.network(nbus=60, nbranch=90, ngen=15, config_id=92)
    st = orc.admm_init(net)
    st, _ = orc.admm_run(net, st, 5)  # a state with nonzero multipliers and copies
    return net, st


def test_generator_update_is_bounded_minimiser(orc, small):
    net, st = small
    after, _ = orc.admm_phase(net, st, 0)
    v0, v1 = orc.admm_views(net, st), orc.admm_views(net, after)
    rho, S = net.rho, net.base_mva
    for g in range(net.ngen):
        c2, c1 = S * S * net.gen_cost[g, 0], S * net.gen_cost[g, 1]
        pmin, pmax, qmin, qmax = net.gen_lim[g]
        fp = lambda p: c2 * p * p + c1 * p + v0["lpg"][g] * (p - v0["pgt"][g]) + 0.5 * rho * (p - v0["pgt"][g]) ** 2
        fq = lambda q: v0["lqg"][g] * (q - v0["qgt"][g]) + 0.5 * rho * (q - v0["qgt"][g]) ** 2
        rp = so.minimize_scalar(fp, bounds=(pmin, pmax), method="bounded", options=dict(xatol=1e-12))
        rq = so.minimize_scalar(fq, bounds=(qmin, qmax), method="bounded", options=dict(xatol=1e-12))
        grid = np.linspace(pmin, pmax, 2001)
        assert fp(v1["pg"][g]) <= min(fp(grid).min(), rp.fun) + 1e-9
        assert abs(v1["pg"][g] - rp.x) <= 1e-6
        assert abs(v1["qg"][g] - rq.x) <= 1e-6


def bus_kkt(net, v, b):
    """Solve one bus subproblem as a generic equality-constrained least squares."""
    rho = net.rho
    names, targets = [], []
    gens = [g for g in range(net.ngen) if net.gen_bus[g] == b]
    ends = [(l, e) for l in range(net.nbranch) for e in (0, 1)
            if (net.br_from[l] if e == 0 else net.br_to[l]) == b]
    for g in gens:
        names += [("pg", g), ("qg", g)]
        targets += [v["pg"][g] + v["lpg"][g] / rho, v["qg"][g] + v["lqg"][g] / rho]
    for l, e in ends:
        names += [("pe", l, e), ("qe", l, e)]
        targets += [v["y"][l, 2 * e] + v["lam"][l, 2 * e] / rho,
                    v["y"][l, 2 * e + 1] + v["lam"][l, 2 * e + 1] / rho]
    nv = len(names) + 2  # + w, theta
    iw, it = nv - 2, nv - 1
    # objective sum_k rho/2 (y_k - t_k)^2 with one term per end for w and theta
    Hm = np.zeros((nv, nv)); rhs = np.zeros(nv)
    for k, t in enumerate(targets):
        Hm[k, k] += rho; rhs[k] += rho * t
    for l, e in ends:
        tw = v["y"][l, 4 + e] + v["lam"][l, 4 + e] / rho
        tt = v["y"][l, 6 + e] + v["lam"][l, 6 + e] / rho
        Hm[iw, iw] += rho; rhs[iw] += rho * tw
        Hm[it, it] += rho; rhs[it] += rho * tt
    pd, qd, gs, bs = net.bus_load[b]
    A = np.zeros((2, nv)); bb = np.array([pd, qd])
    for k, nm in enumerate(names):
        if nm[0] == "pg": A[0, k] = 1
        if nm[0] == "qg": A[1, k] = 1
        if nm[0] == "pe": A[0, k] = -1
        if nm[0] == "qe": A[1, k] = -1
    A[0, iw] = -gs; A[1, iw] = bs
    K = np.block([[Hm, A.T], [A, np.zeros((2, 2))]])
    sol = np.linalg.solve(K, np.concatenate([rhs, bb]))[:nv]
    return names, sol, gens, ends


def test_bus_update_matches_kkt_solve(orc, small):
    net, st = small
    # give two buses shunts so that w enters the balance rows
    net2 = W.Network(net.nbus, net.br_from, net.br_to, net.br_adm, net.br_lo, net.br_hi,
                     net.gen_bus, net.gen_cost, net.gen_lim, net.bus_load.copy(), rho=net.rho)
    net2.bus_load[3, 2:] = [0.05, -0.2]
    net2.bus_load[net.gen_bus[0], 2:] = [0.1, 0.3]
    before = orc.admm_views(net2, st)
    after_st, _ = orc.admm_phase(net2, st, 2)
    after = orc.admm_views(net2, after_st)
    for b in list(range(0, net.nbus, 3)) + [3, int(net.gen_bus[0])]:
        names, sol, gens, ends = bus_kkt(net2, before, b)
        for k, nm in enumerate(names):
            got = {"pg": lambda: after["pgt"][nm[1]], "qg": lambda: after["qgt"][nm[1]],
                   "pe": lambda: after["yt"][nm[1], 2 * nm[2]],
                   "qe": lambda: after["yt"][nm[1], 2 * nm[2] + 1]}[nm[0]]()
            assert got == pytest.approx(sol[k], rel=1e-10, abs=1e-10)
        assert after["wt"][b] == pytest.approx(sol[-2], rel=1e-10, abs=1e-12)
        if b == net.ref_bus:
            assert after["tht"][b] == 0.0
        else:
            assert after["tht"][b] == pytest.approx(sol[-1], rel=1e-10, abs=1e-12)
        # the balance rows hold after the update
        pd, qd, gs, bs = net2.bus_load[b]
        P = sum(after["pgt"][g] for g in gens) - sum(after["yt"][l, 2 * e] for l, e in ends) - gs * after["wt"][b]
        Qr = sum(after["qgt"][g] for g in gens) - sum(after["yt"][l, 2 * e + 1] for l, e in ends) + bs * after["wt"][b]
        assert P == pytest.approx(pd, abs=1e-12) and Qr == pytest.approx(qd, abs=1e-12)


def test_multiplier_update_identity(orc, small):
    net, st = small
    after_st, p2 = orc.admm_phase(net, st, 3)
    a, b = orc.admm_views(net, st), orc.admm_views(net, after_st)
    rho = net.rho
    assert np.allclose(b["lpg"] - a["lpg"], rho * (a["pg"] - a["pgt"]), rtol=1e-12, atol=1e-9)
    copies = np.concatenate([a["yt"], a["wt"][net.br_from][:, None], a["wt"][net.br_to][:, None],
                             a["tht"][net.br_from][:, None], a["tht"][net.br_to][:, None]], axis=1)
    assert np.allclose(b["lam"] - a["lam"], rho * (a["y"] - copies), rtol=1e-12, atol=1e-9)
    assert np.allclose(b["mu"] - a["mu"], rho * (a["x"][:, 4:6] - a["y"][:, [0, 2]]), atol=1e-9)
    r2 = np.sum((a["pg"] - a["pgt"]) ** 2 + (a["qg"] - a["qgt"]) ** 2) + np.sum((a["y"] - copies) ** 2)
    assert p2 == pytest.approx(r2, rel=1e-12)


def test_iteration_is_the_four_phases(orc, small):
    net, st = small
    s = st
    for ph in range(4):
        s, _ = orc.admm_phase(net, s, ph)
    whole, res = orc.admm_run(net, st, 1)
    assert np.array_equal(s, whole)
    assert res.shape == (1, 2) and np.all(np.isfinite(res))


def test_branch_phase_solves_each_branch(orc, small):
    """After the branch phase every branch variable satisfies the first-order conditions of
    its BR6 problem built from the state, and the stored couplings are its flows."""
    net, st = small
    after_st, _ = orc.admm_phase(net, st, 1)
    a, b = orc.admm_views(net, st), orc.admm_views(net, after_st)
    for l in range(0, net.nbranch, 5):
        i, j = net.br_from[l], net.br_to[l]
        p = np.concatenate([net.br_adm[l], a["yt"][l], [a["wt"][i], a["wt"][j], a["tht"][i], a["tht"][j]],
                            a["lam"][l], a["mu"][l], np.full(10, net.rho)])
        x = b["x"][l]
        g = orc.eval_g(1, 6, p, x)
        assert orc.projgrad_inf(x, net.br_lo[l], net.br_hi[l], g) <= 1e-6
        fl = orc.br6_flows(p, x)
        assert np.allclose(b["y"][l], [*fl, x[0] ** 2, x[1] ** 2, x[2], x[3]], rtol=0, atol=0)


def test_bus_update_on_a_hub_bus(orc):
    """A hub bus with 24 more branch ends, 6 more generators and a shunt: the oracle's bus
    update still equals the generic KKT solve, and the balance rows hold after it."""
    net = W.network(nbus=80, nbranch=110, ngen=12, config_id=94, hub_ends=24, hub_gens=6,
                    hub_shunt=(0.04, 0.15))
    st = orc.admm_init(net)
    st, _ = orc.admm_run(net, st, 3)
    before = orc.admm_views(net, st)
    after = orc.admm_views(net, orc.admm_phase(net, st, 2)[0])
    b = 0
    names, sol, gens, ends = bus_kkt(net, before, b)
    assert len(ends) > 16 and len(gens) > 4
    for k, nm in enumerate(names):
        got = {"pg": lambda: after["pgt"][nm[1]], "qg": lambda: after["qgt"][nm[1]],
               "pe": lambda: after["yt"][nm[1], 2 * nm[2]],
               "qe": lambda: after["yt"][nm[1], 2 * nm[2] + 1]}[nm[0]]()
        assert got == pytest.approx(sol[k], rel=1e-10, abs=1e-10)
    assert after["wt"][b] == pytest.approx(sol[-2], rel=1e-10, abs=1e-12)
    pd, qd, gs, bs = net.bus_load[b]
    P = sum(after["pgt"][g] for g in gens) - sum(after["yt"][l, 2 * e] for l, e in ends) - gs * after["wt"][b]
    Qr = sum(after["qgt"][g] for g in gens) - sum(after["yt"][l, 2 * e + 1] for l, e in ends) + bs * after["wt"][b]
    assert P == pytest.approx(pd, abs=1e-12) and Qr == pytest.approx(qd, abs=1e-12)
