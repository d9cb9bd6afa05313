"""Seeded synthetic workloads for the batched TRON solve and the component ADMM.

This module only draws inputs. It holds no step of the solver: the GPU library and the
CPU oracle each evaluate the problems with their own code, and both receive the arrays
made here.

Every instance has its own generator, ``SeedSequence(entropy=210614995,
spawn_key=(config_id, instance_id))`` with PCG64, so any instance can be rebuilt alone
(needed to show that a result does not depend on what it was batched with).

Packing (an interface shared with the C ABI): instance b of size n_b has a parameter
block of ``param_size(family, n_b)`` doubles and vectors (lo, hi, x0) of n_b doubles,
stored back to back in instance order.

Workload recipes:
  * QP4 (a strictly convex quartic box problem): f = x'Qx/2 + c'x + kappa sum x_i^4,
    Q = A'A + 0.1 I with A ~ N(0,1)^{n x n}, c ~ N(0,1)^n, l ~ U[-2,-0.5], u ~ U[0.5,2],
    x0 = 0, kappa = 0.1.
  * BR6 (the branch subproblem of the component ADMM, eq. exp-branch, with two flow
    copies): g ~ U[0.5,5], b ~ U[-20,-1] for all four g-type and b-type admittances;
    a nominal point v ~ U[0.95,1.05]^2, th_i ~ U[-0.2,0.2], th_j = th_i + U[-0.25,0.25];
    targets = the nominal couplings + 0.05 N(0,1); lambda ~ N(0,1); mu = 0; rho = 400;
    bounds v in [0.9,1.1], th in [-pi,pi], z in [-5,5]; warm start at the nominal point.
    The nominal flows come from the complex power p + jq = y V_l conj(V_l - V_m) with
    y = g + jb, which is the same physics as the flow equations of the paper written in
    complex form.
  * BR8L (BR6 with the line limits p^2 + q^2 <= smax^2 of both ends as equalities with
    slacks, for the augmented-Lagrangian loop): smax = U[0.85, 1.3] x the larger nominal
    |S|, lambda_h = 0, rho_h = 10, slacks in [0, smax^2] starting feasible.
  * HS45M (the paper's modified hs45): f = 120 - prod x_i, 0 <= x_i <= i, x0_i = i/2 (the
    paper's start), or x0_i ~ U[0, i] for the random-start variant.
  * Network for the ADMM: random recursive spanning tree plus distinct extra edges,
    generators on distinct buses, quadratic costs, loads scaled to the generation.
"""
from __future__ import annotations

import math

import numpy as np

ENTROPY = 210614995
QP4, BR6, HS45M, BR8L = 0, 1, 2, 3
FAMILY_NAMES = {QP4: "qp4", BR6: "br6", HS45M: "hs45m", BR8L: "br8l"}


def rng_for(config_id: int, instance_id: int) -> np.random.Generator:
    ss = np.random.SeedSequence(entropy=ENTROPY, spawn_key=(int(config_id), int(instance_id)))
    return np.random.Generator(np.random.PCG64(ss))


def param_size(family: int, n: int) -> int:
    if family == QP4:
        return n * (n + 1) // 2 + n + 1
    if family == BR6:
        return 36
    if family == BR8L:
        return 40
    return 0


class Batch:
    """A packed batch: params, lo, hi, x0 plus the per-instance sizes."""

    def __init__(self, family, n, params, lo, hi, x0):
        self.family = int(family)
        self.n = np.ascontiguousarray(n, dtype=np.int32)
        self.params = np.ascontiguousarray(params, dtype=np.float64)
        self.lo = np.ascontiguousarray(lo, dtype=np.float64)
        self.hi = np.ascontiguousarray(hi, dtype=np.float64)
        self.x0 = np.ascontiguousarray(x0, dtype=np.float64)

    @property
    def batch(self) -> int:
        return int(self.n.shape[0])

    @property
    def uniform_n(self):
        if self.batch and np.all(self.n == self.n[0]):
            return int(self.n[0])
        return None

    def voff(self):
        return np.concatenate([[0], np.cumsum(self.n.astype(np.int64))])

    def poff(self):
        sizes = np.array([param_size(self.family, int(k)) for k in self.n], dtype=np.int64)
        return np.concatenate([[0], np.cumsum(sizes)])

    def instance(self, b):
        """(n, params, lo, hi, x0) of instance b (views)."""
        vo, po = self.voff(), self.poff()
        s = slice(vo[b], vo[b + 1])
        return (int(self.n[b]), self.params[po[b]:po[b + 1]], self.lo[s], self.hi[s], self.x0[s])

    def subset(self, idx):
        """A new batch holding the listed instances, in the given order."""
        vo, po = self.voff(), self.poff()
        idx = list(idx)
        params = [self.params[po[b]:po[b + 1]] for b in idx]
        vs = [slice(vo[b], vo[b + 1]) for b in idx]
        cat = lambda parts: np.concatenate(parts) if parts else np.zeros(0)
        return Batch(self.family, self.n[idx], cat(params), cat([self.lo[s] for s in vs]),
                     cat([self.hi[s] for s in vs]), cat([self.x0[s] for s in vs]))


# ------------------------------------------------------------------------------------
# QP4
# ------------------------------------------------------------------------------------
def qp4_instance(rng: np.random.Generator, n: int, kappa: float = 0.1):
    a = rng.standard_normal((n, n))
    q = a.T @ a + 0.1 * np.eye(n)
    c = rng.standard_normal(n)
    lo = rng.uniform(-2.0, -0.5, n)
    hi = rng.uniform(0.5, 2.0, n)
    packed = q[np.tril_indices(n)]  # row by row: Q00 Q10 Q11 Q20 ...
    params = np.concatenate([packed, c, [kappa]])
    return params, lo, hi, np.zeros(n)


def qp4_batch(batch: int, n, config_id: int = 0, kappa: float = 0.1, first: int = 0) -> Batch:
    """QP4 instances first..first+batch-1 of config `config_id`; n is an int or per-instance."""
    ns = np.full(batch, n, dtype=np.int32) if np.isscalar(n) else np.asarray(n, dtype=np.int32)
    ps, ls, hs, xs = [], [], [], []
    for b in range(batch):
        p, l, h, x = qp4_instance(rng_for(config_id, first + b), int(ns[b]), kappa)
        ps.append(p); ls.append(l); hs.append(h); xs.append(x)
    cat = lambda v: np.concatenate(v) if v else np.zeros(0)
    return Batch(QP4, ns, cat(ps), cat(ls), cat(hs), cat(xs))


def qp4_half_rank_batch(batch: int, n: int, config_id: int = 90, kappa: float = 0.1) -> Batch:
    """QP4 with Q = A'A for a Gaussian A of n // 2 rows (rank n // 2): with the quartic term f
    stays strictly convex, but its Hessian at the start x0 = 0 is Q itself, singular, so the
    first factorisations meet non-positive pivots and the shifted retries run."""
    ps, ls, hs, xs = [], [], [], []
    for b in range(batch):
        rng = rng_for(config_id, b)
        a = rng.standard_normal((n // 2, n)) / np.sqrt(n)
        q = a.T @ a
        c = rng.standard_normal(n)
        ps.append(np.concatenate([q[np.tril_indices(n)], c, [kappa]]))
        ls.append(np.full(n, -2.0)); hs.append(np.full(n, 2.0)); xs.append(np.zeros(n))
    return Batch(QP4, np.full(batch, n, dtype=np.int32), np.concatenate(ps), np.concatenate(ls),
                 np.concatenate(hs), np.concatenate(xs))


def loguniform_sizes(batch: int, nmin: int, nmax: int, config_id: int, salt: int = 7777777):
    """n_b = clamp(round(exp(U[ln nmin, ln nmax]))), one draw per instance."""
    out = np.empty(batch, dtype=np.int32)
    for b in range(batch):
        r = rng_for(config_id, salt + b)  # a stream apart from the instance's own data
        v = math.exp(r.uniform(math.log(nmin), math.log(nmax)))
        out[b] = min(max(int(round(v)), nmin), nmax)
    return out


def qp4_uneven_batch(batch: int, nmin: int = 4, nmax: int = 64, config_id: int = 3) -> Batch:
    sizes = loguniform_sizes(batch, nmin, nmax, config_id)
    return qp4_batch(batch, sizes, config_id=config_id)


# ------------------------------------------------------------------------------------
# BR6
# ------------------------------------------------------------------------------------
BR6_LO = np.array([0.9, 0.9, -math.pi, -math.pi, -5.0, -5.0])
BR6_HI = np.array([1.1, 1.1, math.pi, math.pi, 5.0, 5.0])


def complex_flows(g, b, vi, vj, thi, thj):
    """(p_ij, q_ij, p_ji, q_ji) from p_lm + j q_lm = y V_l conj(V_l - V_m), y = g + jb."""
    y = g + 1j * b
    Vi = vi * np.exp(1j * thi)
    Vj = vj * np.exp(1j * thj)
    sij = y * Vi * np.conj(Vi - Vj)
    sji = y * Vj * np.conj(Vj - Vi)
    return np.array([sij.real, sij.imag, sji.real, sji.imag])


def br6_instance(rng: np.random.Generator, rho: float = 400.0, sigma: float = 0.05):
    g = rng.uniform(0.5, 5.0)
    b = rng.uniform(-20.0, -1.0)
    v = rng.uniform(0.95, 1.05, 2)
    thi = rng.uniform(-0.2, 0.2)
    thj = thi + rng.uniform(-0.25, 0.25)
    pq = complex_flows(g, b, v[0], v[1], thi, thj)
    nominal = np.array([pq[0], pq[1], pq[2], pq[3], v[0] ** 2, v[1] ** 2, thi, thj])
    targets = nominal + sigma * rng.standard_normal(8)
    lam = rng.standard_normal(8)
    adm = np.array([g, b, g, b, g, b, g, b])
    params = np.concatenate([adm, targets, lam, [0.0, 0.0], np.full(10, rho)])
    x0 = np.array([v[0], v[1], thi, thj, np.clip(pq[0], -5, 5), np.clip(pq[2], -5, 5)])
    return params, BR6_LO.copy(), BR6_HI.copy(), x0


def br6_batch(batch: int, config_id: int = 1, first: int = 0) -> Batch:
    ps, xs = [], []
    for k in range(batch):
        p, _, _, x = br6_instance(rng_for(config_id, first + k))
        ps.append(p); xs.append(x)
    params = np.concatenate(ps) if ps else np.zeros(0)
    x0 = np.concatenate(xs) if xs else np.zeros(0)
    return Batch(BR6, np.full(batch, 6, dtype=np.int32), params, np.tile(BR6_LO, batch),
                 np.tile(BR6_HI, batch), x0)


def br8l_instance(rng: np.random.Generator, rho_h: float = 10.0):
    """A BR6 instance plus apparent-power limits on both ends: smax = U[0.85, 1.3] times the
    larger nominal |S| (binding on about half the instances), lambda_h = 0, rho_h given;
    slacks start at the value that makes the limit equalities hold at the start."""
    params, lo, hi, x0 = br6_instance(rng)
    g, b = params[0], params[1]
    pq = complex_flows(g, b, x0[0], x0[1], x0[2], x0[3])
    s2 = np.array([pq[0] ** 2 + pq[1] ** 2, pq[2] ** 2 + pq[3] ** 2])
    smax2 = (rng.uniform(0.85, 1.3) ** 2) * float(s2.max())
    params = np.concatenate([params, [smax2, 0.0, 0.0, rho_h]])
    lo = np.concatenate([lo, [0.0, 0.0]])
    hi = np.concatenate([hi, [smax2, smax2]])
    x0 = np.concatenate([x0, np.clip(smax2 - s2, 0.0, smax2)])
    return params, lo, hi, x0


def br8l_batch(batch: int, config_id: int = 5, first: int = 0, rho_h: float = 10.0) -> Batch:
    """Branch subproblems with line limits (family BR8L, n = 8, 40 parameters)."""
    ps, ls, hs, xs = [], [], [], []
    for k in range(batch):
        p, lo, hi, x = br8l_instance(rng_for(config_id, first + k), rho_h)
        ps.append(p); ls.append(lo); hs.append(hi); xs.append(x)
    cat = lambda v: np.concatenate(v) if v else np.zeros(0)
    return Batch(BR8L, np.full(batch, 8, dtype=np.int32), cat(ps), cat(ls), cat(hs), cat(xs))


def br6_zero_residual(batch: int, config_id: int = 91) -> Batch:
    """Instances whose minimum is known: targets are the nominal couplings exactly,
    lambda = mu = 0, the flow copies start equal to the flows (|p| < 5), so x* = nominal
    and f* = 0. The start point is moved away from the nominal point."""
    ps, xs, nominal = [], [], []
    for k in range(batch):
        rng = rng_for(config_id, k)
        g = rng.uniform(0.5, 5.0)
        b = rng.uniform(-20.0, -1.0)
        v = rng.uniform(0.95, 1.05, 2)
        thi = rng.uniform(-0.2, 0.2)
        thj = thi + rng.uniform(-0.1, 0.1)
        pq = complex_flows(g, b, v[0], v[1], thi, thj)
        tgt = np.array([pq[0], pq[1], pq[2], pq[3], v[0] ** 2, v[1] ** 2, thi, thj])
        adm = np.array([g, b, g, b, g, b, g, b])
        ps.append(np.concatenate([adm, tgt, np.zeros(8), [0.0, 0.0], np.full(10, 400.0)]))
        xstar = np.array([v[0], v[1], thi, thj, pq[0], pq[2]])
        nominal.append(xstar)
        start = xstar + rng.uniform(-0.02, 0.02, 6)
        xs.append(np.clip(start, BR6_LO, BR6_HI))
    bt = Batch(BR6, np.full(batch, 6, dtype=np.int32), np.concatenate(ps),
               np.tile(BR6_LO, batch), np.tile(BR6_HI, batch), np.concatenate(xs))
    bt.xstar = np.concatenate(nominal)
    return bt


# ------------------------------------------------------------------------------------
# HS45M
# ------------------------------------------------------------------------------------
def hs45m_batch(batch: int, n: int) -> Batch:
    i = np.arange(1, n + 1, dtype=np.float64)
    return Batch(HS45M, np.full(batch, n, dtype=np.int32), np.zeros(0), np.tile(np.zeros(n), batch),
                 np.tile(i, batch), np.tile(i / 2.0, batch))


def hs45m_random_start(batch: int, n, config_id: int = 70) -> Batch:
    """HS45M instances (0 <= x_i <= i) with x0_i ~ U[0, i]; n an int or one size per instance."""
    ns = np.full(batch, n, dtype=np.int32) if np.isscalar(n) else np.asarray(n, dtype=np.int32)
    los, his, x0s = [], [], []
    for b in range(batch):
        k = int(ns[b])
        i = np.arange(1, k + 1, dtype=np.float64)
        los.append(np.zeros(k))
        his.append(i)
        x0s.append(rng_for(config_id, b).uniform(0.0, 1.0, k) * i)
    cat = lambda v: np.concatenate(v) if v else np.zeros(0)
    return Batch(HS45M, ns, np.zeros(0), cat(los), cat(his), cat(x0s))


# ------------------------------------------------------------------------------------
# Dense SPD blocks for the kernel-design microbenchmarks (section 4, Tables 1-2)
# ------------------------------------------------------------------------------------
def spd_blocks(count: int, n: int, config_id: int = 80):
    """(A, b): count SPD matrices A = M'M + n I with M ~ N(0,1)^{n x n} (eigenvalues in
    about [n, 5n]) and right-hand sides b ~ N(0,1)^n, as float64 arrays (count, n, n), (count, n)."""
    A = np.empty((count, n, n))
    B = np.empty((count, n))
    for p in range(count):
        r = rng_for(config_id, p)
        M = r.standard_normal((n, n))
        A[p] = M.T @ M + n * np.eye(n)
        B[p] = r.standard_normal(n)
    return A, B


# ------------------------------------------------------------------------------------
# Network for the component ADMM
# ------------------------------------------------------------------------------------
class Network:
    """Host arrays of a synthetic transmission network (per-unit quantities)."""

    def __init__(self, nbus, br_from, br_to, br_adm, br_lo, br_hi, gen_bus, gen_cost, gen_lim,
                 bus_load, rho=400.0, base_mva=100.0, ref_bus=0):
        self.nbus = int(nbus)
        self.br_from = np.ascontiguousarray(br_from, dtype=np.int32)
        self.br_to = np.ascontiguousarray(br_to, dtype=np.int32)
        self.br_adm = np.ascontiguousarray(br_adm, dtype=np.float64)
        self.br_lo = np.ascontiguousarray(br_lo, dtype=np.float64)
        self.br_hi = np.ascontiguousarray(br_hi, dtype=np.float64)
        self.gen_bus = np.ascontiguousarray(gen_bus, dtype=np.int32)
        self.gen_cost = np.ascontiguousarray(gen_cost, dtype=np.float64)
        self.gen_lim = np.ascontiguousarray(gen_lim, dtype=np.float64)
        self.bus_load = np.ascontiguousarray(bus_load, dtype=np.float64)
        self.rho = float(rho)
        self.base_mva = float(base_mva)
        self.ref_bus = int(ref_bus)

    @property
    def nbranch(self):
        return int(self.br_from.shape[0])

    @property
    def ngen(self):
        return int(self.gen_bus.shape[0])

    def state_size(self):
        return 6 * self.ngen + 30 * self.nbranch + 2 * self.nbus


def network(nbus: int = 2000, nbranch: int = 3000, ngen: int = 500, config_id: int = 2,
            rho: float = 400.0, hub_ends: int = 0, hub_gens: int = 0,
            hub_shunt=(0.0, 0.0)) -> Network:
    """Random recursive spanning tree (bus k joins a uniform j < k) plus distinct extra
    non-adjacent edges; branch g, b as in BR6; generators on distinct uniform buses with
    c2 ~ U[0.01,0.1], c1 ~ U[5,40], pmax ~ U[1,5], pmin = 0, q in [-pmax/2, pmax/2];
    loads pd = 0.6 sum(pmax)/nbus U[0.5,1.5], qd = 0.3 pd; no shunts.
    hub_ends / hub_gens > 0 add a hub at bus 0 (drawn from a stream of its own, so the
    rest of the network is unchanged): hub_ends more branches from bus 0 to distinct buses
    it does not yet touch, hub_gens more generators on bus 0, and the shunt (g, b) there."""
    rng = rng_for(config_id, 0)
    edges = set()
    frm, to = [], []
    for k in range(1, nbus):
        j = int(rng.integers(0, k))
        frm.append(j); to.append(k); edges.add((j, k))
    while len(frm) < nbranch:
        a, b = sorted(int(v) for v in rng.integers(0, nbus, 2))
        if a == b or (a, b) in edges:
            continue
        edges.add((a, b)); frm.append(a); to.append(b)
    nb = len(frm)
    g = rng.uniform(0.5, 5.0, nb)
    bb = rng.uniform(-20.0, -1.0, nb)
    adm = np.stack([g, bb, g, bb, g, bb, g, bb], axis=1)
    lo = np.tile(BR6_LO, (nb, 1))
    hi = np.tile(BR6_HI, (nb, 1))
    gen_bus = rng.choice(nbus, size=ngen, replace=False).astype(np.int32)
    c2 = rng.uniform(0.01, 0.1, ngen)
    c1 = rng.uniform(5.0, 40.0, ngen)
    pmax = rng.uniform(1.0, 5.0, ngen)
    lim = np.stack([np.zeros(ngen), pmax, -pmax / 2.0, pmax / 2.0], axis=1)
    pd = 0.6 * pmax.sum() / nbus * rng.uniform(0.5, 1.5, nbus)
    load = np.stack([pd, 0.3 * pd, np.zeros(nbus), np.zeros(nbus)], axis=1)
    cost = np.stack([c2, c1], axis=1)
    if hub_ends or hub_gens:
        hr = rng_for(config_id, 1)
        touched = {b for e in edges for b in e if 0 in e}
        cand = np.array([k for k in range(1, nbus) if k not in touched])
        ends = hr.choice(cand, size=hub_ends, replace=False)
        for k in sorted(int(v) for v in ends):
            frm.append(0); to.append(k)
        ne = len(ends)
        g2 = hr.uniform(0.5, 5.0, ne)
        b2 = hr.uniform(-20.0, -1.0, ne)
        adm = np.concatenate([adm, np.stack([g2, b2, g2, b2, g2, b2, g2, b2], axis=1)])
        lo = np.tile(BR6_LO, (len(frm), 1))
        hi = np.tile(BR6_HI, (len(frm), 1))
        pm2 = hr.uniform(1.0, 5.0, hub_gens)
        gen_bus = np.concatenate([gen_bus, np.zeros(hub_gens, dtype=np.int32)])
        cost = np.concatenate([cost, np.stack([hr.uniform(0.01, 0.1, hub_gens),
                                               hr.uniform(5.0, 40.0, hub_gens)], axis=1)])
        lim = np.concatenate([lim, np.stack([np.zeros(hub_gens), pm2, -pm2 / 2.0, pm2 / 2.0], axis=1)])
        load = load.copy()
        load[0, 2], load[0, 3] = hub_shunt
    return Network(nbus, frm, to, adm, lo, hi, gen_bus, cost, lim, load, rho=rho)
