"""GPU parity of the batched TRON solve against the CPU oracle, through the C ABI.

The bars and the comparison are in tests/parity.py: strictly convex (QP4) instances must
match the oracle to 1e-8 relative in f and 1e-6 in x; nonconvex ones (BR6, HS45M) must meet
the projected-gradient tolerance 1e-6 at an f no worse than the oracle's plus 1e-8. Full
batches are compared element by element, including the benchmark's 65,536-instance branch
batch and the 50,000-instance uneven batch in the launch configurations the benchmark
times; companion tests solve both sides to gtol = 1e-10, where the convex x bar holds with
no trajectory-split allowance.
"""
import numpy as np
import pytest

import oracle
from paper_2106_14995_amd import workloads as W
from parity import PG_TOL, check_parity, oracle_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tron():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2106_14995_amd import tron as T
    T.lib()
    return T


def gpu_solve(T, bt, **kw):
    import torch
    h = T.Batch(bt.family, bt.n, opts=T.options(**kw))
    x, f, st, it = h.solve(*T.to_device(bt))
    torch.cuda.synchronize()
    out = dict(x=x.cpu().numpy(), f=f.cpu().numpy(), status=st.cpu().numpy(), iters=it.cpu().numpy())
    h.close()
    return out


def test_qp4_config0(tron):
    bt = W.qp4_batch(256, 8, config_id=0)
    g = gpu_solve(tron, bt)
    ref = oracle_ref(bt)
    w = check_parity(bt, g, ref, convex=True)
    print("worst", w)
    assert w["pg"] <= PG_TOL
    # same algorithm: iteration counts agree on (almost) every instance
    assert np.mean(g["iters"] == ref["iters"]) >= 0.95


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8])
def test_qp4_each_small_n(tron, n):
    bt = W.qp4_batch(300, n, config_id=40 + n)
    check_parity(bt, gpu_solve(tron, bt), oracle_ref(bt), convex=True)


def test_br6_ragged(tron):
    bt = W.br6_batch(4096 + 37, config_id=1)
    g = gpu_solve(tron, bt)
    ref = oracle_ref(bt)
    check_parity(bt, g, ref, convex=False)
    assert np.all(g["status"] == 0)


def test_br6_full_size(tron):
    """The benchmark's batch (65,536 branch subproblems, one launch), every instance compared
    with the oracle's solve of the same batch."""
    bt = W.br6_batch(65536, config_id=1)
    g = gpu_solve(tron, bt)
    assert np.all(g["status"] == 0)
    check_parity(bt, g, oracle_ref(bt), convex=False, label="br6 65536")


def test_br6_workgroup_sizes_agree(tron):
    """The branch lane kernel keeps each wave's parameters in its own block of the workgroup's
    LDS: 64- and 256-lane workgroups (18 and 72 KB) give the same bits, with a ragged last
    workgroup, and match the oracle."""
    bt = W.br6_batch(3 * 256 + 61, config_id=5)
    g64, plan = _solve_spec(tron, bt, tron.plan_spec(lane_block=64))
    g256, _ = _solve_spec(tron, bt, tron.plan_spec(lane_block=256))
    assert plan[0]["lanes"] == 1
    for k in ("x", "f", "status", "iters"):
        assert np.array_equal(g64[k], g256[k]), k
    check_parity(bt, g256, oracle_ref(bt), convex=False, label="br6 256-lane workgroups")


def _uneven_setup(tron, B=50000):
    import torch
    sizes = W.loguniform_sizes(B, 4, 64, config_id=3)
    bt = W.qp4_batch(B, sizes, config_id=3)
    dev = tron.to_device(bt)
    out = dict(x=torch.empty(int(sizes.astype(np.int64).sum()), dtype=torch.float64, device="cuda"),
               f=torch.empty(B, dtype=torch.float64, device="cuda"),
               status=torch.empty(B, dtype=torch.int32, device="cuda"),
               iters=torch.empty(B, dtype=torch.int32, device="cuda"))
    return sizes, bt, dev, out


def _run_plan(tron, sizes, dev, out, spec=None, **kw):
    import torch
    h = tron.Batch(W.QP4, sizes, opts=tron.options(graph=True, **kw), spec=spec)
    for _ in range(3):  # capture, then replays
        h.solve(*dev, **out)
    torch.cuda.synchronize()
    h.close()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_uneven_full_size(tron):
    """The uneven benchmark's batch (50,000 quartic problems, n log-uniform in [4,64]) in the
    launch configurations the benchmark times: the default plan captured in a graph and
    replayed, and the autotuned plan; every instance is compared with the oracle."""
    sizes, bt, dev, out = _uneven_setup(tron)
    ref = oracle_ref(bt)
    spec, _ = tron.autotune(W.QP4, sizes, *dev, out["x"], out["f"], out["status"], out["iters"], reps=1)
    for name, sp in (("default plan", None), ("bucketed plan", tron.plan_spec(pool_waves=0)),
                     ("autotuned plan", spec)):
        g = _run_plan(tron, sizes, dev, out, spec=sp)
        assert np.all(g["status"] == 0)
        check_parity(bt, g, ref, convex=True, label="uneven 50000, " + name)


def test_uneven_full_size_tight(tron):
    """The same batch with both sides solving to gtol = 1e-10: the strictly convex x bar
    (1e-6) holds for every instance with no trajectory-split allowance."""
    sizes, bt, dev, out = _uneven_setup(tron)
    ref = oracle_ref(bt, gtol=1e-10)
    g = _run_plan(tron, sizes, dev, out, gtol=1e-10)
    assert np.all(g["status"] == 0)
    check_parity(bt, g, ref, convex=True, allow_splits=False, label="uneven 50000 gtol 1e-10")


def test_qp4_config0_tight(tron):
    bt = W.qp4_batch(256, 8, config_id=0)
    g = gpu_solve(tron, bt, gtol=1e-10)
    check_parity(bt, g, oracle_ref(bt, gtol=1e-10), convex=True, allow_splits=False,
                 label="qp4 256 gtol 1e-10")


def test_br6_zero_residual(tron):
    bt = W.br6_zero_residual(512)
    g = gpu_solve(tron, bt, gtol=1e-9)
    assert np.all(g["status"] == 0)
    assert np.abs(g["x"] - bt.xstar).max() <= 1e-7
    assert np.abs(g["f"]).max() <= 1e-12


@pytest.mark.parametrize("n", [1, 3, 5, 8])
def test_hs45m_known_optimum(tron, n):
    import math
    bt = W.hs45m_batch(130, n)
    g = gpu_solve(tron, bt, gtol=1e-9)
    assert np.all(g["status"] == 0)
    assert np.allclose(g["x"].reshape(-1, n), np.arange(1, n + 1), atol=1e-12)
    assert np.allclose(g["f"], 120.0 - math.factorial(n), rtol=1e-14)


@pytest.mark.parametrize("n", [9, 16, 32, 33, 64, 65, 100, 128])
def test_hs45m_wave_known_optimum(tron, n):
    """The wave kernel on the paper's hs45 variant: x* = (1, ..., n) exactly, and f computed
    as 120 minus the left-to-right product, bitwise equal to the oracle's."""
    import math
    bt = W.hs45m_batch(70, n)
    g = gpu_solve(tron, bt, gtol=1e-9)
    ref = oracle_ref(bt, gtol=1e-9)
    assert np.all(g["status"] == 0)
    assert np.array_equal(g["x"].reshape(-1, n), np.tile(np.arange(1.0, n + 1), (70, 1)))
    assert np.array_equal(g["f"], ref["f"])
    assert np.allclose(g["f"], 120.0 - float(math.factorial(n)), rtol=1e-13)


def test_hs45m_random_starts_mixed_sizes(tron):
    """Random interior starts, n log-uniform in [1, 32]: lane and wave buckets in one batch,
    every instance on the global minimiser (the upper corner), nonconvex parity bar."""
    sizes = W.loguniform_sizes(1500, 1, 32, config_id=71)
    bt = W.hs45m_random_start(1500, sizes, config_id=71)
    g = gpu_solve(tron, bt)
    check_parity(bt, g, oracle_ref(bt), convex=False)
    assert np.array_equal(g["x"], bt.hi)


def test_uneven_small_buckets(tron):
    sizes = W.loguniform_sizes(1111, 1, 8, config_id=30)
    bt = W.qp4_batch(1111, sizes, config_id=30)
    g = gpu_solve(tron, bt)
    check_parity(bt, g, oracle_ref(bt), convex=True)


def test_edge_cases(tron):
    import torch
    # empty batch
    h = tron.Batch(W.QP4, 4, batch=0)
    z = torch.zeros(0, dtype=torch.float64, device="cuda")
    h.solve(z, z, z, z)
    h.close()
    # bad bounds, NaN start, fixed variable, a normal instance: statuses match the oracle
    n = 4
    bt = W.qp4_batch(4, n, config_id=60)
    bt.lo[1 * n + 2] = 3.0                      # l > u
    bt.x0[2 * n + 1] = np.nan                   # non-finite start
    bt.lo[3 * n + 0] = bt.hi[3 * n + 0] = 0.25  # fixed variable
    g = gpu_solve(tron, bt)
    ref = oracle_ref(bt)
    assert list(g["status"]) == list(ref["status"]) == [0, 4, 3, 0]
    assert np.array_equal(g["x"][n:2 * n], bt.x0[n:2 * n])  # bad bounds leave x0
    assert g["x"][3 * n] == 0.25
    # max_iter = 1 stops every unfinished instance with MAX_ITER after one iteration
    bt1 = W.qp4_batch(64, 8, config_id=0)
    g1 = gpu_solve(tron, bt1, max_iter=1)
    assert np.all(g1["status"] == 1) and np.all(g1["iters"] == 1)


def test_in_place_and_warm_state(tron):
    import torch
    bt = W.br6_batch(1000, config_id=1)
    h = tron.Batch(W.BR6, 6, batch=1000)
    params, lo, hi, x0 = tron.to_device(bt)
    x = x0.clone()
    _, f1, s1, it1 = h.solve(params, lo, hi, x, x=x)  # x0 and x alias
    st = h.get_state().clone()
    torch.cuda.synchronize()
    assert torch.all(s1 == 0) and torch.all(st[:1000] > 0)
    # solving again from the solution takes no iteration
    _, f2, s2, it2 = h.solve(params, lo, hi, x, x=x)
    torch.cuda.synchronize()
    assert torch.all(s2 == 0) and torch.all(it2 == 0)
    # warm flag: radius and step length come from the handle; set_state restores them
    h.set_options(tron.options(warm=True))
    h.set_state(st)
    back = h.get_state()
    torch.cuda.synchronize()
    assert torch.equal(back, st)
    h.close()


def test_packing_invariance(tron):
    """An instance gives the same bits whatever slot, wave or batch it is solved in."""
    bt = W.br6_batch(700, config_id=1)
    g = gpu_solve(tron, bt)
    idx = [699, 5, 64, 63, 0, 128, 333]
    sub = bt.subset(idx)
    gs = gpu_solve(tron, sub)
    for j, b in enumerate(idx):
        assert np.array_equal(gs["x"][6 * j:6 * j + 6], g["x"][6 * b:6 * b + 6])
        assert gs["f"][j] == g["f"][b] and gs["iters"][j] == g["iters"][b]


# ---------------------------------------------------------------- wavefront-per-instance sizes
@pytest.mark.parametrize("n", [9, 16, 17, 31, 33, 64, 65, 100, 128])
def test_qp4_wave_sizes(tron, n):
    bt = W.qp4_batch(40 if n <= 64 else 16, n, config_id=70 + n)
    g = gpu_solve(tron, bt)
    w = check_parity(bt, g, oracle_ref(bt), convex=True)
    assert np.all(g["status"] == 0), np.bincount(g["status"])


def test_uneven_4_to_64(tron):
    sizes = W.loguniform_sizes(600, 4, 64, config_id=3)
    bt = W.qp4_batch(600, sizes, config_id=3)
    g = gpu_solve(tron, bt)
    check_parity(bt, g, oracle_ref(bt), convex=True)


def test_uneven_4_to_128(tron):
    sizes = W.loguniform_sizes(150, 4, 128, config_id=4)
    bt = W.qp4_batch(150, sizes, config_id=4)
    g = gpu_solve(tron, bt)
    check_parity(bt, g, oracle_ref(bt), convex=True)
    h = tron.Batch(W.QP4, sizes)
    plan = h.plan()
    h.close()
    assert sum(b["count"] for b in plan) == 150
    assert {b["lanes"] for b in plan} == {1, 64}


@pytest.mark.parametrize("n,count", [(129, 24), (200, 16), (256, 12), (257, 8), (400, 6), (512, 6)])
def test_qp4_above_lds_sizes(tron, n, count):
    """n > 128: one wavefront per instance with the Hessian and factor in the handle's
    global-memory workspace."""
    bt = W.qp4_batch(count, n, config_id=70 + n)
    check_parity(bt, gpu_solve(tron, bt), oracle_ref(bt), convex=True)


@pytest.mark.parametrize("n,count", [(40, 8), (100, 6), (150, 4), (300, 3)])
def test_shifted_factorisation_retries(tron, n, count):
    """A singular Hessian at the start (QP4 with a half-rank Q, still strictly convex): the
    factorisation fails on a non-positive pivot and retries with a larger shift, in every
    form of the blocked factorisation (LDS with 1 and 2 rows per lane, global memory with 4
    and 8). The oracle's counters confirm the retries; the result meets the convex bar."""
    bt = W.qp4_half_rank_batch(count, n)
    ref = oracle_ref(bt)
    st = oracle.solve(bt, nthreads=0)["stats"]
    assert np.all(st[:, 3] > st[:, 6]), "no shifted retry in the oracle"  # attempts > passes
    check_parity(bt, gpu_solve(tron, bt), ref, convex=True)


def test_uneven_across_the_lds_limit(tron):
    sizes = np.array([100, 128, 129, 140, 7, 255, 256, 3, 257, 300, 64, 512, 130, 129], dtype=np.int32)
    bt = W.qp4_batch(len(sizes), sizes, config_id=77)
    check_parity(bt, gpu_solve(tron, bt), oracle_ref(bt), convex=True)
    h = tron.Batch(W.QP4, sizes)
    plan = h.plan()
    h.close()
    assert sum(b["count"] for b in plan) == len(sizes)
    assert {b["nmax"] for b in plan if b["lanes"] == 64} >= {256, 512}


def test_wave_edge_cases(tron):
    n = 20
    bt = W.qp4_batch(4, n, config_id=61)
    bt.lo[1 * n + 7] = 5.0                        # l > u
    bt.x0[2 * n + 3] = np.nan                     # non-finite start (inf would be projected)
    bt.lo[3 * n + 4] = bt.hi[3 * n + 4] = -0.75   # fixed variable
    g = gpu_solve(tron, bt)
    ref = oracle_ref(bt)
    assert list(g["status"]) == list(ref["status"])
    assert list(g["status"]) == [0, 4, 3, 0]
    assert g["x"][3 * n + 4] == -0.75
    check_parity(bt, g, ref, convex=True)


def test_wave_packing_invariance(tron):
    sizes = W.loguniform_sizes(300, 4, 80, config_id=33)
    bt = W.qp4_batch(300, sizes, config_id=33)
    g = gpu_solve(tron, bt)
    idx = [299, 3, 150, 77, 0]
    sub = bt.subset(idx)
    gs = gpu_solve(tron, sub)
    vo, svo = bt.voff(), sub.voff()
    for j, b in enumerate(idx):
        assert np.array_equal(gs["x"][svo[j]:svo[j + 1]], g["x"][vo[b]:vo[b + 1]])
        assert gs["f"][j] == g["f"][b]


def test_graph_replays_match_eager(tron):
    """The captured, bucket-concurrent solve replays to the same bits as the eager solve, with
    the program's own eager work and synchronisations between replays."""
    import torch
    sizes = W.loguniform_sizes(900, 2, 72, config_id=34)
    bt = W.qp4_batch(900, sizes, config_id=34)
    dev = tron.to_device(bt)
    buckets = tron.plan_spec(pool_waves=0)
    eager = tron.Batch(W.QP4, sizes, spec=buckets)
    xe, fe, se, ie = [t.clone() for t in eager.solve(*dev)]
    torch.cuda.synchronize()
    g = tron.Batch(W.QP4, sizes, opts=tron.options(graph=True), spec=buckets)
    x = torch.empty_like(xe); f = torch.empty_like(fe)
    st = torch.empty_like(se); it = torch.empty_like(ie)
    for rep in range(4):
        x.fill_(-7.0); f.zero_(); st.fill_(-1); it.fill_(-1)
        g.solve(*dev, x=x, f=f, status=st, iters=it)
        torch.cuda.synchronize()
        assert torch.equal(x, xe) and torch.equal(f, fe), rep
        assert torch.equal(st, se) and torch.equal(it, ie), rep
        # eager work of the program between replays
        eager.solve(*dev)
        _ = (x * 2).sum().item()
        torch.cuda.synchronize()
    # new output pointers: the graph is captured again and still matches
    x2 = torch.empty_like(xe)
    g.solve(*dev, x=x2, f=f, status=st, iters=it)
    torch.cuda.synchronize()
    assert torch.equal(x2, xe)
    g.close()
    eager.close()


def test_plan_specs_and_autotune(tron, tmp_path):
    """Every plan (edges, lane/wave split, streams, lane workgroup size) meets the parity bars
    (a plan only changes where an instance runs), and the autotuner returns a valid plan and
    caches it."""
    import torch
    sizes = W.loguniform_sizes(700, 2, 90, config_id=35)
    bt = W.qp4_batch(700, sizes, config_id=35)
    dev = tron.to_device(bt)
    ref = oracle_ref(bt)
    for spec in (tron.plan_spec(), tron.plan_spec(pool_waves=0),
                 tron.plan_spec(lane_max_n=4, edges=(12, 24, 48, 96), streams=1, lane_block=64, pool_waves=0),
                 tron.plan_spec(lane_max_n=0, edges=(8, 16, 32, 64, 128), streams=2, pool_waves=0)):
        h = tron.Batch(W.QP4, sizes, spec=spec)
        x, f, st, it = h.solve(*dev)
        torch.cuda.synchronize()
        g = dict(x=x.cpu().numpy(), f=f.cpu().numpy(), status=st.cpu().numpy(), iters=it.cpu().numpy())
        h.close()
        check_parity(bt, g, ref, convex=True)
    with pytest.raises(tron.TronError):
        tron.Batch(W.QP4, sizes, spec=tron.plan_spec(edges=(16, 32, 64), pool_waves=0))  # 90 above the last edge
    x = torch.empty(int(bt.n.sum()), dtype=torch.float64, device="cuda")
    f = torch.empty(700, dtype=torch.float64, device="cuda")
    st = torch.empty(700, dtype=torch.int32, device="cuda")
    it = torch.empty(700, dtype=torch.int32, device="cuda")
    cache = str(tmp_path / "tune.txt")
    best, ms = tron.autotune(W.QP4, sizes, *dev, x, f, st, it, reps=1, cache_path=cache)
    assert ms > 0 and best.nedges >= 1
    best2, ms2 = tron.autotune(W.QP4, sizes, *dev, x, f, st, it, reps=1, cache_path=cache)
    assert ms2 == -1.0 and best2.describe() == best.describe()
    h = tron.Batch(W.QP4, sizes, spec=best)
    h.close()


# ---------------------------------------------------------------------------------------
# the persistent size-bucketed launch (plan spec pool_waves 8 or 12)
# ---------------------------------------------------------------------------------------
def _solve_spec(T, bt, spec, **kw):
    import torch
    h = T.Batch(bt.family, bt.n, spec=spec, opts=T.options(**kw))
    x, f, st, it = h.solve(*T.to_device(bt))
    torch.cuda.synchronize()
    out = dict(x=x.cpu().numpy(), f=f.cpu().numpy(), status=st.cpu().numpy(), iters=it.cpu().numpy())
    plan = h.plan()
    h.close()
    return out, plan


def test_default_plan_forms(tron):
    """The default plan runs a batch of mixed sizes up to n = 128 as one persistent launch
    (one wavefront entry holding every n > 8 instance, then the lane sizes); pool_waves 0
    asks for the buckets; a uniform batch, and a mixed batch with an n above 128, take the
    buckets whatever the spec says."""
    sizes = W.loguniform_sizes(300, 2, 100, config_id=36)
    h = tron.Batch(W.QP4, sizes)
    plan = h.plan()
    h.close()
    waves = [b for b in plan if b["lanes"] == 64]
    assert len(waves) == 1 and waves[0]["count"] == int((sizes > 8).sum()) and waves[0]["nmax"] == int(sizes.max())
    assert sum(b["count"] for b in plan) == 300
    h = tron.Batch(W.QP4, sizes, spec=tron.plan_spec(pool_waves=0))
    plan0 = h.plan()
    h.close()
    assert len([b for b in plan0 if b["lanes"] == 64]) > 1
    assert {b["nmax"] for b in plan0 if b["lanes"] == 64} <= set(tron.DEFAULT_EDGES)
    assert sum(b["count"] for b in plan0) == 300
    h = tron.Batch(W.QP4, 40, batch=100)
    assert h.plan() == [dict(nmax=40, lanes=64, count=100)]
    h.close()
    big = np.array([10, 20, 200, 30], dtype=np.int32)
    h = tron.Batch(W.QP4, big)
    assert len([b for b in h.plan() if b["lanes"] == 64]) >= 2
    h.close()


@pytest.mark.parametrize("waves", [8, 12])
def test_pool_plan_uneven_full_size(tron, waves):
    """The uneven benchmark's batch (50,000 quartic problems, n log-uniform in [4,64]) through
    the persistent launch, captured in a graph and replayed: every instance against the
    oracle, and the same bits as the bucketed plan (the same solver code runs each
    instance; only where it runs differs)."""
    sizes, bt, dev, out = _uneven_setup(tron)
    ref = oracle_ref(bt)
    g = _run_plan(tron, sizes, dev, out, spec=tron.plan_spec(pool_waves=waves))
    assert np.all(g["status"] == 0)
    check_parity(bt, g, ref, convex=True, label=f"uneven 50000, persistent {waves} waves")
    b = _run_plan(tron, sizes, dev, out)
    for k in ("x", "f", "status", "iters"):
        assert np.array_equal(g[k], b[k]), k


@pytest.mark.parametrize("fam", ["qp4", "hs45m"])
def test_pool_plan_mixed_to_128(tron, fam):
    """Sizes 1..128 in one persistent launch (one and two rows per lane in the same kernel),
    with every lane size in the lane packs, against the oracle."""
    sizes = W.loguniform_sizes(700, 1, 128, config_id=36)
    bt = W.qp4_batch(700, sizes, config_id=36) if fam == "qp4" else W.hs45m_random_start(700, sizes, config_id=36)
    ref = oracle_ref(bt)
    for waves in (8, 12):
        g, plan = _solve_spec(tron, bt, tron.plan_spec(pool_waves=waves))
        assert plan[0]["lanes"] == 64 and plan[0]["nmax"] == int(sizes.max())
        assert sum(p["count"] for p in plan) == 700
        check_parity(bt, g, ref, convex=(fam == "qp4"), label=f"pool {fam} {waves} waves, n to 128")
        if fam == "hs45m":
            assert np.array_equal(g["x"], bt.hi)  # the global minimiser, the upper corner


def test_pool_plan_partitions(tron):
    """Every instance in the persistent launch (lane_max_n 0, sizes from 1), every instance in
    the lane packs (all n <= 8), and a tiny batch with fewer wave instances than CUs."""
    sizes = W.loguniform_sizes(500, 1, 40, config_id=37)
    bt = W.qp4_batch(500, sizes, config_id=37)
    ref = oracle_ref(bt)
    g, plan = _solve_spec(tron, bt, tron.plan_spec(lane_max_n=0, pool_waves=8))
    assert len(plan) == 1 and plan[0]["count"] == 500
    check_parity(bt, g, ref, convex=True, label="pool, no lane packs")
    small = W.qp4_batch(300, W.loguniform_sizes(300, 1, 8, config_id=38), config_id=38)
    g, plan = _solve_spec(tron, small, tron.plan_spec(pool_waves=12))
    assert all(p["lanes"] == 1 for p in plan)
    check_parity(small, g, oracle_ref(small), convex=True, label="lane packs only")
    few = W.qp4_batch(7, np.array([9, 64, 33, 2, 17, 50, 12], dtype=np.int32), config_id=39)
    g, _ = _solve_spec(tron, few, tron.plan_spec(pool_waves=8))
    check_parity(few, g, oracle_ref(few), convex=True, label="pool, 7 instances")


def test_pool_graph_replays_and_warm(tron):
    """Graph replays of the persistent launch (its claim counter is reset inside the graph)
    give the eager bits every time; warm starts read the resident state it wrote."""
    import torch
    sizes = W.loguniform_sizes(900, 2, 72, config_id=34)
    bt = W.qp4_batch(900, sizes, config_id=34)
    dev = tron.to_device(bt)
    spec = tron.plan_spec(pool_waves=8)
    eager = tron.Batch(W.QP4, sizes, spec=spec)
    xe, fe, se, ie = [t.clone() for t in eager.solve(*dev)]
    torch.cuda.synchronize()
    g = tron.Batch(W.QP4, sizes, spec=spec, opts=tron.options(graph=True))
    x = torch.empty_like(xe); f = torch.empty_like(fe)
    st = torch.empty_like(se); it = torch.empty_like(ie)
    for rep in range(4):
        x.fill_(-7.0); f.zero_(); st.fill_(-1); it.fill_(-1)
        g.solve(*dev, x=x, f=f, status=st, iters=it)
        torch.cuda.synchronize()
        assert torch.equal(x, xe) and torch.equal(f, fe) and torch.equal(st, se) and torch.equal(it, ie), rep
        eager.solve(*dev)
        _ = (x * 2).sum().item()
        torch.cuda.synchronize()
    g.close()
    # warm restart from the solution: every instance converges at once with the stored radius
    w = tron.Batch(W.QP4, sizes, spec=spec)
    x1, _, _, _ = w.solve(*dev)
    w.set_options(tron.options(warm=True))
    p, lo, hi, _ = dev
    x2, _, s2, i2 = w.solve(p, lo, hi, x1.clone())
    torch.cuda.synchronize()
    assert int((s2 == 0).sum()) == 900 and int(i2.max()) == 0
    w.close()
    eager.close()


# ---------------------------------------------------------------------------------------
# the group kernel: one instance per group of G lanes (plan spec lane_group / group16)
# ---------------------------------------------------------------------------------------
@pytest.mark.parametrize("g", [2, 4, 8])
def test_group_kernel_lane_sizes(tron, g):
    """n <= 8 on groups of 2, 4 or 8 lanes: QP4 at every n (padded rows inside a group),
    the branch batch with a ragged tail, and HS45M from random starts, against the oracle."""
    spec = tron.plan_spec(lane_group=g)
    for n in (1, 3, 6, 8):
        bt = W.qp4_batch(257, n, config_id=110 + n)
        out, plan = _solve_spec(tron, bt, spec)
        assert plan[0]["lanes"] == g
        check_parity(bt, out, oracle_ref(bt), convex=True, label=f"group {g}, qp4 n={n}")
    bt = W.br6_batch(4096 + 37, config_id=1)
    out, plan = _solve_spec(tron, bt, spec)
    assert plan[0]["lanes"] == g and np.all(out["status"] == 0)
    check_parity(bt, out, oracle_ref(bt), convex=False, label=f"group {g}, br6")
    hs = W.hs45m_random_start(300, W.loguniform_sizes(300, 1, 8, config_id=72), config_id=72)
    out, _ = _solve_spec(tron, hs, spec)
    check_parity(hs, out, oracle_ref(hs), convex=False, label=f"group {g}, hs45m")
    assert np.array_equal(out["x"], hs.hi)


@pytest.mark.parametrize("g", [8, 16])
def test_group_kernel_to_16(tron, g):
    """8 < n <= 16 on groups of 8 or 16 lanes (two or four instances per 16-lane row) in a
    mixed batch with lane and wavefront sizes around it, and the full-size uneven batch's
    small instances, against the oracle; the tight-tolerance companion meets the x bar with
    no allowance."""
    sizes = W.loguniform_sizes(900, 1, 40, config_id=73)
    bt = W.qp4_batch(900, sizes, config_id=73)
    spec = tron.plan_spec(group16=g, pool_waves=0)  # a bucketed-plan option
    out, plan = _solve_spec(tron, bt, spec)
    mid = [p for p in plan if p["lanes"] == g]
    assert len(mid) == 1 and mid[0]["count"] == int(((sizes > 8) & (sizes <= 16)).sum())
    check_parity(bt, out, oracle_ref(bt), convex=True, label=f"group16={g}")
    out, _ = _solve_spec(tron, bt, spec, gtol=1e-10)
    check_parity(bt, out, oracle_ref(bt, gtol=1e-10), convex=True, allow_splits=False,
                 label=f"group16={g}, gtol 1e-10")
    hs = W.hs45m_random_start(400, W.loguniform_sizes(400, 9, 16, config_id=74), config_id=74)
    out, _ = _solve_spec(tron, hs, spec)
    check_parity(hs, out, oracle_ref(hs), convex=False, label=f"group16={g}, hs45m")
    assert np.array_equal(out["x"], hs.hi)


def test_group_kernel_edge_cases(tron):
    """Bad bounds, a NaN start, fixed variables and max_iter = 1 on the group kernels give
    the oracle's statuses, and an instance's result does not depend on its group neighbours
    (the same instance alone and inside a batch, bitwise)."""
    import torch
    for spec, n in ((tron.plan_spec(lane_group=4), 6), (tron.plan_spec(group16=16), 12)):
        bt = W.qp4_batch(6, n, config_id=75)
        bt.lo[2 * n] = 3.0  # instance 2: l > u
        bt.x0[3 * n + 1] = np.nan  # instance 3: NaN start
        bt.lo[4 * n:5 * n] = bt.hi[4 * n:5 * n] = 0.25  # instance 4: every variable fixed
        out, _ = _solve_spec(tron, bt, spec)
        ref = oracle_ref(bt)
        assert np.array_equal(out["status"], ref["status"]), (out["status"], ref["status"])
        out1, _ = _solve_spec(tron, bt, spec, max_iter=1)
        ref1 = oracle_ref(bt, max_iter=1)
        assert np.array_equal(out1["status"] != 0, ref1["status"] != 0)
        big = W.qp4_batch(64, n, config_id=76)
        full, _ = _solve_spec(tron, big, spec)
        one, _ = _solve_spec(tron, big.subset(np.array([37])), spec)
        vo = big.voff()
        assert np.array_equal(one["x"], full["x"][vo[37]:vo[38]]) and one["f"][0] == full["f"][37]


def test_wave_global_workspace_below_the_lds_limit(tron):
    """The workspace comparison's third form (plan spec wave_global): wavefront instances up
    to n = 128 with the Hessian and factor in a global-memory workspace instead of LDS, one
    and two rows per lane, against the oracle; a uniform batch takes the same form."""
    sizes = W.loguniform_sizes(400, 2, 128, config_id=78)
    bt = W.qp4_batch(400, sizes, config_id=78)
    g, plan = _solve_spec(tron, bt, tron.plan_spec(wave_global=1, pool_waves=0))  # a bucketed-plan option
    check_parity(bt, g, oracle_ref(bt), convex=True, label="wave_global mixed")
    uni = W.qp4_batch(200, 40, config_id=79)
    g, plan = _solve_spec(tron, uni, tron.plan_spec(wave_global=1))
    assert plan[0]["lanes"] == 64
    check_parity(uni, g, oracle_ref(uni), convex=True, label="wave_global n=40")
