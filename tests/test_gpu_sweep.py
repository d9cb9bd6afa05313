"""A seeded random sweep of batches against the oracle, beside the fixed cases: the family
(QP4 of one size, of mixed sizes up to 128 or beyond 128; BR6; HS45M from random starts),
the batch size and the launch plan (default, persistent with 8 or 12 waves per CU, groups of
4 or 8 lanes for the lane sizes, 16-lane groups for 8 < n <= 16, 256-lane workgroups, the
global-memory workspace) are drawn from a fixed seed, and every instance meets the bars of
tests/parity.py. The draws cover the corners the fixed cases visit one at a time in
combination, including the group kernels' row slots past n = 6 on 4 and 8 lanes."""
import numpy as np
import pytest

from paper_2106_14995_amd import workloads as W
from parity import check_parity, oracle_ref

pytestmark = pytest.mark.gpu

PLANS = ["default", "pool12", "pool8", "group8", "group4", "g16", "lane256", "global"]


def _draws(seed, count):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        out.append((int(rng.integers(1000, 100000)),
                    str(rng.choice(["qp4_mixed", "qp4_uniform", "br6", "hs45m", "qp4_big"])),
                    str(rng.choice(PLANS)), int(rng.integers(1, 1 << 30))))
    return out


@pytest.fixture(scope="module")
def tron():
    import torch
    assert torch.cuda.is_available()
    from paper_2106_14995_amd import tron as T
    T.lib()
    return T


def _spec(T, name):
    # the default plan runs a mixed batch on the persistent launch; the other options shape
    # the bucketed plan
    return {"default": None, "pool12": T.plan_spec(pool_waves=12), "pool8": T.plan_spec(pool_waves=8),
            "group8": T.plan_spec(lane_group=8, pool_waves=0), "group4": T.plan_spec(lane_group=4, pool_waves=0),
            "g16": T.plan_spec(group16=16, pool_waves=0), "lane256": T.plan_spec(lane_block=256, pool_waves=0),
            "global": T.plan_spec(wave_global=1, pool_waves=0)}[name]


@pytest.mark.parametrize("cid,kind,plan,salt", _draws(20261203, 24))
def test_random_batch_against_the_oracle(tron, cid, kind, plan, salt):
    import torch
    r = np.random.default_rng(salt)
    if kind == "qp4_mixed":
        B = int(r.integers(1, 3000))
        sizes = W.loguniform_sizes(B, 1, int(r.choice([8, 16, 32, 64, 128])), config_id=cid)
        bt, convex = W.qp4_batch(B, sizes, config_id=cid), True
    elif kind == "qp4_uniform":
        bt, convex = W.qp4_batch(int(r.integers(1, 3000)), int(r.integers(1, 65)), config_id=cid), True
    elif kind == "qp4_big":
        bt, convex = W.qp4_batch(int(r.integers(1, 48)), int(r.choice([129, 160, 200, 256])), config_id=cid), True
    elif kind == "br6":
        bt, convex = W.br6_batch(int(r.integers(1, 20000)), config_id=cid), False
    else:
        B = int(r.integers(1, 2000))
        bt, convex = W.hs45m_random_start(B, W.loguniform_sizes(B, 1, int(r.choice([8, 16, 32, 64])), config_id=cid),
                                          config_id=cid), False
    h = tron.Batch(bt.family, bt.n, batch=bt.batch if np.isscalar(bt.n) else None, spec=_spec(tron, plan))
    x, f, st, it = h.solve(*tron.to_device(bt))
    torch.cuda.synchronize()
    g = dict(x=x.cpu().numpy(), f=f.cpu().numpy(), status=st.cpu().numpy(), iters=it.cpu().numpy())
    h.close()
    check_parity(bt, g, oracle_ref(bt), convex=convex, label=f"{kind} cid {cid} B {bt.batch} {plan}")
