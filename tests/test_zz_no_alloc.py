"""The allocation-free entry point (tron_solve_noalloc) through the C ABI: its results equal
those of the handle-based solve (tron_batch_create + tron_batch_solve) on the same inputs,
bit for bit (the same kernels run in the same geometry), on two calls in a row with the
second batch smaller, for a lane-kernel family (BR6, n = 6), an LDS wave kernel (QP4,
n = 40) and the global-workspace wave kernel (QP4, n = 200, whose matrix slots then live in
the fixed array); the results also meet the oracle's bars. Batches whose working memory
exceeds the fixed array, and flags, are rejected."""
import numpy as np
import pytest

from paper_2106_14995_amd import workloads as W
from parity import check_parity, oracle_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tron():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2106_14995_amd import tron as T
    T.lib()
    return T


def _handle_solve(T, bt):
    import torch
    h = T.Batch(bt.family, bt.n)
    x, f, st, it = h.solve(*T.to_device(bt))
    torch.cuda.synchronize()
    out = dict(x=x.cpu().numpy(), f=f.cpu().numpy(), status=st.cpu().numpy(), iters=it.cpu().numpy())
    h.close()
    return out


def _noalloc_solve(T, bt, n):
    import torch
    x, f, st, it = T.solve_noalloc(bt.family, n, bt.batch, *T.to_device(bt))
    torch.cuda.synchronize()
    return dict(x=x.cpu().numpy(), f=f.cpu().numpy(), status=st.cpu().numpy(), iters=it.cpu().numpy())


CASES = [
    ("br6", 6, (4133, 1000)),
    ("qp4", 40, (600, 257)),
    ("qp4", 200, (100, 37)),
]


@pytest.mark.parametrize("fam,n,sizes", CASES)
def test_noalloc_matches_handle_solve(tron, fam, n, sizes):
    for call, B in enumerate(sizes):
        print(f"noalloc {fam} n={n} batch={B} call {call}", flush=True)
        if fam == "br6":
            bt = W.br6_batch(B, config_id=90 + call)
        else:
            bt = W.qp4_batch(B, n, config_id=91 + call)
        got = _noalloc_solve(tron, bt, n)
        ref = _handle_solve(tron, bt)
        for k in ("x", "f", "status", "iters"):
            assert np.array_equal(got[k], ref[k]), (fam, n, B, k)
        if call == len(sizes) - 1:
            check_parity(bt, got, oracle_ref(bt), convex=(fam == "qp4"), label=f"noalloc {fam} n={n}")


def test_noalloc_rejects(tron):
    import torch
    cap = int(tron.lib().tron_noalloc_scratch_bytes())
    assert cap == 64 << 20
    # n = 512: 512 x 513 doubles per instance; 40 instances exceed 64 MiB
    n, B = 512, 40
    assert B * n * 513 * 8 > cap
    z = torch.zeros(B * n, dtype=torch.float64, device="cuda")
    p = torch.zeros(B * tron.param_size(tron.QP4, n), dtype=torch.float64, device="cuda")
    with pytest.raises(tron.TronError) as e:
        tron.solve_noalloc(tron.QP4, n, B, p, z - 1, z + 1, z)
    assert e.value.code == 1 and "working memory" in str(e.value)
    bt = W.qp4_batch(8, 8, config_id=0)
    with pytest.raises(tron.TronError):
        tron.solve_noalloc(tron.QP4, 8, 8, *tron.to_device(bt), opts=tron.options(warm=True))
    with pytest.raises(tron.TronError):
        tron.solve_noalloc(tron.BR6, 5, 8, *tron.to_device(bt))
