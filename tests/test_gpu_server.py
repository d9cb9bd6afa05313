"""GPU tests of the continuous-batching server (tron_server_* in include/tron.h).

The instances of a request are solved by the same kernels as the batch API, one instance per
lane or per wavefront, with nothing shared between instances; so a request's results are
compared bitwise between "alone" and "in a mix" (the stated tolerance is exact equality),
and against the oracle with the parity bars of test_gpu_tron."""
import threading
import time

import numpy as np
import pytest

from paper_2106_14995_amd import workloads as W
from parity import check_parity, oracle_ref

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    import torch
    assert torch.cuda.is_available()
    from paper_2106_14995_amd import tron
    tron.lib()
    return tron


def mixed(count, cfg, nmax=100):
    sizes = W.loguniform_sizes(count, 2, nmax, config_id=cfg)
    return W.qp4_batch(count, sizes, config_id=cfg)


def test_alone_equals_mix_and_batch_api(T):
    import torch
    probe = mixed(300, 80)
    others = [mixed(int(k), 81 + i) for i, k in enumerate([700, 3, 1200, 64, 1, 500, 250, 2000])]
    srv = T.Server(W.QP4, hbm_budget=1 << 30, max_inflight=6, streams=4)
    t = srv.submit_batch(probe)
    srv.wait(t)
    alone = srv.result(t)
    # the same request in the middle of a stream of others, submitted from two threads
    tickets = {}

    def feed(lst, tag):
        for j, b in enumerate(lst):
            tickets[(tag, j)] = srv.submit_batch(b)

    th = threading.Thread(target=feed, args=(others[:4], "a"))
    th.start()
    tp = srv.submit_batch(probe)
    feed(others[4:], "b")
    th.join()
    srv.wait(tp)
    mix = srv.result(tp)
    for k in tickets.values():
        srv.wait(k)
        srv.result(k)
    srv.close()
    for key in ("x", "f", "status", "iters"):
        assert np.array_equal(alone[key], mix[key]), key
    # the batch API gives the same bits
    h = T.Batch(W.QP4, probe.n)
    x, f, st, it = h.solve(*T.to_device(probe))
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), alone["x"])
    assert np.array_equal(st.cpu().numpy(), alone["status"])
    h.close()


def test_server_matches_oracle(T):
    """Every instance of a mixed-size request meets the strictly convex bars against the
    oracle (f to 1e-8 relative, x to 1e-6, projected gradient 1e-6)."""
    bt = mixed(200, 82, nmax=128)
    srv = T.Server(W.QP4)
    t = srv.submit_batch(bt)
    srv.wait(t)
    r = srv.result(t)
    srv.close()
    assert np.all(r["status"] == 0)
    check_parity(bt, r, oracle_ref(bt), convex=True, label="server request")
    assert r["latency"] > 0


def test_session_warm_start(T):
    bt = mixed(150, 83)
    srv = T.Server(W.QP4)
    t1 = srv.submit_batch(bt, session=7)
    srv.wait(t1)
    r1 = srv.result(t1)
    with pytest.raises(T.TronError):
        srv.close_session(12345)
    # from the resident solution: converged before any iteration, same point
    t2 = srv.submit_batch(bt, x0=False, session=7)
    srv.wait(t2)
    r2 = srv.result(t2)
    assert np.all(r2["status"] == 0) and np.all(r2["iters"] == 0)
    assert np.array_equal(r2["x"], r1["x"])
    srv.close_session(7)
    srv.close()


def test_admission_under_a_tight_budget(T):
    small = [mixed(40, 90 + i, nmax=40) for i in range(12)]
    srv = T.Server(W.QP4, hbm_budget=1 << 20, max_inflight=4, streams=2)
    too_big = mixed(3000, 95, nmax=128)
    with pytest.raises(T.TronError) as e:
        srv.submit_batch(too_big)
    assert e.value.code == 5  # BUSY: can never fit
    tickets = [srv.submit_batch(b) for b in small]
    peak = 0
    while any(srv.poll(t) != 2 for t in tickets):
        peak = max(peak, srv.stats()["device_bytes"])
        time.sleep(0.0005)
    assert peak <= 1 << 20
    for t, b in zip(tickets, small):
        r = srv.result(t)
        assert np.all(r["status"] == 0)
    assert srv.stats()["requests"] == len(small)
    srv.close()


def test_sizes_above_the_lds_limit_are_refused(T):
    bt = W.qp4_batch(2, 200, config_id=101)
    srv = T.Server(W.QP4)
    with pytest.raises(T.TronError) as e:
        srv.submit_batch(bt)
    assert e.value.code == 4  # UNSUPPORTED
    srv.close()


def test_destroy_with_work_pending(T):
    srv = T.Server(W.QP4, max_inflight=2)
    for i in range(6):
        srv.submit_batch(mixed(500, 100 + i))
    srv.close()  # waits for what is on the device, drops the queue, returns


def test_resident_sessions_limit_admission(T):
    """Sessions keep their device memory until closed. Sessions are opened until the next one
    no longer fits; then a request that fits the budget alone but not next to the resident
    sessions is refused at submission with BUSY (instead of waiting for memory that never
    frees), and admitted once the sessions close."""
    budget = 1 << 20
    srv = T.Server(W.QP4, hbm_budget=budget, max_inflight=2, streams=1)
    opened = []
    for k in range(1, 200):
        bt = W.qp4_batch(800, 4, config_id=120 + k)
        try:
            t = srv.submit_batch(bt, session=k)
        except T.TronError as e:
            assert e.code == 5
            break
        srv.wait(t)
        assert np.all(srv.result(t)["status"] == 0)
        opened.append(k)
    assert len(opened) >= 2
    held = srv.stats()["device_bytes"]
    big = W.qp4_batch(1600, 4, config_id=119)   # about half the budget on its own
    with pytest.raises(T.TronError) as e:
        srv.submit_batch(big)
    assert e.value.code == 5
    for k in opened:
        srv.close_session(k)
    assert srv.stats()["device_bytes"] < held
    t2 = srv.submit_batch(big)
    srv.wait(t2)
    assert np.all(srv.result(t2)["status"] == 0)
    srv.close()


def test_cancel_queued_requests(T):
    """A queued request can be taken off the queue. One group on the device at a time, and
    ahead of the request three requests of 1,000 hs45-variant instances at n = 128 from
    random starts (one instance per CU at a time: tens of milliseconds on the device, a few
    megabytes to submit), so the last submission is still queued when it is cancelled. Its
    result call reports the cancellation (BUSY) and releases the ticket, its session can take
    a new request, and every other request completes at the known minimiser (the upper
    corner). A request already finished cannot be cancelled."""
    srv = T.Server(W.HS45M, max_inflight=1, streams=1, coalesce=False)
    heads = [W.hs45m_random_start(1000, 128, config_id=140 + i) for i in range(3)]
    last = W.hs45m_random_start(50, 16, config_id=150)
    tickets = [srv.submit_batch(b) for b in heads]
    t_last = srv.submit_batch(last, session=7)
    srv.cancel(t_last)
    srv.wait(t_last)
    with pytest.raises(T.TronError) as e:
        srv.result(t_last)
    assert e.value.code == 5 and "cancelled" in str(e.value)
    with pytest.raises(T.TronError):
        srv.result(t_last)  # the ticket is released
    for t, b in zip(tickets, heads):
        srv.wait(t)
        r = srv.result(t)
        assert np.all(r["status"] == 0) and np.array_equal(r["x"], b.hi)
    t2 = srv.submit_batch(last, session=7)  # the session is free again
    srv.wait(t2)
    r2 = srv.result(t2)
    assert np.all(r2["status"] == 0) and np.array_equal(r2["x"], last.hi)
    t3 = srv.submit_batch(last)
    srv.wait(t3)
    with pytest.raises(T.TronError) as e:
        srv.cancel(t3)
    assert e.value.code == 5
    srv.result(t3)
    srv.close()


def test_random_soak_two_submitters(T):
    """Two threads submit 60 requests each (sizes drawn from a seed: 1-800 instances, n log-
    uniform in [2, 96]) to a server with two groups in flight and coalescing, cancelling every
    seventh right after submission; a third thread collects. Every request ends either with
    results bitwise equal to the batch API's for the same instances, or, if its cancel came
    before admission, with the cancellation; nothing stays pending, and the server's device
    memory returns to zero."""
    import torch
    srv = T.Server(W.QP4, hbm_budget=256 << 20, max_inflight=2, streams=2, coalesce=True)
    lock = threading.Lock()
    reqs, order, results = {}, [], {}
    done_submitting = threading.Event()

    def submitter(tid):
        r = np.random.default_rng(1000 + tid)
        for k in range(60):
            B = int(np.exp(r.uniform(0, np.log(800))))
            bt = mixed(B, 5000 + 100 * tid + k, nmax=96)
            t = srv.submit_batch(bt)
            with lock:
                reqs[t] = bt
                order.append(t)
            if k % 7 == 3:
                try:
                    srv.cancel(t)
                except T.TronError:
                    pass

    def collector():
        i = 0
        while True:
            with lock:
                t = order[i] if i < len(order) else None
            if t is None:
                if done_submitting.is_set():
                    with lock:
                        if i >= len(order):
                            return
                    continue
                time.sleep(0.001)
                continue
            srv.wait(t, 30.0)
            try:
                results[t] = srv.result(t)
            except T.TronError as e:
                assert "cancel" in str(e), e
                results[t] = None
            i += 1

    subs = [threading.Thread(target=submitter, args=(i,)) for i in range(2)]
    col = threading.Thread(target=collector)
    col.start()
    for th in subs:
        th.start()
    for th in subs:
        th.join()
    done_submitting.set()
    col.join(120)
    assert not col.is_alive()
    assert set(results) == set(reqs)
    assert srv.stats()["device_bytes"] == 0
    srv.close()
    checked = 0
    for t, res in results.items():
        if res is None:
            continue
        bt = reqs[t]
        h = T.Batch(W.QP4, bt.n)
        x, f, st, it = h.solve(*T.to_device(bt))
        torch.cuda.synchronize()
        assert np.array_equal(x.cpu().numpy(), res["x"]) and np.array_equal(f.cpu().numpy(), res["f"]), t
        assert np.array_equal(st.cpu().numpy(), res["status"]), t
        h.close()
        checked += 1
    assert checked >= 100
