"""GPU tests of the serving loop (tc_server_*): every result of a mixed
request stream is bit-identical to the same product computed alone and to
Python's integer product; admission limits and draining behave as stated."""
import time

import numpy as np
import pytest

from paper_1602_02740_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def T():
    from paper_1602_02740_amd import toom
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    toom.init()
    return toom


def wait_all(srv, tickets, timeout_s=120.0):
    res = {}
    deadline = time.monotonic() + timeout_s
    while len(res) < len(tickets):
        for t in tickets:
            if t not in res:
                r = srv.poll(t)
                if r is not None:
                    res[t] = r
        assert time.monotonic() < deadline, f"{len(tickets) - len(res)} requests not done"
        time.sleep(0.0005)
    return res


def test_mixed_stream_equals_alone(T):
    # Zipf-distributed power-of-two sizes (capped for test time) plus ragged
    # sizes; a budget of a few products forces admission to wait for memory
    sizes = [int(x) for x in I.zipf_sizes(48, seed=41, ranks=10)]
    sizes += [37, 37, 37, 1000, 1000, 4097, 5, 5]
    budget = 3 * T.workspace_bytes(max(sizes), max(sizes))
    ops = []
    for i, n in enumerate(sizes):
        u = I.random_limbs(4100 + i, 1, n)
        v = I.random_limbs(4100 + i, 2, n)
        if i % 7 == 3:
            v = u.copy()  # squaring through distinct buffers
        ops.append((u, v))
    dus = [(T.to_device(u), T.to_device(v)) for u, v in ops]
    outs = [T.empty(2 * n) for n in sizes]
    with T.Server(hbm_budget=budget, max_inflight=32, streams=3, max_batch=8) as srv:
        tickets = [srv.submit(du, dv, w) for (du, dv), w in zip(dus, outs)]
        res = wait_all(srv, tickets)
        st = srv.stats()
    assert all(r["status"] == 0 for r in res.values())
    assert all(r["submit_us"] <= r["start_us"] <= r["finish_us"] for r in res.values())
    assert st["completed"] == len(sizes) and st["submitted"] == len(sizes)
    assert 0 < st["p50_us"] <= st["p99_us"]
    assert st["batches"] <= len(sizes)
    for (u, v), (du, dv), w in zip(ops, dus, outs):
        alone = T.mul(du, dv)
        T.sync()
        got = T.to_host(w)
        np.testing.assert_array_equal(got, T.to_host(alone))
        assert I.to_int(got) == I.to_int(u) * I.to_int(v)


def test_unbalanced_and_square_requests(T):
    """Requests of unequal lengths (cut into balanced pieces) and squares
    (u and v the same tensor) batched with ordinary ones: each result equals
    Python's integer product."""
    shapes = [(9000, 1000), (300, 7000), (4096, 4096), (20000, 3), (3000, 3000),
              (1500, 700), (64, 64), (2, 1)]
    reqs = []
    for i, (a, b) in enumerate(shapes):
        u = I.random_limbs(4200 + i, 1, a)
        v = u if a == b and i % 2 == 0 else I.random_limbs(4200 + i, 2, b)
        du = T.to_device(u)
        dv = du if v is u else T.to_device(v)
        reqs.append((u, v, du, dv, T.empty(a + b)))
    with T.Server(max_inflight=16, streams=2, max_batch=4) as srv:
        tickets = [srv.submit(du, dv, w) for _, _, du, dv, w in reqs]
        res = wait_all(srv, tickets)
    assert all(r["status"] == 0 for r in res.values())
    for u, v, _, _, w in reqs:
        assert I.to_int(T.to_host(w)) == I.to_int(u) * I.to_int(v)


def test_results_survive_interleaved_submits(T):
    # requests submitted while earlier ones run, polled in random order
    rng = np.random.default_rng(5)
    with T.Server(streams=2, max_batch=4) as srv:
        live = {}
        for i in range(40):
            n = int(rng.choice([32, 64, 300, 2048, 9000]))
            u = I.random_limbs(700 + i, 1, n)
            v = I.random_limbs(700 + i, 2, n)
            du, dv, w = T.to_device(u), T.to_device(v), T.empty(2 * n)
            live[srv.submit(du, dv, w)] = (u, v, w)
            if i % 5 == 4:
                time.sleep(0.001)
        keys = list(live)
        rng.shuffle(keys)
        res = wait_all(srv, keys)
    for t, (u, v, w) in live.items():
        assert res[t]["status"] == 0
        assert I.to_int(T.to_host(w)) == I.to_int(u) * I.to_int(v)


def test_caller_allocates_while_server_compiles(T):
    # The caller's thread makes fresh device allocations (each one asks the
    # runtime whether the legacy stream is capturing) between submits, while
    # the server thread compiles and captures a plan for every new size and
    # the submits plan workspace sizes (which may add divisor-table entries)
    # on the caller's thread: no library call may leave the caller's thread
    # in an error state or touch the legacy stream.
    sizes = [1 << k for k in range(5, 19)]
    with T.Server(streams=4, max_batch=8) as srv:
        live = {}
        for i, n in enumerate(sizes):
            u = I.random_limbs(900 + i, 1, n)
            v = I.random_limbs(900 + i, 2, n)
            du, dv = T.to_device(u), T.to_device(v)
            # odd sizes defeat the caching allocator: every call allocates
            w = torch.empty(2 * n + 2 * i + 1, dtype=torch.int32, device="cuda")[: 2 * n]
            pad = torch.empty((1 << 21) + 64 * i + 1, dtype=torch.int32, device="cuda")
            del pad
            live[srv.submit(du, dv, w)] = (u, v, du, dv, w)
        res = wait_all(srv, list(live))
    for t, (u, v, du, dv, w) in live.items():
        assert res[t]["status"] == 0
        if u.size <= 1 << 14:
            assert I.to_int(T.to_host(w)) == I.to_int(u) * I.to_int(v)
        else:
            assert torch.equal(w, T.mul(du, dv))


def test_admission_limits(T):
    n = 4096
    u = T.to_device(I.random_limbs(9, 1, n))
    w = T.empty(2 * n)
    # a request larger than the whole budget is refused outright
    with T.Server(hbm_budget=1024) as srv:
        with pytest.raises(T.ToomError) as e:
            srv.submit(u, u, w)
        assert e.value.code == -2
        assert srv.stats()["rejected"] == 1
    # a full queue answers TC_ERR_AGAIN; the queued work still completes
    small = [T.to_device(I.random_limbs(10 + i, 1, 64)) for i in range(8)]
    outs = [T.empty(128) for _ in range(8)]
    with T.Server(max_queued=2, max_inflight=1, streams=1) as srv:
        tickets, again = [], 0
        for x, o in zip(small, outs):
            try:
                tickets.append(srv.submit(x, x, o))
            except T.ToomError as err:
                assert err.code == -4
                again += 1
        res = wait_all(srv, tickets)
        assert all(r["status"] == 0 for r in res.values())
    assert again + len(tickets) == 8
    # unknown tickets are invalid; a ticket is reported once
    with T.Server() as srv:
        with pytest.raises(T.ToomError):
            srv.poll(12345)
        t = srv.submit(small[0], small[0], outs[0])
        wait_all(srv, [t])
        with pytest.raises(T.ToomError):
            srv.poll(t)


def test_destroy_drains_queue(T):
    n = 20000
    u = I.random_limbs(77, 1, n)
    v = I.random_limbs(77, 2, n)
    du, dv = T.to_device(u), T.to_device(v)
    outs = [T.empty(2 * n) for _ in range(6)]
    srv = T.Server(streams=2, max_batch=2)
    for w in outs:
        srv.submit(du, dv, w)
    srv.close()  # returns after every request has completed
    torch.cuda.synchronize()
    want = I.to_int(u) * I.to_int(v)
    for w in outs:
        assert I.to_int(T.to_host(w)) == want
