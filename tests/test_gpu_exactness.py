"""The device exactness checks fire, through the C ABI, and only where the
arithmetic went wrong.

Section 3's divisions are exact for values that come from products, and
section 4's even-odd combine halves even values; values that no product can
give break one of those, and the kernels must report it (TC_ERR_INEXACT)
rather than return a wrong product.  The checks only set an error word:
every kernel still runs to its end."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1602_02740_amd import inputs as I
from tests.helpers import signed_to_sm, sm_to_signed

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def T():
    """The library in strict mode: every coefficient of every level in its
    own exact step, so a corrupted point product is caught wherever it is."""
    from paper_1602_02740_amd import toom
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    toom.init()
    toom.sync()  # start from a clean sticky word
    toom.set_strict(True)
    yield toom
    toom.set_strict(False)


def point_products(B, var, bl, seed):
    """Signed point products (Python ints) of two random operands of B blocks."""
    n = B * bl
    u, v = I.random_limbs(seed, 1, n), I.random_limbs(seed, 2, n)
    nout = bl + oracle.growth_limbs(B, var)
    ue, us = oracle.eval_points(B, var, u, bl, nout)
    ve, vs = oracle.eval_points(B, var, v, bl, nout)
    y = []
    for a, sa, b, sb in zip(ue, us, ve, vs):
        p = I.to_int(a) * I.to_int(b)
        y.append(-p if (sa ^ sb) else p)
    return y, 2 * nout


def run_interp(T, y, ny, B, var, nw):
    mag, sign = signed_to_sm(y, ny)
    return T.interp(T.to_device(mag.ravel()), torch.from_numpy(sign.astype(np.uint8)).cuda(),
                    B, var, nw)


def expect_inexact(T):
    with pytest.raises(T.ToomError) as e:
        T.sync()
    assert e.value.code == T.TC_ERR_INEXACT


@pytest.mark.parametrize("B,bl", [(2, 5), (3, 40), (4, 300), (16, 64), (32, 60)])
def test_interp_flags_odd_halving(T, B, bl):
    """One bit flipped in y(+1): (y(+1) + y(-1)) / 2 is no longer exact."""
    y, ny = point_products(B, 0, bl, 500 + B)
    nw = 2 * bl + 1
    bad = list(y)
    bad[1] ^= 1
    run_interp(T, bad, ny, B, 0, nw)
    expect_inexact(T)
    # the word was cleared: a clean call afterwards reports nothing, and is right
    got = T.to_host(run_interp(T, y, ny, B, 0, nw)).reshape(2 * B - 1, nw)
    T.sync()
    mag, sign = signed_to_sm(y, ny)
    np.testing.assert_array_equal(got, oracle.interp(B, 0, mag, sign, nw))


@pytest.mark.parametrize("B,bl", [(3, 40), (4, 300), (16, 64)])
def test_interp_flags_division_remainder(T, B, bl):
    """y(+2) and y(-2) both raised by one: the combine stays exact (their sum
    is even), but the even polynomial's divided difference over the nodes
    X = 1 and X = 4 is no longer divisible by 4 - 1 = 3."""
    y, ny = point_products(B, 0, bl, 600 + B)
    bad = list(y)
    bad[3] += 1
    bad[4] += 1
    run_interp(T, bad, ny + 1, B, 0, 2 * bl + 1)
    expect_inexact(T)
    run_interp(T, y, ny, B, 0, 2 * bl + 1)
    T.sync()


def test_interp_flags_infinity_variant(T):
    y, ny = point_products(3, 1, 40, 700)
    bad = list(y)
    bad[3] += 1  # W(2) off by one: the cubic's divided differences divide by 2 and 3
    run_interp(T, bad, ny + 1, 3, 1, 81)
    expect_inexact(T)


def test_recompose_flags_overflow(T):
    """Coefficients whose sum does not fit nout limbs."""
    B, bl = 3, 50
    nw = 2 * bl + 1
    w = np.zeros((2 * B - 1, nw), dtype=np.uint32)
    w[0, 0] = 7
    nout = 2 * B * bl
    T.recompose(T.to_device(w.ravel()), B, bl, nout)
    T.sync()  # fits
    w[2 * B - 2, nw - 1] = 1  # limb (2B-2) bl + 2 bl > nout
    T.recompose(T.to_device(w.ravel()), B, bl, nout)
    expect_inexact(T)
    w[2 * B - 2, nw - 1] = 0
    w[2 * B - 2, 2 * bl - 1] = 0xFFFFFFFF
    w[2 * B - 3, 2 * bl - 1] = 0xFFFFFFFF  # carries into limb nout
    w[2 * B - 2, bl - 1] = 0xFFFFFFFF
    T.recompose(T.to_device(w.ravel()), B, bl, 2 * B * bl - 1)
    expect_inexact(T)


def test_fault_hook_single_product(T):
    """A flipped product bit between the leaves and the top interpolation of
    tc_mul is reported; with the hook off the same product is right again."""
    n = 20000
    u, v = I.random_limbs(710, 1, n), I.random_limbs(710, 2, n)
    du, dv = T.to_device(u), T.to_device(v)
    try:
        for plan in (None, T.Plan.make([16, 3]), T.Plan.make([3, 3, 3]), T.Plan.make([2, 3, 3])):
            T.debug_fault(0)
            T.mul(du, dv, plan=plan)
            expect_inexact(T)
    finally:
        T.debug_fault(-1)
    w = T.mul(du, dv)
    T.sync()
    assert I.to_int(T.to_host(w)) == I.to_int(u) * I.to_int(v)


def test_batch_status_per_item(T):
    """tc_mul_batch with a status array: only the faulted item reports
    TC_ERR_INEXACT, the others TC_OK with correct products, the sticky word
    stays clear; device, pinned and pageable host status arrays."""
    sizes = [5000, 3000, 20000, 700, 9000]
    us = [I.random_limbs(720, i, n) for i, n in enumerate(sizes)]
    vs = [I.random_limbs(721, i, n) for i, n in enumerate(sizes)]
    du, dv = [T.to_device(u) for u in us], [T.to_device(v) for v in vs]
    k = 2
    try:
        T.debug_fault(k)
        for kind in ("device", "pinned", "pageable"):
            if kind == "device":
                st = torch.full((len(sizes),), 99, dtype=torch.int32, device="cuda")
            elif kind == "pinned":
                st = torch.full((len(sizes),), 99, dtype=torch.int32).pin_memory()
            else:
                st = torch.full((len(sizes),), 99, dtype=torch.int32)
            outs = T.mul_batch(du, dv, status=st)
            T.sync()  # the sticky word is not touched
            got = st.cpu().numpy().tolist()
            want = [0] * len(sizes)
            want[k] = T.TC_ERR_INEXACT
            assert got == want, kind
            for i, w in enumerate(outs):
                if i != k:
                    assert I.to_int(T.to_host(w)) == I.to_int(us[i]) * I.to_int(vs[i])
        # without a status array the failure goes to the sticky word
        T.mul_batch(du, dv)
        expect_inexact(T)
    finally:
        T.debug_fault(-1)
    st = torch.full((len(sizes),), 99, dtype=torch.int32, device="cuda")
    outs = T.mul_batch(du, dv, status=st)
    T.sync()
    assert st.cpu().numpy().tolist() == [0] * len(sizes)
    for u, v, w in zip(us, vs, outs):
        assert I.to_int(T.to_host(w)) == I.to_int(u) * I.to_int(v)


def test_batch_rejects_cross_item_aliasing(T):
    a = T.empty(1000)
    b = T.empty(1000)
    u = T.to_device(I.random_limbs(730, 1, 200))
    v = T.to_device(I.random_limbs(730, 2, 200))
    descs = (T.MulDesc * 2)()
    descs[0] = T.MulDesc(a.data_ptr(), u.data_ptr(), 200, v.data_ptr(), 200)
    descs[1] = T.MulDesc(a.data_ptr() + 4 * 300, u.data_ptr(), 200, v.data_ptr(), 200)
    assert T.lib().tc_mul_batch(descs, 2, None, None) == -1
    descs[1] = T.MulDesc(b.data_ptr(), a.data_ptr() + 4 * 100, 200, v.data_ptr(), 200)
    assert T.lib().tc_mul_batch(descs, 2, None, None) == -1
    descs[1] = T.MulDesc(b.data_ptr(), u.data_ptr(), 200, v.data_ptr(), 200)
    assert T.lib().tc_mul_batch(descs, 2, None, None) == 0
    T.sync()


def test_server_reports_status_on_the_faulted_ticket(T):
    """The serving loop charges a device exactness failure to exactly the
    request that had it: with the hook on item 0 of every batch, the one
    request with a Toom level fails, the single-leaf requests (no
    interpolation, so nothing to corrupt) succeed."""
    n_bad, n_ok = 6000, 1000
    u = T.to_device(I.random_limbs(740, 1, n_bad))
    v = T.to_device(I.random_limbs(740, 2, n_bad))
    small = [(I.random_limbs(741, i, n_ok), I.random_limbs(742, i, n_ok)) for i in range(6)]
    try:
        T.debug_fault(0)
        with T.Server(streams=2, max_batch=8) as srv:
            tickets = []
            outs = []
            for i, (a, b) in enumerate(small[:3]):
                o = T.empty(2 * n_ok)
                tickets.append(srv.submit(T.to_device(a), T.to_device(b), o))
                outs.append(o)
            bad_out = T.empty(2 * n_bad)
            bad = srv.submit(u, v, bad_out)
            for a, b in small[3:]:
                o = T.empty(2 * n_ok)
                tickets.append(srv.submit(T.to_device(a), T.to_device(b), o))
                outs.append(o)
            res = {}
            import time
            t0 = time.time()
            while len(res) < len(tickets) + 1 and time.time() - t0 < 60:
                for t in tickets + [bad]:
                    if t not in res:
                        r = srv.poll(t)
                        if r is not None:
                            res[t] = r
                time.sleep(0.001)
        assert res[bad]["status"] == T.TC_ERR_INEXACT
        for t, o, (a, b) in zip(tickets, outs, small):
            assert res[t]["status"] == 0
            assert I.to_int(T.to_host(o)) == I.to_int(a) * I.to_int(b)
    finally:
        T.debug_fault(-1)
    T.sync()  # the server never touches the sticky word


def test_interp_half_points_flags_a_flipped_bit(T):
    """The fixed-n interpolation of the 0, +-1, +-2, 1/2, infinity points
    divides each coefficient's row exactly; a flipped bit in any of the five
    non-trivial point products breaks one of those divisions."""
    B, bl = 4, 50
    y, ny = point_products_half(bl, 770)
    for k in range(1, 6):
        bad = list(y)
        bad[k] ^= 1
        run_interp(T, bad, ny, B, 2, 2 * bl + 1)
        expect_inexact(T)
    run_interp(T, y, ny, B, 2, 2 * bl + 1)
    T.sync()


def point_products_half(bl, seed):
    B = 4
    n = B * bl
    u, v = I.random_limbs(seed, 1, n), I.random_limbs(seed, 2, n)
    nout = bl + oracle.growth_limbs(B, oracle.VAR_HALF)
    ue, us = oracle.eval_points(B, oracle.VAR_HALF, u, bl, nout)
    ve, vs = oracle.eval_points(B, oracle.VAR_HALF, v, bl, nout)
    y = []
    for a, sa, b, sb in zip(ue, us, ve, vs):
        p = I.to_int(a) * I.to_int(b)
        y.append(-p if (sa ^ sb) else p)
    return y, 2 * nout
