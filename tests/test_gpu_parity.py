"""GPU parity: every phase and the whole product against the CPU oracle,
bit for bit (the arithmetic is exact, so the tolerance is zero)."""
import numpy as np
import pytest

import oracle
from paper_1602_02740_amd import inputs as I
from tests.helpers import residue_np

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def T():
    from paper_1602_02740_amd import toom
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    toom.init()
    return toom


def dev(a):
    from paper_1602_02740_amd import toom
    return toom.to_device(a)


def host(t):
    from paper_1602_02740_amd import toom
    return toom.to_host(t)


def check_clean(T):
    T.sync()  # raises on a device exactness error


# ------------------------------------------------------------------ leaves

# widths up to 32 run on the vector ALUs; the wider ones reach every
# band/diagonal tiling of the matrix-core leaf: (SM, DM) = (1,2) 33..137,
# (2,2) 256, 257, (2,3) 343, (3,3) 512, 513, (3,4) 700, (4,4) 767, (4,5) 900,
# (5,5) 1024, (5,6) 1216, (6,6) 1279, (6,7) 1500, (7,7) 1535, (7,8) 1700,
# (8,8) 1791, (8,9) 1900, (9,9) 2048
@pytest.mark.parametrize("n", [1, 2, 3, 17, 32, 33, 63, 64, 65, 100, 137, 256, 257, 343,
                               512, 513, 700, 767, 900, 1024, 1216, 1279, 1500, 1535, 1700,
                               1791, 1900, 2048])
def test_school_leaves(T, n):
    count = 37
    rng = np.random.default_rng(n)
    U = rng.integers(0, 2 ** 32, size=(count, n), dtype=np.uint64).astype(np.uint32)
    V = rng.integers(0, 2 ** 32, size=(count, n), dtype=np.uint64).astype(np.uint32)
    U[0] = 0xFFFFFFFF
    V[0] = 0xFFFFFFFF
    U[1] = 0
    if n > 2:
        U[2] = rng.integers(0, 2, size=n, dtype=np.uint64).astype(np.uint32) * np.uint32(0x7F7F7F7F)
        V[2] = 0x80808080
        V[3] = 0x7FFFFFFF
    P = host(T.school(dev(U.ravel()), dev(V.ravel()), n, count)).reshape(count, 2 * n)
    check_clean(T)
    for i in range(count):
        np.testing.assert_array_equal(P[i], oracle.mul_school(U[i], V[i]), err_msg=f"leaf {i}")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 9, 16, 17, 31, 32, 33, 100])
def test_school_squares(T, n):
    # u and v at one address: leaves of up to 32 limbs take the squaring
    # path (pairs below the diagonal once, doubled, plus the diagonal squares)
    count = 29
    rng = np.random.default_rng(1000 + n)
    U = rng.integers(0, 2 ** 32, size=(count, n), dtype=np.uint64).astype(np.uint32)
    U[0] = 0xFFFFFFFF
    U[1] = 0
    U[2, :] = 0
    U[2, -1] = 0x80000000
    if n > 1:
        U[3] = 0xFFFFFFFF
        U[3, 0] = 1
    du = dev(U.ravel())
    P = host(T.school(du, du, n, count)).reshape(count, 2 * n)
    check_clean(T)
    for i in range(count):
        np.testing.assert_array_equal(P[i], oracle.mul_school(U[i], U[i]), err_msg=f"leaf {i}")


# ------------------------------------------------------------------ phases

@pytest.mark.parametrize("B,var,n", [(2, 0, 9), (3, 0, 1000), (3, 1, 1024), (4, 0, 4000),
                                     (7, 0, 777), (16, 0, 16 * 600 + 5), (16, 0, 40000),
                                     (32, 0, 32 * 100 - 3)])
def test_eval_parity(T, B, var, n):
    for u in (I.random_limbs(11, B + n, n), I.all_ones(n)):
        bl = oracle.block_limbs(n, B)
        nout = bl + oracle.growth_limbs(B, var)
        want, wsign = oracle.eval_points(B, var, u, bl, nout)
        got, gsign = T.eval_points(dev(u), B, var, bl, nout)
        check_clean(T)
        np.testing.assert_array_equal(host(got).reshape(want.shape), want)
        np.testing.assert_array_equal(gsign.cpu().numpy().astype(np.int8), wsign)


def products_for(B, var, bl, seed, ones=False):
    """Point products of two random operands of B blocks (magnitudes + signs)."""
    n = B * bl
    u = I.all_ones(n) if ones else I.random_limbs(seed, 1, n)
    v = I.all_ones(n) if ones else I.random_limbs(seed, 2, n)
    nout = bl + oracle.growth_limbs(B, var)
    ue, us = oracle.eval_points(B, var, u, bl, nout)
    ve, vs = oracle.eval_points(B, var, v, bl, nout)
    y = np.stack([oracle.mul_school(a, b) for a, b in zip(ue, ve)])
    sign = (us ^ vs) * np.array([int(r.any()) for r in y], dtype=np.int8)
    return y, sign.astype(np.int8)


@pytest.mark.parametrize("B,var,bl", [(2, 0, 5), (3, 0, 40), (3, 1, 40), (4, 0, 300),
                                      (8, 0, 70), (16, 0, 64), (16, 0, 300), (32, 0, 60)])
def test_interp_parity(T, B, var, bl):
    for ones in (False, True):
        y, sign = products_for(B, var, bl, 100 + B, ones)
        nw = 2 * bl + 1
        want = oracle.interp(B, var, y, sign, nw)
        got = T.interp(dev(y.ravel()), torch.from_numpy(sign.astype(np.uint8)).cuda(), B, var, nw)
        check_clean(T)
        np.testing.assert_array_equal(host(got).reshape(want.shape), want)


@pytest.mark.parametrize("B,bl", [(2, 3), (3, 100), (16, 50), (32, 300)])
def test_recompose_parity(T, B, bl):
    rng = np.random.default_rng(B)
    nw = 2 * bl + 1
    w = rng.integers(0, 2 ** 32, size=(2 * B - 1, nw), dtype=np.uint64).astype(np.uint32)
    w[:, -1] &= np.uint32(15)
    nout = 2 * B * bl + 2
    want = oracle.recompose(B, bl, w, nout)
    got = host(T.recompose(dev(w.ravel()), B, bl, nout))
    check_clean(T)
    np.testing.assert_array_equal(got, want)


# ------------------------------------------------------------------ products

def gpu_mul(T, u, v, plan=None):
    w = host(T.mul(dev(u), dev(v), plan=plan))
    check_clean(T)
    return w


@pytest.mark.parametrize("case", ["uniform", "all_ones", "single_bit"])
@pytest.mark.parametrize("variant", [1, 0])
def test_config1_toom3(T, case, variant):
    """1024-limb operands, one 3-way level (points 0, 1, -1, 2, inf, or the
    paper's 0, +-1, +-2), schoolbook leaves of 343 limbs."""
    u, v = {"uniform": I.config1_uniform, "all_ones": I.config1_all_ones,
            "single_bit": I.config1_single_bit}[case]()
    plan = T.Plan.make([3], [variant])
    want = oracle.mul_toom(u, v, [3], [variant])
    np.testing.assert_array_equal(want, oracle.mul_school(u, v))
    np.testing.assert_array_equal(gpu_mul(T, u, v, plan), want)


def leaf_width(n, Bs):
    for B in Bs:
        n = oracle.block_limbs(n, B) + oracle.growth_limbs(B)
    return n


def max_width_for_leaf(Bs, leaf, cap=40000):
    """Largest operand width <= cap whose plan keeps leaves <= leaf limbs."""
    lo, hi = 1, cap
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if leaf_width(mid, Bs) <= leaf:
            lo = mid
        else:
            hi = mid - 1
    return lo


@pytest.mark.parametrize("Bs", [[2], [3], [4], [5], [8], [16], [32], [16, 3], [3, 3, 2],
                                [32, 2], [4, 4, 4], [3, 2, 2, 2]])
def test_plans_against_oracle(T, Bs):
    rng = np.random.default_rng(sum(Bs))
    nmax = max_width_for_leaf(Bs, 512)
    for n in (int(rng.integers(nmax // 4, nmax // 2)), nmax):
        u, v = I.random_limbs(31, n, n), I.random_limbs(32, n, n)
        want = oracle.mul_toom(u, v, Bs)
        np.testing.assert_array_equal(gpu_mul(T, u, v, T.Plan.make(Bs)), want)


@pytest.mark.parametrize("Bs", [[16, 3], [3, 3, 2], [4, 16]])
def test_chunk_scales_against_oracle(T, Bs):
    """Every chunk scale of the linear passes (the tile shape the autotuner
    picks) gives the oracle's product, across several chunks and a ragged
    tail."""
    n = max_width_for_leaf(Bs, 512) - 37
    u, v = I.random_limbs(33, n, n), I.random_limbs(34, n, n)
    want = oracle.mul_toom(u, v, Bs)
    for ch in (-2, -1, 1, 2):
        np.testing.assert_array_equal(gpu_mul(T, u, v, T.Plan.make(Bs, chunk=ch)), want,
                                      err_msg=f"chunk {ch}")


def test_default_plan_sizes_and_ragged(T):
    rng = np.random.default_rng(7)
    sizes = [1, 2, 5, 64, 159, 160, 161, 511, 512, 513, 1000, 4095, 4096, 12345, 70000]
    for n in sizes:
        m = max(1, n - int(rng.integers(0, max(1, n // 3))))
        u, v = I.random_limbs(41, n, n), I.random_limbs(42, n, m)
        want = oracle.mul_toom(u, v, [])  if n * m < 4_000_000 else \
            oracle.mul_toom(u, v, [3, 3, 3, 3])
        np.testing.assert_array_equal(gpu_mul(T, u, v), want, err_msg=f"{n}x{m}")


def test_edge_operands(T):
    n = 3000
    cases = [(I.all_ones(n), I.all_ones(n)), (np.zeros(n, np.uint32), I.random_limbs(1, 5, n)),
             (I.single_bit(n, 32 * n - 1), I.single_bit(n, 0)),
             (I.sparse_limbs(2, 3, n), I.random_limbs(2, 4, n))]
    for u, v in cases:
        want = oracle.mul_school(u, v)
        np.testing.assert_array_equal(gpu_mul(T, u, v), want)
        np.testing.assert_array_equal(gpu_mul(T, u, v, T.Plan.make([16, 3])), want)


@pytest.mark.parametrize("Bs", [[3], [16], [16, 3], [3, 3], [32], [2]])
def test_plans_with_matrix_core_leaves(T, Bs):
    """Plans whose leaves are wider than 512 limbs (matrix-core schoolbook)."""
    rng = np.random.default_rng(len(Bs) * 7 + Bs[0])
    nmax = max_width_for_leaf(Bs, 2048, cap=200000)
    for n in (nmax, int(rng.integers(nmax // 2, nmax))):
        if leaf_width(n, Bs) <= 512:
            continue
        u, v = I.random_limbs(51, n, n), I.random_limbs(52, n, n)
        want = oracle.mul_toom(u, v, Bs, threads=8)
        np.testing.assert_array_equal(gpu_mul(T, u, v, T.Plan.make(Bs)), want)


def test_squaring_alias(T):
    u = I.random_limbs(3, 3, 9000)
    du = dev(u)
    w = host(T.mul(du, du))
    check_clean(T)
    np.testing.assert_array_equal(w, oracle.mul_toom(u, u, [3, 3, 3]))


def square(T, u, plan=None):
    du = dev(u)
    w = host(T.mul(du, du, plan=plan))
    check_clean(T)
    return w


# u * u with one evaluation per node (children of a square are squares)
@pytest.mark.parametrize("Bs,n", [([], 7), ([], 1500), ([3], 3000), ([2, 3], 5001),
                                  ([16, 3], 60000), ([32], 20000), ([3, 3], 4000)])
def test_squares(T, Bs, n):
    u = I.random_limbs(91, len(Bs), n)
    want = oracle.mul_toom(u, u, Bs, threads=8)
    np.testing.assert_array_equal(square(T, u, T.Plan.make(Bs)), want)
    np.testing.assert_array_equal(square(T, u), want)
    # the same operand copied to a second buffer takes the general path
    np.testing.assert_array_equal(gpu_mul(T, u, u.copy()), want)


def test_square_edge_operands(T):
    n = 5000
    for u in (I.all_ones(n), I.single_bit(n, 32 * n - 1), I.sparse_limbs(92, 1, n),
              np.zeros(n, np.uint32)):
        want = oracle.mul_school(u, u)
        np.testing.assert_array_equal(square(T, u), want)
        np.testing.assert_array_equal(square(T, u, T.Plan.make([16, 3])), want)


def test_squares_in_batch(T):
    """Squares and products of the same sizes in one batch: each item keeps
    its own kind; a square reads only its u entry."""
    sizes = [3000, 3000, 800, 800, 20000, 9000]
    us = [I.random_limbs(93, i, n) for i, n in enumerate(sizes)]
    vs = [I.random_limbs(94, i, n) for i, n in enumerate(sizes)]
    du = [dev(u) for u in us]
    dv = [du[i] if i % 2 == 0 else dev(vs[i]) for i in range(len(sizes))]
    outs = T.mul_batch(du, dv)
    check_clean(T)
    for i, w in enumerate(outs):
        v = us[i] if i % 2 == 0 else vs[i]
        assert I.to_int(host(w)) == I.to_int(us[i]) * I.to_int(v)


def test_square_full_size(T):
    """A 2^19-limb square with the plan of the 2^19 x 2^19 product."""
    n = 1 << 19
    u = I.random_limbs(95, 1, n)
    got = square(T, u, T.Plan.make([16, 3, 3, 3]))
    assert I.to_int(got) == I.to_int(u) ** 2


@pytest.mark.parametrize("plan", [[16, 3, 3, 3, 3, 3], [16, 3, 3, 3]])
def test_config2_full_size(T, plan):
    """2^19 x 2^19 limbs, 16-way top level then 3-way levels (vector-ALU
    leaves of 137 limbs, or the benchmark's matrix-core leaves of 1215): the
    whole product against the oracle, plus residues."""
    u, v = I.config2()
    got = gpu_mul(T, u, v, T.Plan.make(plan))
    want = oracle.mul_toom(u, v, plan, threads=8)
    np.testing.assert_array_equal(got, want)
    for p in (2147483647, 4294967291):
        assert residue_np(got, p) == residue_np(u, p) * residue_np(v, p) % p


# (nu, nv) pairs with max >= 2 min: the longer operand is cut into pieces as
# long as the shorter; the cases cover a last piece that is full, one limb,
# or short enough to be cut again (nested), both operand orders, pieces on
# the vector leaf, on the matrix-core leaf and through Toom levels
UNBALANCED = [(2, 1), (1, 5), (3, 1), (100, 1), (1, 1000), (64, 32), (65, 32), (4800, 2400),
              (5000, 2400), (7201, 2400), (70000, 3000), (3000, 70000), (40000, 33),
              (131149, 5000), (1 << 20, 64), (300001, 40000)]


@pytest.mark.parametrize("nu,nv", UNBALANCED)
def test_unbalanced_products(T, nu, nv):
    u, v = I.random_limbs(81, 1, nu), I.random_limbs(81, 2, nv)
    got = gpu_mul(T, u, v)
    assert I.to_int(got) == I.to_int(u) * I.to_int(v)
    if nu * nv <= 4_000_000:
        np.testing.assert_array_equal(got, oracle.mul_school(u, v))


def test_unbalanced_edge_operands(T):
    """All-ones operands carry through every limb of the final sum; a zero
    shorter operand and single bits at the far ends."""
    a, s = 10007, 3000
    cases = [(I.all_ones(a), I.all_ones(s)), (I.random_limbs(82, 1, a), np.zeros(s, np.uint32)),
             (I.single_bit(a, 32 * a - 1), I.single_bit(s, 32 * s - 1)),
             (I.sparse_limbs(82, 2, a), I.all_ones(s))]
    for u, v in cases:
        want = oracle.mul_school(u, v)
        np.testing.assert_array_equal(gpu_mul(T, u, v), want)
        np.testing.assert_array_equal(gpu_mul(T, v, u), want)


def test_unbalanced_batch_and_workspace(T):
    """Unbalanced items in a batch (merged into the other items' launches)
    equal their single products; the workspace of a cut product is below
    that of the zero-padded balanced plan for max(nu, nv)."""
    pairs = [(9000, 1000), (777, 5000), (4096, 4096), (20000, 2), (3001, 1500)]
    us = [I.random_limbs(83, i, a) for i, (a, _) in enumerate(pairs)]
    vs = [I.random_limbs(84, i, b) for i, (_, b) in enumerate(pairs)]
    outs = T.mul_batch([dev(u) for u in us], [dev(v) for v in vs])
    check_clean(T)
    for u, v, w in zip(us, vs, outs):
        np.testing.assert_array_equal(host(w), gpu_mul(T, u, v))
        assert I.to_int(host(w)) == I.to_int(u) * I.to_int(v)
    nu, nv = 1 << 20, 1 << 12
    cut = T.workspace_bytes(nu, nv)
    padded = T.workspace_bytes(nu, nv, T.plan_default(nu, nv))
    assert 0 < cut < padded


def test_random_shapes(T):
    """Seeded random operand lengths from 1 to 60000 limbs, balanced and not,
    through tc_mul (the default plans, cuts and leaves), one batch of all of
    them, and the same operand squared: each equals Python's product."""
    rng = np.random.default_rng(97)
    shapes = [(int(np.exp(rng.uniform(0, np.log(60000)))),
               int(np.exp(rng.uniform(0, np.log(60000))))) for _ in range(40)]
    us = [I.random_limbs(97, 2 * i, a) for i, (a, _) in enumerate(shapes)]
    vs = [I.random_limbs(97, 2 * i + 1, b) for i, (_, b) in enumerate(shapes)]
    for u, v in zip(us, vs):
        assert I.to_int(gpu_mul(T, u, v)) == I.to_int(u) * I.to_int(v), (len(u), len(v))
    outs = T.mul_batch([dev(u) for u in us], [dev(v) for v in vs])
    check_clean(T)
    for u, v, w in zip(us, vs, outs):
        assert I.to_int(host(w)) == I.to_int(u) * I.to_int(v), (len(u), len(v))
    for u in us[:10]:
        assert I.to_int(square(T, u)) == I.to_int(u) ** 2, len(u)


def test_position_major_steps(T):
    """2^18 limbs with a 2-way top level: its interpolation values have about
    2^18 limbs (256 chunks), so its step and evaluation launches run chunk
    position by chunk position over all values; the product is compared whole
    with Python's integer product."""
    n = 1 << 18
    u, v = I.random_limbs(71, 1, n), I.random_limbs(71, 2, n)
    got = gpu_mul(T, u, v, T.Plan.make([2, 16, 3, 3]))
    assert I.to_int(got) == I.to_int(u) * I.to_int(v)


def test_batch_equals_single(T):
    rng = np.random.default_rng(5)
    pairs = []
    for i in range(24):
        n = int(np.exp(rng.uniform(np.log(64), np.log(6000))))
        pairs.append((I.config3_operand(3, 2 * i + 10, n), I.config3_operand(3, 2 * i + 11, n)))
    us = [dev(u) for u, _ in pairs]
    vs = [dev(v) for _, v in pairs]
    outs = T.mul_batch(us, vs)
    check_clean(T)
    for (u, v), w in zip(pairs, outs):
        single = gpu_mul(T, u, v)
        np.testing.assert_array_equal(host(w), single)
        np.testing.assert_array_equal(single, oracle.mul_toom(u, v, [3, 3]))


def test_batch_mixed_matrix_core_leaf_widths(T):
    # leaves of different widths share one matrix-core launch per 256-limb
    # width class; each workgroup must use its own width
    sizes = [513, 600, 700, 767, 768, 769, 900, 1023, 1024, 1100, 1300, 1536, 1537, 2000, 2048]
    us = [I.random_limbs(300 + i, 1, n) for i, n in enumerate(sizes)]
    vs = [I.random_limbs(300 + i, 2, n) for i, n in enumerate(sizes)]
    outs = T.mul_batch([dev(u) for u in us], [dev(v) for v in vs])
    check_clean(T)
    for u, v, w in zip(us, vs, outs):
        assert I.to_int(host(w)) == I.to_int(u) * I.to_int(v)


def test_autotune_sets_default_plan(T):
    try:
        for n in (700, 3000, 20000):
            plan, ms = T.autotune(n)
            assert ms > 0
            got = T.plan_default(n, n)
            assert got.as_list() == plan.as_list()
            # the tuned plan serves the whole size class, ragged sizes included
            for m in (n, n - 3):
                u, v = I.random_limbs(600 + m, 1, m), I.random_limbs(600 + m, 2, m)
                assert I.to_int(gpu_mul(T, u, v)) == I.to_int(u) * I.to_int(v)
    finally:
        T.autotune_clear()
    assert T.plan_default(3000, 3000).as_list() == [(3, 0)]


@pytest.mark.parametrize("Y", [512, 513, 514, 515, 1024, 1026, 1536, 2048, 2049, 3072, 3073, 4095,
                               4096, 4097, 4098, 4099])
def test_values_at_chunk_boundaries(T, Y):
    # widths on and next to multiples of the 512-limb chunk (1024 limbs for
    # interpolation values above 4096): evaluations of Y limbs (nout + 1) and
    # interpolations of Y limbs (ny + 2), negative values included
    B = 4
    nout = Y - 1
    bl = nout - oracle.growth_limbs(B, 0)
    for u in (I.random_limbs(800 + Y, 1, B * bl), I.all_ones(B * bl),
              np.concatenate([I.random_limbs(801 + Y, 1, (B - 1) * bl),
                              np.zeros(bl, np.uint32)])):
        want, wsign = oracle.eval_points(B, 0, u, bl, nout)
        got, gsign = T.eval_points(dev(u), B, 0, bl, nout)
        check_clean(T)
        np.testing.assert_array_equal(host(got).reshape(want.shape), want)
        np.testing.assert_array_equal(gsign.cpu().numpy().astype(np.int8), wsign)
    # one 3-way level: children of bl2 + 1 limbs, interpolation width
    # 2 (bl2 + 1) + 2 = Y or Y - 1
    bl2 = (Y - 4) // 2
    u = I.random_limbs(802 + Y, 1, 3 * bl2)
    v = I.random_limbs(802 + Y, 2, 3 * bl2)
    want = oracle.mul_toom(u, v, [3])
    np.testing.assert_array_equal(gpu_mul(T, u, v, T.Plan.make([3])), want)


def test_repeat_is_deterministic(T):
    u, v = I.random_limbs(9, 9, 30000), I.random_limbs(9, 10, 30000)
    a = gpu_mul(T, u, v)
    b = gpu_mul(T, u, v)
    np.testing.assert_array_equal(a, b)


def test_graph_replays_with_new_addresses(T):
    """A compiled plan is replayed from a captured graph with new operand and
    result addresses each call; eager runs (timing mode launches directly)
    are interleaved; every replay matches the oracle."""
    n = 20000
    pairs = [(I.random_limbs(60 + i, 1, n), I.random_limbs(60 + i, 2, n)) for i in range(3)]
    want = [oracle.mul_toom(u, v, [3, 3, 3]) for u, v in pairs]
    dpairs = [(dev(u), dev(v)) for u, v in pairs]
    for rep in range(3):
        for i, (du, dv) in enumerate(dpairs):
            eager = rep == 1 and i == 1
            if eager:
                T.timing_enable(True)
            w = T.mul(du, dv)
            if eager:
                T.timing_read()
                T.timing_enable(False)
            torch.cuda.synchronize()
            check_clean(T)
            np.testing.assert_array_equal(host(w), want[i], err_msg=f"rep {rep} item {i}")


def test_batch_graph_replays(T):
    rng = np.random.default_rng(17)
    sizes = [int(x) for x in rng.integers(64, 3000, 12)]
    for rep in range(3):
        pairs = [(I.random_limbs(70 + rep, i, n), I.random_limbs(80 + rep, i, n))
                 for i, n in enumerate(sizes)]
        outs = T.mul_batch([dev(u) for u, _ in pairs], [dev(v) for _, v in pairs])
        torch.cuda.synchronize()
        check_clean(T)
        for (u, v), w in zip(pairs, outs):
            np.testing.assert_array_equal(host(w), oracle.mul_toom(u, v, [3]))


# plans whose top level interpolates in several grouped rounds over long
# values, with all-ones operands (every carry chain) and squares
@pytest.mark.parametrize("n,Bs", [(60000, [16, 3]), (40000, [4, 3, 3]), (100000, [8, 3, 3]),
                                  (70001, [5, 3, 3]), (1 << 19, [16, 3, 3, 3]),
                                  (300000, [16, 16]), (2 ** 17 + 3, [32, 3])])
def test_multi_round_levels(T, n, Bs):
    u, v = I.random_limbs(990, len(Bs), n), I.random_limbs(991, len(Bs), n)
    want = oracle.mul_toom(u, v, Bs, threads=16)
    np.testing.assert_array_equal(gpu_mul(T, u, v, T.Plan.make(Bs)), want)
    # worst-case carries and signs
    a = I.all_ones(n)
    np.testing.assert_array_equal(gpu_mul(T, a, a, T.Plan.make(Bs)), oracle.mul_toom(a, a, Bs, threads=16))
    # a square through the same plan
    np.testing.assert_array_equal(square(T, u, T.Plan.make(Bs)), oracle.mul_toom(u, u, Bs, threads=16))


# ------------------------------------------------------------------ Toom-4 on 0, +-1, +-2, 1/2, infinity

HALF = 2             # the library's variant id
ORACLE_HALF = oracle.VAR_HALF


@pytest.mark.parametrize("n", [4000, 4 * 300 + 1, 9 * 64, 40000])
def test_half_points_eval_and_interp(T, n):
    """Evaluation at 0, +-1, +-2, 2^3 U(1/2), U(inf) and the fixed-n
    interpolation, each phase against the oracle's."""
    B = 4
    bl = oracle.block_limbs(n, B)
    nout = bl + oracle.growth_limbs(B, ORACLE_HALF)
    for u in (I.random_limbs(960, n, n), I.all_ones(n)):
        want, wsign = oracle.eval_points(B, ORACLE_HALF, u, bl, nout)
        got, gsign = T.eval_points(dev(u), B, HALF, bl, nout)
        check_clean(T)
        np.testing.assert_array_equal(host(got).reshape(want.shape), want)
        np.testing.assert_array_equal(gsign.cpu().numpy().astype(np.int8), wsign)
    for ones in (False, True):
        u = I.all_ones(B * bl) if ones else I.random_limbs(961, 1, B * bl)
        v = I.all_ones(B * bl) if ones else I.random_limbs(961, 2, B * bl)
        ue, us = oracle.eval_points(B, ORACLE_HALF, u, bl, nout)
        ve, vs = oracle.eval_points(B, ORACLE_HALF, v, bl, nout)
        y = np.stack([oracle.mul_school(a, b) for a, b in zip(ue, ve)])
        sign = ((us ^ vs) * np.array([int(r.any()) for r in y], dtype=np.int8)).astype(np.int8)
        nw = 2 * bl + 1
        want = oracle.interp(B, ORACLE_HALF, y, sign, nw)
        got = T.interp(dev(y.ravel()), torch.from_numpy(sign.astype(np.uint8)).cuda(), B, HALF, nw)
        check_clean(T)
        np.testing.assert_array_equal(host(got).reshape(want.shape), want)


@pytest.mark.parametrize("n,Bs,Vs", [(1024, [4], [HALF]), (4000, [4], [HALF]),
                                     (40000, [4, 3, 3], [HALF, 0, 0]),
                                     (30000, [4, 4], [HALF, HALF]),
                                     (100000, [16, 4, 3], [0, HALF, 0]),
                                     (9000, [3, 4], [1, HALF])])
def test_half_points_products(T, n, Bs, Vs):
    ov = [ORACLE_HALF if x == HALF else x for x in Vs]
    for u, v in ((I.random_limbs(962, n, n), I.random_limbs(963, n, n)),
                 (I.all_ones(n), I.all_ones(n)),
                 (I.single_bit(n, 32 * n - 1), I.sparse_limbs(964, 1, n))):
        want = oracle.mul_toom(u, v, Bs, ov, threads=8)
        np.testing.assert_array_equal(gpu_mul(T, u, v, T.Plan.make(Bs, Vs)), want)
    u = I.random_limbs(965, 1, n)
    np.testing.assert_array_equal(square(T, u, T.Plan.make(Bs, Vs)),
                                  oracle.mul_toom(u, u, Bs, ov, threads=8))


@pytest.mark.parametrize("n,Bs,Vs", [(20000, [3, 3, 3], [0, 0, 0]), (1 << 19, [16, 3, 3, 3], None),
                                     (9000, [2, 3], [0, 1]), (40000, [4, 3, 3], [HALF, 0, 0])])
def test_strict_mode_products(T, n, Bs, Vs):
    """Strict mode (every coefficient of single-round levels in its own exact
    step, recomposed separately) gives the same products as the default
    recomposing steps and as the oracle."""
    u, v = I.random_limbs(980, n, n), I.random_limbs(981, n, n)
    plan = T.Plan.make(Bs, Vs)
    fast = gpu_mul(T, u, v, plan)
    try:
        T.set_strict(True)
        strict = gpu_mul(T, u, v, plan)
    finally:
        T.set_strict(False)
    ov = [ORACLE_HALF if x == HALF else x for x in (Vs or [0] * len(Bs))]
    want = oracle.mul_toom(u, v, Bs, ov, threads=16)
    np.testing.assert_array_equal(fast, want)
    np.testing.assert_array_equal(strict, want)
