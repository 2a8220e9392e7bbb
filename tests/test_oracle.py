"""Pins of the CPU oracle against facts independent of it.

The oracle (oracle/toomref.c) is the checker of the GPU path, so before it is
trusted it is pinned here to the definition of the product (brute force,
Python's own integer product), closed forms, residues, algebraic identities,
the Newton = Lagrange-Waring identity of section 3 in exact rationals, the
direct block convolution w_k = sum_{i+j=k} u_i v_j of section 1, and the
complexity exponents printed in section 2.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1602_02740_amd import inputs as I
from tests.helpers import residue, residue_np, signed_to_sm, sm_to_signed

EDGE = [0, 1, 2, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF, 0x12345678]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def pyint(a):
    return I.to_int(a)


# ---------------------------------------------------------------- products

def test_brute_force_tiny_edge_limbs():
    """nu, nv <= 2 over edge limbs: schoolbook and Toom equal Python's product."""
    vals1 = [np.array([a], dtype=np.uint32) for a in EDGE]
    vals2 = [np.array([a, b], dtype=np.uint32) for a in EDGE[::2] for b in EDGE[1::2]]
    for x in vals1 + vals2:
        for y in vals1 + vals2:
            ref = pyint(x) * pyint(y)
            assert pyint(oracle.mul_school(x, y)) == ref
            for Bs, var in (([2], None), ([3], None), ([3], [oracle.VAR_INF]),
                            ([2], [oracle.VAR_PLAIN])):
                assert pyint(oracle.mul_toom(x, y, Bs, var)) == ref


@pytest.mark.parametrize("n", [1, 2, 7, 100, 1024])
def test_closed_form_all_ones_square(n):
    """(2^k - 1)^2 = 2^(2k) - 2^(k+1) + 1 with k = 32 n (built without multiplying)."""
    k = 32 * n
    expect = np.zeros(2 * n, dtype=np.uint32)
    expect[0] = 1
    expect[n] = 0xFFFFFFFE
    expect[n + 1:] = 0xFFFFFFFF
    assert pyint(expect) == (1 << (2 * k)) - (1 << (k + 1)) + 1
    u = I.all_ones(n)
    np.testing.assert_array_equal(oracle.mul_school(u, u), expect)
    plans = [([2], None), ([3], [oracle.VAR_INF])] if n < 8 else \
        [([3], [oracle.VAR_INF]), ([3], None), ([16, 2], None), ([4, 3], None)]
    for Bs, var in plans:
        np.testing.assert_array_equal(oracle.mul_toom(u, u, Bs, var), expect)


def test_closed_form_single_bits_and_mersenne_pairs():
    rng = np.random.default_rng(11)
    for _ in range(20):
        n = int(rng.integers(1, 300))
        a, c = (int(x) for x in rng.integers(0, 32 * n, 2))
        u, v = I.single_bit(n, a), I.single_bit(n, c)
        expect = I.single_bit(2 * n, a + c)
        np.testing.assert_array_equal(oracle.mul_school(u, v), expect)
        np.testing.assert_array_equal(oracle.mul_toom(u, v, [3, 2]), expect)
    # (2^k - 1)(2^j - 1) = 2^(k+j) - 2^k - 2^j + 1
    for k, j in [(32, 64), (100, 37), (1000, 999), (32 * 64, 32 * 64 - 5)]:
        n = (max(k, j) + 31) // 32
        u = I.from_int((1 << k) - 1, n)
        v = I.from_int((1 << j) - 1, n)
        expect = I.from_int((1 << (k + j)) - (1 << k) - (1 << j) + 1, 2 * n)
        np.testing.assert_array_equal(oracle.mul_school(u, v), expect)
        np.testing.assert_array_equal(oracle.mul_toom(u, v, [4]), expect)


def test_config1_operands_against_python():
    for u, v in (I.config1_uniform(), I.config1_all_ones(), I.config1_single_bit()):
        ref = pyint(u) * pyint(v)
        assert pyint(oracle.mul_school(u, v)) == ref
        assert pyint(oracle.mul_toom(u, v, [3], [oracle.VAR_INF])) == ref
        assert pyint(oracle.mul_toom(u, v, [3])) == ref


@pytest.mark.parametrize("B", [2, 3, 4, 5, 8, 16, 32])
@pytest.mark.parametrize("variant", [oracle.VAR_EVENODD, oracle.VAR_PLAIN, oracle.VAR_ODD_DIRECT])
def test_toom_equals_python_int(B, variant):
    rng = np.random.default_rng(B * 10 + variant)
    for n in [1, 3, B, 2 * B + 1, 257, 1500]:
        u = I.random_limbs(100 + B, n, n)
        v = I.random_limbs(200 + B, n + 1, max(1, n - int(rng.integers(0, n))))
        ref = pyint(u) * pyint(v)
        assert pyint(oracle.mul_toom(u, v, [B], [variant])) == ref


def test_half_points_equal_python_int():
    """Toom-4 on 0, +-1, +-2, 1/2, inf with the fixed-n inverse, alone and
    under and over other levels, against Python's product; all-ones
    operands reach the largest values (growth of 4 bits)."""
    H = oracle.VAR_HALF
    for n in [4, 9, 257, 1500, 5001]:
        u, v = I.random_limbs(150, n, n), I.random_limbs(151, n, n)
        ref = pyint(u) * pyint(v)
        assert pyint(oracle.mul_toom(u, v, [4], [H])) == ref
        assert pyint(oracle.mul_toom(u, v, [4, 3], [H, 0])) == ref
        assert pyint(oracle.mul_toom(u, v, [3, 4], [0, H])) == ref
        a = I.all_ones(n)
        assert pyint(oracle.mul_toom(a, a, [4, 4], [H, H])) == pyint(a) ** 2
    # a flipped bit in one point product is caught by the exact divisions
    bl = 3
    ub = [(1 << (32 * bl)) - 1 - 5 * t for t in range(4)]
    ys = [at(ub, x) ** 2 for x in points(4, H)]
    mag, sign = signed_to_sm(ys, 8)
    oracle.interp(4, H, mag, sign, 2 * bl + 1)
    for k in range(1, 6):
        bad = mag.copy()
        bad[k, 0] ^= np.uint32(1)
        with pytest.raises(oracle.OracleError):
            oracle.interp(4, H, bad, sign, 2 * bl + 1)


def test_recursive_plans_and_threads():
    u, v = I.random_limbs(9, 1, 20000), I.random_limbs(9, 2, 20000)
    ref = pyint(u) * pyint(v)
    for Bs in ([16, 3, 2], [32, 3], [4, 4, 4], [8, 2, 2, 2]):
        serial = oracle.mul_toom(u, v, Bs)
        assert pyint(serial) == ref
        np.testing.assert_array_equal(oracle.mul_toom(u, v, Bs, threads=6), serial)


def test_residues_mod_primes():
    """w mod p = (u mod p)(v mod p) mod p, computed from the limbs alone."""
    u, v = I.random_limbs(5, 7, 30000), I.random_limbs(5, 8, 29000)
    w = oracle.mul_toom(u, v, [16, 3])
    for p in (2147483647, 998244353, 4294967291, 65521):
        assert residue_np(w, p) == residue_np(u, p) * residue_np(v, p) % p
        assert residue(w[:50], p) == residue_np(w[:50], p)
    p61 = (1 << 61) - 1
    assert residue(w, p61) == residue(u, p61) * residue(v, p61) % p61


def test_commutativity_distributivity_squaring():
    rng = np.random.default_rng(3)
    for n in (50, 700, 3000):
        u = I.random_limbs(3, n, n)
        v1 = I.random_limbs(4, n, n)
        v2 = I.random_limbs(6, n, n) >> np.uint32(1)
        v1 = v1 >> np.uint32(1)
        s = I.from_int(pyint(v1) + pyint(v2), n)  # no overflow: both < 2^(32n-1)
        a = oracle.mul_toom(u, v1, [3, 2])
        b = oracle.mul_toom(u, v2, [4])
        c = oracle.mul_toom(u, s, [8])
        assert pyint(c) == pyint(a) + pyint(b)
        np.testing.assert_array_equal(oracle.mul_toom(v1, u, [3, 2]), a)
        sq = oracle.mul_toom(u, u, [5])
        np.testing.assert_array_equal(sq, oracle.mul_school(u, u))
        assert int(rng.integers(0, 2)) in (0, 1)


# ---------------------------------------------------------------- phases

def points(B, variant):
    if variant == oracle.VAR_INF:
        return [0, 1, -1, 2, None]
    if variant == oracle.VAR_HALF:
        return [0, 1, -1, 2, -2, Fraction(1, 2), None]
    pts = [0]
    for j in range(B - 1):
        pts += [1 << j, -(1 << j)]
    return pts


def at(blk, x):
    """A polynomial with coefficients blk at x (None: infinity, its top
    coefficient); at x = 1/2 the homogeneous value 2^(deg) P(1/2)."""
    if x is None:
        return blk[-1]
    if isinstance(x, Fraction):
        v = sum(b * x ** t for t, b in enumerate(blk)) * 2 ** (len(blk) - 1)
        assert v.denominator == 1
        return int(v)
    return sum(b * x ** t for t, b in enumerate(blk))


def blocks_of(u, bl, B):
    x = pyint(u)
    return [(x >> (32 * bl * t)) & ((1 << (32 * bl)) - 1) for t in range(B)]


@pytest.mark.parametrize("B,variant", [(2, 0), (3, 0), (3, 1), (4, 0), (7, 0), (16, 0), (32, 0),
                                       (4, 4)])
def test_eval_equals_direct_polynomial(B, variant):
    """U(x_k) = sum_t u_t x_k^t evaluated directly with Python ints (section 1)."""
    n = 40 * B + 3
    u = I.random_limbs(21, B, n)
    bl = oracle.block_limbs(n, B)
    nout = bl + oracle.growth_limbs(B, variant)
    mag, sign = oracle.eval_points(B, variant, u, bl, nout)
    blk = blocks_of(u, bl, B)
    got = sm_to_signed(mag, sign)
    for k, x in enumerate(points(B, variant)):
        assert got[k] == at(blk, x), (k, x)
    # worst case (all ones) fits the stated growth
    oracle.eval_points(B, variant, I.all_ones(n), bl, nout)


@pytest.mark.parametrize("B,variant", [(2, 0), (3, 0), (3, 1), (4, 0), (5, 0), (16, 0), (32, 0),
                                       (3, 2), (8, 2), (2, 3), (3, 3), (4, 3), (16, 3), (32, 3),
                                       (4, 4)])
def test_interp_equals_block_convolution(B, variant):
    """Interpolated w_k equal the direct convolution sum_{i+j=k} u_i v_j."""
    rng = np.random.default_rng(B)
    bl = 3
    for trial in range(3):
        ub = [int.from_bytes(rng.bytes(4 * bl), "little") for _ in range(B)]
        vb = [int.from_bytes(rng.bytes(4 * bl), "little") for _ in range(B)]
        if trial == 2:
            ub = vb = [(1 << (32 * bl)) - 1] * B
        ys = [at(ub, x) * at(vb, x) for x in points(B, variant)]
        ny = max(abs(y).bit_length() for y in ys) // 32 + 1
        mag, sign = signed_to_sm(ys, ny)
        nw = 2 * bl + 1
        w = oracle.interp(B, variant, mag, sign, nw)
        for k in range(2 * B - 1):
            conv = sum(ub[i] * vb[k - i] for i in range(max(0, k - B + 1), min(k, B - 1) + 1))
            assert pyint(w[k]) == conv, (k, trial)


@pytest.mark.parametrize("B", [2, 3, 4, 7, 16, 32])
def test_odd_polynomial_two_readings_agree(B):
    """Section 4's odd part read two ways -- X W_o(X) of degree n at X = 0 and
    the n non-zero nodes, or W_o of degree n-1 at the non-zero nodes alone --
    give identical coefficients on the same point products, and both equal
    the block convolution (checked for every k above)."""
    rng = np.random.default_rng(B + 77)
    bl = 4
    ub = [int.from_bytes(rng.bytes(4 * bl), "little") for _ in range(B)]
    vb = [int.from_bytes(rng.bytes(4 * bl), "little") for _ in range(B)]
    ys = [sum(b * x ** t for t, b in enumerate(ub)) * sum(b * x ** t for t, b in enumerate(vb))
          for x in points(B, 0)]
    ny = max(abs(y).bit_length() for y in ys) // 32 + 1
    mag, sign = signed_to_sm(ys, ny)
    a = oracle.interp(B, oracle.VAR_EVENODD, mag, sign, 2 * bl + 1)
    b = oracle.interp(B, oracle.VAR_ODD_DIRECT, mag, sign, 2 * bl + 1)
    np.testing.assert_array_equal(a, b)
    # a value no product gives: W(+1) - W(-1) off by two keeps the halving
    # exact, but W_o(1) then differs, and the X W_o route's constant term
    # (asserted zero) or the direct route's divisions must notice
    ys[1] += 2
    mag, sign = signed_to_sm(ys, ny)
    if B > 2:
        with pytest.raises(oracle.OracleError):
            oracle.interp(B, oracle.VAR_EVENODD, mag, sign, 2 * bl + 1)
        with pytest.raises(oracle.OracleError):
            oracle.interp(B, oracle.VAR_ODD_DIRECT, mag, sign, 2 * bl + 1)


def test_interp_detects_planted_error():
    """A product with one flipped bit makes a halving or division inexact."""
    B, bl = 4, 2
    rng = np.random.default_rng(5)
    ub = [int.from_bytes(rng.bytes(4 * bl), "little") for _ in range(B)]
    ys = [sum(b * x ** t for t, b in enumerate(ub)) ** 2 for x in points(B, 0)]
    mag, sign = signed_to_sm(ys, 8)
    oracle.interp(B, 0, mag, sign, 2 * bl + 1)
    mag[1, 0] ^= np.uint32(1)
    with pytest.raises(oracle.OracleError):
        oracle.interp(B, 0, mag, sign, 2 * bl + 1)


def test_recompose_definition():
    rng = np.random.default_rng(8)
    B, bl = 5, 4
    nw = 2 * bl + 1
    w = rng.integers(0, 2 ** 32, size=(2 * B - 1, nw), dtype=np.uint64).astype(np.uint32)
    w[:, -1] &= np.uint32(7)
    expect = sum(pyint(w[k]) << (32 * bl * k) for k in range(2 * B - 1))
    nout = (expect.bit_length() + 31) // 32 + 1
    assert pyint(oracle.recompose(B, bl, w, nout)) == expect
    with pytest.raises(oracle.OracleError):
        oracle.recompose(B, bl, w, nout - 2)


# ------------------------------------------------------------- section 3

def random_poly(rng, n, bits=40):
    return [int(rng.integers(-(1 << bits), 1 << bits)) for _ in range(n + 1)]


def alpha_closed_form(x, y):
    """alpha_k = sum_{i<=k} y_i / prod_{j<=k, j!=i}(x_i - x_j)  (Theorem 3.1)."""
    out = []
    for k in range(len(x)):
        s = Fraction(0)
        for i in range(k + 1):
            d = 1
            for j in range(k + 1):
                if j != i:
                    d *= x[i] - x[j]
            s += Fraction(y[i], d)
        out.append(s)
    return out


def lagrange_waring(x, y, t):
    s = Fraction(0)
    for k in range(len(x)):
        term = Fraction(y[k])
        for j in range(len(x)):
            if j != k:
                term *= Fraction(t - x[j], x[k] - x[j])
        s += term
    return s


NODE_SETS = [
    [0, 1, 4, 16, 64, 256],            # X = 0, 4^(m-1): the even-odd nodes
    [0, 1, -1, 2],                      # the infinity variant's finite points
    [0, 1, -1, 2, -2, 4, -4],           # plain variant, B = 4
    [3, -7, 11, 0, 5],
    [0, 1, 4, 16, 64, 256, 1024, 4096, 16384, 65536, 1 << 20, 1 << 22, 1 << 24, 1 << 26,
     1 << 28, 0][:16],
]


@pytest.mark.parametrize("x", NODE_SETS[:4] + [[0] + [4 ** m for m in range(15)]])
def test_newton_equals_lagrange_and_monomial(x):
    """Section 3: the divided-difference loop gives the alpha_k of Theorem 3.1,
    the Newton form equals Lagrange-Waring, and the second loop recovers the
    monomial coefficients."""
    rng = np.random.default_rng(len(x))
    n = len(x) - 1
    for _ in range(3):
        c = random_poly(rng, n)
        y = [sum(cl * xi ** l for l, cl in enumerate(c)) for xi in x]
        nl = max(abs(v).bit_length() for v in y) // 32 + 2
        mag, sign = signed_to_sm(y, nl)
        am, asg = oracle.newton(x, mag, sign, phase=1)
        alpha = sm_to_signed(am, asg)
        assert [Fraction(a) for a in alpha] == alpha_closed_form(x, y)
        for t in (-3, 2, 5, 1000):
            newton_form = sum(Fraction(alpha[k]) * math.prod(t - x[j] for j in range(k))
                              for k in range(n + 1))
            assert newton_form == lagrange_waring(x, y, t)
        cm, csg = oracle.newton(x, mag, sign, phase=2)
        assert sm_to_signed(cm, csg) == c


def test_newton_vandermonde_solve():
    """The monomial coefficients equal the Vandermonde solve (section 3, last
    paragraph) in exact rationals."""
    x = [0, 1, 4, 16, 64]
    rng = np.random.default_rng(2)
    c = random_poly(rng, 4, bits=60)
    y = [sum(cl * xi ** l for l, cl in enumerate(c)) for xi in x]
    n = len(x)
    A = [[Fraction(xi) ** l for l in range(n)] + [Fraction(yi)] for xi, yi in zip(x, y)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    sol = [A[i][n] / A[i][i] for i in range(n)]
    mag, sign = signed_to_sm(y, 6)
    cm, csg = oracle.newton(x, mag, sign, phase=2)
    assert [Fraction(v) for v in sm_to_signed(cm, csg)] == sol == [Fraction(v) for v in c]


def test_newton_rejects_non_integer_divided_difference():
    """Values that are not from an integer polynomial give an inexact division."""
    x = [0, 1, 4]
    mag, sign = signed_to_sm([0, 1, 0], 2)
    with pytest.raises(oracle.OracleError):
        oracle.newton(x, mag, sign, phase=1)


# ------------------------------------------------------------- section 2

def read_golden_exponents():
    out = {}
    with open(os.path.join(GOLDEN, "exponents.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                b, a = line.split()
                out[int(b)] = float(a)
    return out


def test_dry_run_counts_match_real_run():
    u, v = I.random_limbs(1, 1, 5000), I.random_limbs(1, 2, 5000)
    for Bs in ([16, 3], [3, 3, 2], [32]):
        oracle.counts_reset()
        oracle.mul_toom(u, v, Bs)
        assert oracle.counts_get() == oracle.plan_counts(5000, Bs)


@pytest.mark.parametrize("B", [2, 3, 16, 32])
def test_complexity_exponent_from_op_counts(B):
    """Leaf work grows as N^(log(2B-1)/log B) (section 2, eqs. 2.1-2.4)."""
    theory = math.log(2 * B - 1) / math.log(B)
    printed = read_golden_exponents()
    if B in printed:
        assert round(theory, 3) == printed[B]
    leaf = 1 << 14  # leaves much wider than the evaluation growth
    levels = 3 if B >= 16 else 6
    ns, ops = [], []
    for L in range(1, levels + 1):
        n = leaf * B ** L
        ns.append(n)
        ops.append(oracle.plan_counts(n, [B] * L)["leaf_mults"])
    slope = np.polyfit(np.log(ns), np.log(ops), 1)[0]
    assert abs(slope - theory) < 0.03, (slope, theory)


def test_even_odd_halves_interpolation_work():
    """Section 4: (2n)^2 Y without the even-odd split against 2 n^2 Y with it;
    exactly (2n+1)/(n+1) with the loops' step counts, -> 2 as n grows."""
    u, v = I.random_limbs(2, 1, 4000), I.random_limbs(2, 2, 4000)
    for B in (4, 16, 32):
        n = B - 1
        oracle.counts_reset()
        w1 = oracle.mul_toom(u, v, [B], [oracle.VAR_EVENODD])
        eo = oracle.counts_get()["interp_limbs"]
        oracle.counts_reset()
        w2 = oracle.mul_toom(u, v, [B], [oracle.VAR_PLAIN])
        pl = oracle.counts_get()["interp_limbs"]
        np.testing.assert_array_equal(w1, w2)
        assert pl * (n + 1) == eo * (2 * n + 1)
    assert (2 * 31 + 1) / (31 + 1) > 1.95


def test_intermediates_fit_fixed_width_worst_case():
    """All-ones operands (largest evaluations) keep every Newton intermediate
    within the signed width 2n'+2 that the GPU path computes in."""
    for B, n in ((16, 16 * 40), (32, 32 * 40), (3, 300), (2, 100)):
        u = I.all_ones(n)
        w = oracle.mul_toom(u, u, [B])  # raises on a width overflow
        assert pyint(w) == pyint(u) ** 2


# ---------------------------------------------------------------- NTT products (section 5)

P_NTT = (1 << 64) - (1 << 32) + 1


def test_ntt_field_and_roots():
    """p = 2^64 - 2^32 + 1 passes Fermat tests to several bases; 7 is a
    quadratic non-residue, so the oracle's w_N has order exactly N: w^N = 1
    and w^(N/2) = p - 1, for every power of two up to 2^32."""
    assert oracle.NTT_P == P_NTT
    for a in (2, 3, 5, 7, 11, 13):
        assert pow(a, P_NTT - 1, P_NTT) == 1
    assert pow(7, (P_NTT - 1) // 2, P_NTT) == P_NTT - 1
    for k in range(1, 33):
        N = 1 << k
        w = oracle.ntt_root(N)
        assert pow(w, N, P_NTT) == 1 and pow(w, N // 2, P_NTT) == P_NTT - 1
    assert oracle.ntt_root(3) == 0 and oracle.ntt_root(1 << 33) == 0


def test_ntt_equals_dft_definition():
    """The transform equals the DFT written out in Python integers,
    X[j] = sum_i x[i] w^(ij) mod p, for N up to 64, on random and edge
    values (0, 1, p - 1); the inverse gives back x."""
    rng = np.random.default_rng(51)
    for k in range(0, 7):
        N = 1 << k
        w = oracle.ntt_root(N)
        for trial in range(3):
            if trial == 0:
                x = [P_NTT - 1] * N
            elif trial == 1:
                x = [int(t) for t in rng.integers(0, 2, N)]
            else:
                x = [int(t) % P_NTT for t in rng.integers(0, 1 << 63, N, dtype=np.uint64)]
            X = oracle.ntt(x)
            ref = [sum(x[i] * pow(w, i * j, P_NTT) for i in range(N)) % P_NTT for j in range(N)]
            assert [int(t) for t in X] == ref
            assert [int(t) for t in oracle.ntt(X, inverse=True)] == x


def test_ntt_inverse_roundtrip_large():
    """inverse(forward(x)) = x for N = 2^12 .. 2^16 (random values below p),
    and the transform of a unit impulse at i is the row w^(ij)."""
    rng = np.random.default_rng(52)
    for k in (12, 16):
        N = 1 << k
        x = rng.integers(0, P_NTT, N, dtype=np.uint64)
        assert np.array_equal(oracle.ntt(oracle.ntt(x), inverse=True), x)
        e = np.zeros(N, dtype=np.uint64)
        e[3] = 1
        X = oracle.ntt(e)
        w3 = pow(oracle.ntt_root(N), 3, P_NTT)
        assert [int(X[j]) for j in (0, 1, 2, N - 1)] == \
            [1, w3, pow(w3, 2, P_NTT), pow(w3, N - 1, P_NTT)]


def test_ntt_pieces_match_shifts():
    """Piece i equals floor(u / 2^(bits i)) mod 2^bits in Python integers,
    for piece widths 1..32, including the zero pieces past the operand."""
    u = I.random_limbs(53, 1, 37)
    U = pyint(u)
    for bits in (1, 7, 16, 17, 18, 20, 24, 31, 32):
        n = oracle.ntt_npieces(len(u), bits)
        assert n == -(-32 * len(u) // bits)
        got = oracle.ntt_pieces(u, bits, n + 3)
        assert [int(t) for t in got] == [(U >> (bits * i)) & ((1 << bits) - 1) for i in range(n + 3)]


def test_mul_ntt_equals_python_product():
    """Products through the transform equal Python's products: sizes that
    make the convolution just fit or just overflow a power of two, unbalanced
    operands, piece widths 16..22, and all-ones operands, whose convolution
    coefficients are the largest the bound allows."""
    cases = [(1, 1), (2, 1), (31, 33), (64, 64), (65, 63), (255, 2), (1000, 999), (4096, 4096),
             (5000, 300)]
    for i, (nu, nv) in enumerate(cases):
        u = I.random_limbs(54, 2 * i, nu)
        v = I.random_limbs(54, 2 * i + 1, nv)
        for bits in (16, 18, 22):
            assert pyint(oracle.mul_ntt(u, v, bits)) == pyint(u) * pyint(v)
    ones = np.full(3000, 0xFFFFFFFF, dtype=np.uint32)
    for bits in (16, 20, 24):
        assert pyint(oracle.mul_ntt(ones, ones, bits)) == (pyint(ones)) ** 2


def test_mul_ntt_rejects_inexact_piece_width():
    """Where (2^bits - 1)^2 min(pieces) reaches p a coefficient could wrap
    modulo p: the oracle refuses (and accepts just below the bound)."""
    n = 1 << 10
    u = np.full(n, 0xFFFFFFFF, dtype=np.uint32)
    pieces = oracle.ntt_npieces(n, 28)
    assert ((1 << 28) - 1) ** 2 * pieces >= P_NTT
    with pytest.raises(oracle.OracleError):
        oracle.mul_ntt(u, u, 28)
    assert ((1 << 26) - 1) ** 2 * oracle.ntt_npieces(n, 26) < P_NTT
    assert pyint(oracle.mul_ntt(u, u, 26)) == pyint(u) ** 2


def test_toom_over_ntt_leaves():
    """Section 5's Toom-Cook over an FFT product: Toom levels with NTT leaves
    equal Python's product, for balanced, unbalanced and square operands."""
    for i, (nu, nv, Bs) in enumerate([(3000, 3000, [3]), (20000, 20000, [16]),
                                      (12000, 7000, [4, 2]), (9000, 9000, [32])]):
        u = I.random_limbs(55, 2 * i, nu)
        v = I.random_limbs(55, 2 * i + 1, nv)
        assert pyint(oracle.mul_toom(u, v, Bs, ntt_bits=16)) == pyint(u) * pyint(v)
    u = I.random_limbs(55, 9, 5000)
    assert pyint(oracle.mul_toom(u, u, [3, 3], ntt_bits=18)) == pyint(u) ** 2
