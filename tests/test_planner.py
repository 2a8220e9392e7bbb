"""Host-side checks of the planner (no GPU needed): plan costs and workspace
sizes are computed without running anything, so the recursion's node counts
and widths, the merged interpolation rounds, the cut of unbalanced products
and the algorithmic byte counts can be checked against independent
derivations here."""
import math

import pytest

from paper_1602_02740_amd import toom


def growth(B, var=toom.VAR_EVENODD):
    """Limbs an evaluation at the points 0, +-1, ..., +-2^(B-2) adds to a
    block (section 6): |U(+-2^j)| < B 2^(32 bl + j (B-1)), plus a sign bit."""
    if var == toom.VAR_INF or B <= 3:
        return 1
    return ((B - 1) * (B - 2) + math.ceil(math.log2(B)) + 1 + 31) // 32


def recursion(n, Bs):
    """(nodes, width) of the leaves of plan Bs on n-limb operands."""
    nodes, w = 1, n
    for B in Bs:
        nodes *= 2 * B - 1
        w = -(-w // B) + growth(B)
    return nodes, w


@pytest.mark.parametrize("n,Bs", [(1 << 19, [16, 3, 3, 3]), (1 << 25, [32, 16, 16, 3]),
                                  (5000, [2, 3]), (70000, [4, 16]), (3000, [5]), (20000, [8, 3])])
def test_leaf_products_follow_the_recursion(n, Bs):
    c = toom.plan_cost(n, n, toom.Plan.make(Bs))
    nodes, w = recursion(n, Bs)
    assert c["leaf_limb_products"] == nodes * w * w
    assert c["launches"]["leaf"] == 1


def test_config2_launches():
    """2^19 x 2^19 limbs, plan 16,3,3,3: one evaluation launch and one sign
    fix-up per level, one leaf launch; the 16-way level's interpolation
    rounds merged into 8 step launches and one recomposition; each 3-way
    level (one interpolation round) one recomposing step, which forms the
    node products straight from the point products."""
    c = toom.plan_cost(1 << 19, 1 << 19, toom.Plan.make([16, 3, 3, 3]))
    assert c["launches"] == {"eval": 8, "leaf": 1, "step": 11, "recomp": 1}


def test_evaluation_bytes_of_config2():
    """Each level reads both operands of every node once and writes 2B-1
    values of nc + 1 limbs (magnitude and sign) per operand."""
    n, Bs = 1 << 19, [16, 3, 3, 3]
    want, nodes, w = 0, 1, n
    for B in Bs:
        nc = -(-w // B) + growth(B)
        want += 4 * nodes * (2 * w + 2 * (2 * B - 1) * (nc + 1))
        nodes, w = nodes * (2 * B - 1), nc
    c = toom.plan_cost(n, n, toom.Plan.make(Bs))
    assert c["bytes"]["eval"] == want


@pytest.mark.parametrize("B", [2, 3, 4, 5, 6, 8, 12, 16, 24, 32])
def test_every_split_plans(B):
    """Section 3's rounds for every B up to 32 fit the step kernel's limits
    (terms, weights, shifts, divisors) once merged."""
    n = 8 * growth(B) * B * 4
    c = toom.plan_cost(n, n, toom.Plan.make([B]))
    assert c["launches"]["step"] >= 1
    assert c["leaf_limb_products"] == (2 * B - 1) * (-(-n // B) + growth(B)) ** 2


def cut_leaf_products(a, s):
    """Leaf limb products of tc_mul's cut of an a x s product (a >= 2 s):
    the full s-limb pieces with the balanced plan of s, then the shorter last
    piece (cut again while unbalanced)."""
    if max(a, s) < 2 * min(a, s):
        n = max(a, s)
        return toom.plan_cost(a, s, toom.plan_default(n, n))["leaf_limb_products"]
    a, s = max(a, s), min(a, s)
    m = -(-a // s)
    r = a - (m - 1) * s
    full = m if r == s else m - 1
    leaf = full * toom.plan_cost(s, s, toom.plan_default(s, s))["leaf_limb_products"]
    if r < s:
        leaf += cut_leaf_products(r, s)
    return leaf


@pytest.mark.parametrize("nu,nv", [(1 << 20, 1 << 12), (1 << 12, 1 << 20), (7201, 2400),
                                   (70000, 3000), (300001, 40000), (100, 1), (65, 32)])
def test_unbalanced_products_are_cut(nu, nv):
    c = toom.plan_cost(nu, nv)
    assert c["leaf_limb_products"] == cut_leaf_products(nu, nv)
    padded = toom.plan_cost(nu, nv, toom.plan_default(nu, nv))
    assert c["leaf_limb_products"] <= padded["leaf_limb_products"]


def test_cut_of_2p20_by_2p12():
    """256 pieces of 4096 limbs, one 3-way level each (leaves of 1367 limbs),
    the pieces' recomposing step and the final sum: far less work and scratch
    than the zero-padded balanced plan of 2^20 limbs."""
    nu, nv = 1 << 20, 1 << 12
    c = toom.plan_cost(nu, nv)
    assert c["leaf_limb_products"] == 256 * 5 * 1367 ** 2
    assert c["launches"]["step"] == 1
    assert c["launches"]["recomp"] == 1
    cut = toom.workspace_bytes(nu, nv)
    padded = toom.workspace_bytes(nu, nv, toom.plan_default(nu, nv))
    assert 0 < cut < padded / 10
    # the final sum reads the two partial sums and writes the product
    per_piece = toom.plan_cost(nv, nv, toom.plan_default(nv, nv))["bytes"]["recomp"]
    assert c["bytes"]["recomp"] == 256 * per_piece + 4 * 3 * (nu + nv)


def test_balanced_products_are_not_cut():
    # ratios below 2, and products of 2^31 limbs or more (the final sum's
    # width is 32-bit), keep the zero-padded balanced plan
    for nu, nv in ((1000, 501), (4096, 2049), (1 << 19, (1 << 18) + 1), ((1 << 31) - 5, 7)):
        n = max(nu, nv)
        assert toom.plan_cost(nu, nv) == toom.plan_cost(nu, nv, toom.plan_default(n, n))


@pytest.mark.parametrize("n,Bs", [(1 << 19, [16, 3, 3, 3]), (12000, [3, 3]), (1 << 16, [4, 16])])
def test_chunk_scale_changes_speed_only(n, Bs):
    """A plan's chunk scale (the linear passes' tile width) changes neither
    the algorithmic bytes nor the launch count; scales beyond +-2 are
    refused."""
    base = toom.plan_cost(n, n, toom.Plan.make(Bs))
    for ch in (-2, -1, 1, 2):
        c = toom.plan_cost(n, n, toom.Plan.make(Bs, chunk=ch))
        assert c["bytes"] == base["bytes"] and c["launches"] == base["launches"]
    with pytest.raises(toom.ToomError):
        toom.plan_cost(n, n, toom.Plan.make(Bs, chunk=3))
