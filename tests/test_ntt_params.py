"""Host-side check of the transform leaves' parameter choice (no GPU
needed): for an na x nb product the library takes the smallest power-of-two
length N that holds the acyclic convolution of the pieces for some width
16..30 while every coefficient stays below p = 2^64 - 2^32 + 1, and the
narrowest such width (section 5 multiplies with an FFT; here an exact NTT,
so the product is exact only under that bound)."""
import pytest

from paper_1602_02740_amd import toom

P = (1 << 64) - (1 << 32) + 1


def pieces(n, bits):
    return -(-32 * n // bits)


def fits(na, nb, bits, N):
    pa, pb = pieces(na, bits), pieces(nb, bits)
    return pa + pb - 1 <= N and ((1 << bits) - 1) ** 2 * min(pa, pb) < P


@pytest.mark.parametrize("na,nb", [(1, 1), (2, 1), (100, 100), (1000, 999), (2048, 2048),
                                   (4096, 4096), (32775, 32775), (5000, 300),
                                   ((1 << 20) + 30, (1 << 20) + 30), (1 << 21, 1 << 21),
                                   (3 << 20, 3 << 20)])
def test_ntt_params_smallest_exact_length(na, nb):
    bits, N, C = toom.ntt_params(na, nb)
    assert N & (N - 1) == 0 and 64 <= N <= 1 << 24
    assert 16 <= bits <= 30 and fits(na, nb, bits, N)
    # no shorter transform works with any width, and no narrower width at N
    assert not any(fits(na, nb, b, N // 2) for b in range(16, 31)) or N == 64
    assert not any(fits(na, nb, b, N) for b in range(16, bits))
    assert C == min(N, 1 << 13)


def test_ntt_params_limits():
    """Products whose convolution needs more than 2^24 points are refused."""
    with pytest.raises(toom.ToomError):
        toom.ntt_params(1 << 23, 1 << 23)
    with pytest.raises(toom.ToomError):
        toom.ntt_params(0, 5)


def test_ntt_plan_costs():
    """A transform-leaf plan plans without a device: the leaves' launches
    are one phase of 5 (4 for squares, 3 without a column pass), and the
    leaf bytes are each leaf's operands and product read or written once."""
    n = 1 << 16
    plan = toom.Plan.make([16], leaf=toom.LEAF_NTT)
    c = toom.plan_cost(n, n, plan)
    bl = -(-n // 16) + 7
    assert c["launches"]["leaf"] == 5
    assert c["bytes"]["leaf"] == pytest.approx(31 * 4.0 * (bl + bl + 2 * bl))
    c0 = toom.plan_cost(2000, 2000, toom.Plan.make([], leaf=toom.LEAF_NTT))
    assert c0["launches"]["leaf"] == 3
