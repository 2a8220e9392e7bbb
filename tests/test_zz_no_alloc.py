"""tc_mul_noalloc, the entry point for callers that cannot allocate: through
the C ABI its products equal tc_mul's bit for bit, call after call, the
second call smaller than the first; a product beyond the fixed workspace is
refused before anything is enqueued; device free memory does not move."""
import ctypes

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
    toom.sync()
    return toom


def noalloc(T, w, u, v, stream):
    return T.lib().tc_mul_noalloc(ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(u.data_ptr()),
                                  u.numel(), ctypes.c_void_p(v.data_ptr()), v.numel(),
                                  ctypes.c_void_p(stream.cuda_stream))


def test_noalloc_matches_tc_mul(T):
    stream = torch.cuda.current_stream()
    # balanced with three Toom levels, then a smaller unbalanced one (cut
    # into pieces), then a single leaf, then a square
    shapes = [(100000, 100000), (20000, 7000), (1500, 1500), (30000, 30000)]
    ops = []
    for i, (a, b) in enumerate(shapes):
        u = T.to_device(I.random_limbs(900 + i, 1, a))
        v = u if i == 3 else T.to_device(I.random_limbs(900 + i, 2, b))
        ops.append((u, v))
    want = []
    for u, v in ops:
        want.append(T.to_host(T.mul(u, v)))
    T.sync()
    outs = [T.empty(u.numel() + v.numel()) for u, v in ops]
    for rep in range(2):
        for k, ((u, v), w) in enumerate(zip(ops, outs)):
            w.fill_(-1)
            assert noalloc(T, w, u, v, stream) == 0
            # the next call reuses the workspace in stream order
        torch.cuda.synchronize()
        T.sync()
        for k, w in enumerate(outs):
            np.testing.assert_array_equal(T.to_host(w), want[k], err_msg=f"rep {rep} shape {k}")
    # two calls back to back without a host wait, the second smaller
    (u0, v0), (u1, v1) = ops[0], ops[1]
    assert noalloc(T, outs[0], u0, v0, stream) == 0
    assert noalloc(T, outs[1], u1, v1, stream) == 0
    T.sync()
    np.testing.assert_array_equal(T.to_host(outs[0]), want[0])
    np.testing.assert_array_equal(T.to_host(outs[1]), want[1])
    a = I.to_int(T.to_host(ops[1][0]))
    b = I.to_int(T.to_host(ops[1][1]))
    assert I.to_int(want[1]) == a * b


def test_noalloc_rejects_beyond_workspace(T):
    stream = torch.cuda.current_stream()
    cap = int(T.lib().tc_noalloc_capacity())
    assert cap == 64 << 20
    n = 1 << 19
    assert T.workspace_bytes(n, n) > cap
    u = T.to_device(I.random_limbs(910, 1, n))
    v = T.to_device(I.random_limbs(910, 2, n))
    w = T.empty(2 * n)
    w.fill_(7)
    torch.cuda.synchronize()
    assert noalloc(T, w, u, v, stream) == -8  # TC_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert int((w != 7).sum()) == 0  # nothing ran
    # argument errors as for tc_mul
    assert T.lib().tc_mul_noalloc(None, ctypes.c_void_p(u.data_ptr()), n,
                                  ctypes.c_void_p(v.data_ptr()), n, None) == -1
    assert noalloc(T, u, u, v, stream) == -1  # output overlaps an input


def test_noalloc_takes_no_device_memory(T):
    stream = torch.cuda.current_stream()
    n = 60000
    u = T.to_device(I.random_limbs(920, 1, n))
    v = T.to_device(I.random_limbs(920, 2, n))
    w = T.empty(2 * n)
    assert noalloc(T, w, u, v, stream) == 0  # first call of this shape: host-side planning
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        assert noalloc(T, w, u, v, stream) == 0
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free0 == free1
    T.sync()
    assert I.to_int(T.to_host(w)) == I.to_int(T.to_host(u)) * I.to_int(T.to_host(v))
