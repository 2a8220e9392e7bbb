"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/toom.h declares, and rejects bad arguments on the host
before touching a device."""
import ctypes
import os

import pytest

from paper_1602_02740_amd import toom

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_boundary():
    names = toom.header_functions()
    for f in ("tc_mul", "tc_mul_plan", "tc_mul_batch", "tc_sync", "tc_get_error",
              "tc_strerror", "tc_eval", "tc_interp", "tc_recompose", "tc_school",
              "tc_workspace_bytes", "tc_plan_default", "tc_timing_enable", "tc_timing_read"):
        assert f in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(toom.LIB_PATH)
    missing = [f for f in toom.header_functions() if not hasattr(L, f)]
    assert not missing, missing


def test_binding_covers_header():
    L = toom.lib()
    for f in toom.header_functions():
        assert getattr(L, f).restype is not None or f in ()


def test_argument_errors_on_host():
    L = toom.lib()
    null = ctypes.c_void_p(0)
    one = ctypes.c_void_p(4096)
    assert L.tc_mul(null, one, 1, one, 1, null) == -1
    assert L.tc_mul(one, one, 0, one, 1, null) == -1
    p = toom.Plan.make([3], [toom.VAR_INF])
    p.B[0] = 4  # infinity variant needs B = 3
    w = ctypes.c_void_p(1 << 20)
    assert L.tc_mul_plan(w, one, 8, one, 8, ctypes.byref(p), null) == -1
    # w overlapping u
    assert L.tc_mul(one, ctypes.c_void_p(4096 + 4), 4, w, 4, null) == -1
    assert L.tc_strerror(-6) == b"device exactness check failed"


def test_batch_aliasing_rejected_on_host():
    """Item outputs may not overlap each other or any item's input; checked
    on the host before any device work (no GPU needed: fake addresses)."""
    L = toom.lib()
    D = toom.MulDesc
    descs = (D * 3)()
    base = 1 << 40
    descs[0] = D(base, base + 10000, 100, base + 20000, 100)          # w: 800 bytes
    descs[1] = D(base + 400, base + 30000, 100, base + 40000, 100)    # w overlaps item 0's w
    descs[2] = D(base + 50000, base + 60000, 100, base + 70000, 100)
    assert L.tc_mul_batch(descs, 3, None, None) == -1
    descs[1] = D(base + 80000, base + 50000 + 100, 100, base + 40000, 100)  # u inside item 2's w
    assert L.tc_mul_batch(descs, 3, None, None) == -1
    descs[1] = D(base + 80000, base + 30000, 100, base + 400, 100)    # v inside item 0's w
    assert L.tc_mul_batch(descs, 3, None, None) == -1
    descs[1] = D(base + 80000, base + 80000 + 800, 100, base + 40000, 100)  # adjacent: fine
    assert L.tc_mul_batch(descs, 0, None, None) == -1  # count 0


def test_default_plans():
    # no Toom level while one leaf does (vector ALUs to 32 limbs, matrix
    # cores to 2048); above, levels until the children fit a 2048-limb leaf
    for n in (1, 100, 512, 513, 2048):
        assert toom.plan_default(n, n).levels == 0
    for n, leaf_max in ((2049, 2048), (5000, 2048), (1 << 19, 2048), (1 << 25, 2048)):
        p = toom.plan_default(n, n)
        assert p.levels >= 1
        w = n
        for B, var in p.as_list():
            assert 2 <= B <= 32 and var == toom.VAR_EVENODD
            w = (w + B - 1) // B + (1 if B <= 3 else ((B - 1) * (B - 2) + 1 + 31) // 32)
        assert w <= max(leaf_max, 1)
    p = toom.plan_default(1 << 19, 1 << 19)
    assert p.as_list()[0][0] == 16
    p = toom.plan_default(1 << 25, 1 << 25)
    assert p.as_list()[0][0] == 32


def test_oracle_and_gpu_library_share_no_source():
    """The checker and the product are independent: no common files, and
    neither includes or imports the other."""
    csrc = os.path.join(ROOT, "paper_1602_02740_amd", "csrc")
    for f in os.listdir(csrc):
        text = open(os.path.join(csrc, f)).read()
        assert "toomref" not in text and "oracle" not in text.lower(), f
    for f in ("toom.py", "inputs.py", "build.py", "__init__.py"):
        text = open(os.path.join(ROOT, "paper_1602_02740_amd", f)).read()
        assert "import oracle" not in text and "from oracle" not in text, f
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".c", ".h", ".py")):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1602_02740_amd" not in text and "toom.h" not in text, f
