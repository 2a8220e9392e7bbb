"""ctypes binding of the CPU oracle (``oracle/toomref.c``, ``oracle/nttref.c``).

TEST INFRASTRUCTURE ONLY: the checker for the GPU library.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg import this
package.  It imports nothing from the GPU package and the GPU package imports
nothing from it.

Arrays are numpy ``uint32`` limb vectors, little-endian (limb 0 least
significant).  Every call raises ``OracleError`` when the C side reports a
failure (an inexact division, a value that overflows its width, ...).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SOURCES = [os.path.join(_HERE, "toomref.c"), os.path.join(_HERE, "nttref.c")]

VAR_EVENODD = 0
VAR_INF = 1
VAR_PLAIN = 2
VAR_ODD_DIRECT = 3
VAR_HALF = 4
MAX_LEVELS = 16

ERRORS = {-1: "bad argument", -2: "inexact division", -3: "value out of range", -4: "out of memory"}


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain -O2, pthreads)."""
    if not force and os.path.exists(LIB_PATH):
        return LIB_PATH
    tmp = LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-o", tmp] + SOURCES + ["-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Plan(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int),
                ("B", ctypes.c_int * MAX_LEVELS),
                ("variant", ctypes.c_int * MAX_LEVELS),
                ("threads", ctypes.c_int),
                ("leaf_ntt_bits", ctypes.c_int)]


class Counts(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in
                ("leaves", "leaf_mults", "toom_nodes", "eval_limbs",
                 "interp_steps", "interp_limbs", "recomp_limbs")]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        u32p, i8p, i64p = P(ctypes.c_uint32), P(ctypes.c_int8), P(ctypes.c_int64)
        sz = ctypes.c_size_t
        L.tcref_growth_limbs.argtypes = [ctypes.c_int, ctypes.c_int]
        L.tcref_growth_limbs.restype = sz
        L.tcref_block_limbs.argtypes = [sz, ctypes.c_int]
        L.tcref_block_limbs.restype = sz
        L.tcref_mul_school.argtypes = [u32p, u32p, sz, u32p, sz]
        L.tcref_mul_toom.argtypes = [u32p, u32p, sz, u32p, sz, P(Plan)]
        L.tcref_eval.argtypes = [ctypes.c_int, ctypes.c_int, u32p, sz, sz, sz, u32p, i8p]
        L.tcref_interp.argtypes = [ctypes.c_int, ctypes.c_int, sz, u32p, i8p, sz, u32p]
        L.tcref_recompose.argtypes = [ctypes.c_int, sz, sz, u32p, sz, u32p]
        L.tcref_newton.argtypes = [ctypes.c_int, i64p, sz, u32p, i8p, u32p, i8p, ctypes.c_int]
        L.tcref_counts_reset.argtypes = []
        L.tcref_counts_reset.restype = None
        L.tcref_counts_get.argtypes = [P(Counts)]
        L.tcref_counts_get.restype = None
        L.tcref_plan_counts.argtypes = [sz, P(Plan), P(Counts)]
        u64p = P(ctypes.c_uint64)
        L.tcref_ntt_root.argtypes = [ctypes.c_uint64]
        L.tcref_ntt_root.restype = ctypes.c_uint64
        L.tcref_ntt.argtypes = [u64p, sz, ctypes.c_int]
        L.tcref_ntt_npieces.argtypes = [sz, ctypes.c_int]
        L.tcref_ntt_npieces.restype = sz
        L.tcref_ntt_pieces.argtypes = [u32p, sz, ctypes.c_int, u64p, sz]
        L.tcref_mul_ntt.argtypes = [u32p, u32p, sz, u32p, sz, ctypes.c_int]
        for f in ("tcref_mul_school", "tcref_mul_toom", "tcref_eval", "tcref_interp",
                  "tcref_recompose", "tcref_newton", "tcref_plan_counts", "tcref_ntt",
                  "tcref_ntt_pieces", "tcref_mul_ntt"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _p(a, ctype=ctypes.c_uint32):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what}: {ERRORS.get(rc, rc)}")


def make_plan(Bs, variants=None, threads=1, ntt_bits=0) -> Plan:
    p = Plan()
    p.levels = len(Bs)
    for i, b in enumerate(Bs):
        p.B[i] = int(b)
        p.variant[i] = int(variants[i]) if variants is not None else VAR_EVENODD
    p.threads = int(threads)
    p.leaf_ntt_bits = int(ntt_bits)
    return p


def growth_limbs(B: int, variant: int = VAR_EVENODD) -> int:
    return int(lib().tcref_growth_limbs(B, variant))


def block_limbs(n: int, B: int) -> int:
    return int(lib().tcref_block_limbs(n, B))


def mul_school(u, v) -> np.ndarray:
    u, v = _u32(u), _u32(v)
    w = np.zeros(len(u) + len(v), dtype=np.uint32)
    _check(lib().tcref_mul_school(_p(w), _p(u), len(u), _p(v), len(v)), "mul_school")
    return w


def mul_toom(u, v, Bs, variants=None, threads=1, ntt_bits=0) -> np.ndarray:
    """Recursive Toom-Cook product; ntt_bits > 0 forms the leaves with
    mul_ntt (section 5's Toom-Cook over an FFT product)."""
    u, v = _u32(u), _u32(v)
    w = np.zeros(len(u) + len(v), dtype=np.uint32)
    plan = make_plan(Bs, variants, threads, ntt_bits)
    _check(lib().tcref_mul_toom(_p(w), _p(u), len(u), _p(v), len(v), ctypes.byref(plan)),
           "mul_toom")
    return w


def npoints(B: int) -> int:
    return 2 * B - 1


def eval_points(B, variant, u, bl, nout):
    """(2B-1, nout) magnitudes and (2B-1,) signs (1 = negative)."""
    u = _u32(u)
    out = np.zeros((npoints(B), nout), dtype=np.uint32)
    sign = np.zeros(npoints(B), dtype=np.int8)
    _check(lib().tcref_eval(B, variant, _p(u), len(u), bl, nout, _p(out),
                            _p(sign, ctypes.c_int8)), "eval")
    return out, sign


def interp(B, variant, y, sign, nw):
    """y: (2B-1, ny) magnitudes; sign: (2B-1,) -> (2B-1, nw) coefficients."""
    y = _u32(y)
    sign = np.ascontiguousarray(sign, dtype=np.int8)
    assert y.shape[0] == npoints(B)
    w = np.zeros((npoints(B), nw), dtype=np.uint32)
    _check(lib().tcref_interp(B, variant, y.shape[1], _p(y), _p(sign, ctypes.c_int8), nw,
                              _p(w)), "interp")
    return w


def recompose(B, bl, w, nout):
    w = _u32(w)
    out = np.zeros(nout, dtype=np.uint32)
    _check(lib().tcref_recompose(B, bl, w.shape[1], _p(w), nout, _p(out)), "recompose")
    return out


def newton(x, ymag, ysign, phase=2):
    """Section 3's loops on int64 nodes x[0..n]; ymag: (n+1, nl)."""
    x = np.ascontiguousarray(x, dtype=np.int64)
    ymag = _u32(ymag)
    ysign = np.ascontiguousarray(ysign, dtype=np.int8)
    n = len(x) - 1
    cmag = np.zeros_like(ymag)
    csign = np.zeros(n + 1, dtype=np.int8)
    _check(lib().tcref_newton(n, _p(x, ctypes.c_int64), ymag.shape[1], _p(ymag),
                              _p(ysign, ctypes.c_int8), _p(cmag), _p(csign, ctypes.c_int8),
                              phase), "newton")
    return cmag, csign


def counts_reset():
    lib().tcref_counts_reset()


def counts_get() -> dict:
    c = Counts()
    lib().tcref_counts_get(ctypes.byref(c))
    return c.as_dict()


def plan_counts(n, Bs, variants=None) -> dict:
    c = Counts()
    plan = make_plan(Bs, variants)
    _check(lib().tcref_plan_counts(n, ctypes.byref(plan), ctypes.byref(c)), "plan_counts")
    return c.as_dict()


# ---- number-theoretic transform (nttref.c)

NTT_P = (1 << 64) - (1 << 32) + 1


def ntt_root(N: int) -> int:
    """w_N = 7^((p-1)/N) for a power of two N <= 2^32 (0 otherwise)."""
    return int(lib().tcref_ntt_root(N))


def ntt(x, inverse=False) -> np.ndarray:
    """X[j] = sum_i x[i] w_N^(i j) mod p (inverse: N^-1 sum_j X[j] w_N^(-i j))."""
    x = np.array(x, dtype=np.uint64)
    _check(lib().tcref_ntt(_p(x, ctypes.c_uint64), len(x), 1 if inverse else 0), "ntt")
    return x


def ntt_npieces(n: int, bits: int) -> int:
    return int(lib().tcref_ntt_npieces(n, bits))


def ntt_pieces(u, bits: int, nout: int) -> np.ndarray:
    u = _u32(u)
    out = np.zeros(nout, dtype=np.uint64)
    _check(lib().tcref_ntt_pieces(_p(u), len(u), bits, _p(out, ctypes.c_uint64), nout),
           "ntt_pieces")
    return out


def mul_ntt(u, v, bits: int) -> np.ndarray:
    u, v = _u32(u), _u32(v)
    w = np.zeros(len(u) + len(v), dtype=np.uint32)
    _check(lib().tcref_mul_ntt(_p(w), _p(u), len(u), _p(v), len(v), bits), "mul_ntt")
    return w
