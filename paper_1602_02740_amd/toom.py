"""Thin ctypes binding of libtoom.so (include/toom.h).

Argument marshalling only: every step of the multiplication runs in the HIP
kernels of libtoom.so.  torch supplies device memory and streams; limb arrays
are 1-D contiguous int32 tensors on the GPU, viewed as raw 32-bit limbs.
There is no CPU fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtoom.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "toom.h")

TC_OK = 0
VAR_EVENODD = 0
VAR_INF = 1
VAR_HALF = 2
LEAF_SCHOOL = 0
LEAF_NTT = 1
MAX_LEVELS = 16
KERNEL_NAMES = ("eval", "leaf", "step", "recomp")
TC_ERR_INEXACT = -6

_ERRNAMES = {
    -1: "TC_ERR_INVALID", -2: "TC_ERR_NOMEM", -3: "TC_ERR_HIP", -4: "TC_ERR_AGAIN",
    -5: "TC_ERR_NOT_READY", -6: "TC_ERR_INEXACT", -7: "TC_ERR_UNSUPPORTED",
    -8: "TC_ERR_WORKSPACE",
}


class ToomError(RuntimeError):
    def __init__(self, code: int, what: str):
        msg = f"{what}: {_ERRNAMES.get(code, code)}"
        if code == -3 and _lib is not None:
            msg += f" ({_lib.tc_hip_error_string().decode()})"
        super().__init__(msg)
        self.code = code


class Plan(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int),
                ("B", ctypes.c_int * MAX_LEVELS),
                ("variant", ctypes.c_int * MAX_LEVELS),
                ("leaf", ctypes.c_int),
                ("chunk", ctypes.c_int)]

    @classmethod
    def make(cls, Bs: Sequence[int], variants: Optional[Sequence[int]] = None,
             leaf: int = LEAF_SCHOOL, chunk: int = 0) -> "Plan":
        p = cls()
        p.levels = len(Bs)
        for i, b in enumerate(Bs):
            p.B[i] = int(b)
            p.variant[i] = int(variants[i]) if variants is not None else VAR_EVENODD
        p.leaf = int(leaf)
        p.chunk = int(chunk)
        return p

    def as_list(self):
        return [(self.B[i], self.variant[i]) for i in range(self.levels)]


class PlanCost(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 4), ("bytes", ctypes.c_double * 4),
                ("leaf_limb_products", ctypes.c_double)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", ctypes.c_size_t),
                ("max_queued", ctypes.c_size_t), ("streams", ctypes.c_int),
                ("max_batch", ctypes.c_int)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("submit_us", ctypes.c_double),
                ("start_us", ctypes.c_double), ("finish_us", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("queued", ctypes.c_uint64), ("inflight", ctypes.c_uint64),
                ("inflight_bytes", ctypes.c_size_t), ("p50_us", ctypes.c_double),
                ("p99_us", ctypes.c_double), ("limb_mults_per_s", ctypes.c_double),
                ("window_s", ctypes.c_double)]


class MulDesc(ctypes.Structure):
    _fields_ = [("w", ctypes.c_void_p), ("u", ctypes.c_void_p), ("nu", ctypes.c_size_t),
                ("v", ctypes.c_void_p), ("nv", ctypes.c_size_t)]


_lib = None


def header_functions() -> list:
    """Names of the functions declared in include/toom.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(tc_\w+)\s*\(", text, re.M)))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, i32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        P = ctypes.POINTER
        sig = {
            "tc_init": ([], i32),
            "tc_hip_error_string": ([], ctypes.c_char_p),
            "tc_strerror": ([i32], ctypes.c_char_p),
            "tc_mul": ([vp, vp, sz, vp, sz, vp], i32),
            "tc_mul_plan": ([vp, vp, sz, vp, sz, P(Plan), vp], i32),
            "tc_plan_default": ([sz, sz, P(Plan)], i32),
            "tc_workspace_bytes": ([sz, sz], sz),
            "tc_workspace_bytes_plan": ([sz, sz, P(Plan)], sz),
            "tc_mul_batch": ([P(MulDesc), sz, vp, vp], i32),
            "tc_mul_batch_plan": ([P(MulDesc), sz, P(Plan), vp, vp], i32),
            "tc_sync": ([vp], i32),
            "tc_get_error": ([], i32),
            "tc_eval": ([vp, vp, vp, sz, i32, i32, sz, sz, vp], i32),
            "tc_interp": ([vp, sz, vp, vp, sz, i32, i32, vp], i32),
            "tc_recompose": ([vp, sz, vp, sz, i32, sz, vp], i32),
            "tc_school": ([vp, vp, vp, sz, sz, vp], i32),
            "tc_ntt_params": ([sz, sz, P(i32), P(sz), P(sz)], i32),
            "tc_ntt_forward": ([vp, vp, sz, i32, sz, vp], i32),
            "tc_measure_mad_rate": ([P(ctypes.c_double)], i32),
            "tc_debug_fault": ([i32], i32),
            "tc_set_strict": ([i32], i32),
            "tc_mul_noalloc": ([vp, vp, sz, vp, sz, vp], i32),
            "tc_noalloc_capacity": ([], sz),
            "tc_plan_cost_get": ([sz, sz, P(Plan), P(PlanCost)], i32),
            "tc_set_cache_limit": ([sz], i32),
            "tc_autotune": ([sz, sz, i32, P(Plan), P(ctypes.c_double)], i32),
            "tc_autotune_clear": ([], i32),
            "tc_autotune_save": ([ctypes.c_char_p], i32),
            "tc_autotune_load": ([ctypes.c_char_p], i32),
            "tc_autotune_count": ([], i32),
            "tc_server_create": ([P(ServerCfg), P(vp)], i32),
            "tc_submit": ([vp, vp, vp, sz, vp, sz, P(ctypes.c_uint64)], i32),
            "tc_poll": ([vp, ctypes.c_uint64, P(Result)], i32),
            "tc_server_stats": ([vp, P(Stats)], i32),
            "tc_server_reset_stats": ([vp], i32),
            "tc_server_destroy": ([vp], i32),
            "tc_timing_enable": ([i32], i32),
            "tc_timing_read": ([P(ctypes.c_int64), P(ctypes.c_double)], i32),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc: int, what: str):
    if rc != TC_OK:
        raise ToomError(rc, what)


# ------------------------------------------------------------------ tensors

def _torch():
    import torch
    return torch


def _stream(stream) -> ctypes.c_void_p:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _limbs(t, name):
    torch = _torch()
    if t.dtype not in (torch.int32, torch.uint32) or t.dim() != 1 or not t.is_contiguous():
        raise TypeError(f"{name}: expected a 1-D contiguous int32 tensor of limbs")
    if not t.is_cuda:
        raise TypeError(f"{name}: expected a GPU tensor")
    return t


def to_device(a, device="cuda") -> "torch.Tensor":
    """numpy uint32 limbs -> int32 GPU tensor (same bits)."""
    torch = _torch()
    a = np.ascontiguousarray(a, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).to(device)


def to_host(t) -> np.ndarray:
    """int32 GPU tensor -> numpy uint32 limbs."""
    return t.detach().cpu().numpy().view(np.uint32).copy()


def empty(n: int, device="cuda"):
    torch = _torch()
    return torch.empty(int(n), dtype=torch.int32, device=device)


# ------------------------------------------------------------------ products

def init():
    _check(lib().tc_init(), "tc_init")


def plan_default(nu: int, nv: int) -> Plan:
    p = Plan()
    _check(lib().tc_plan_default(nu, nv, ctypes.byref(p)), "tc_plan_default")
    return p


def workspace_bytes(nu: int, nv: int, plan: Optional[Plan] = None) -> int:
    if plan is None:
        return int(lib().tc_workspace_bytes(nu, nv))
    return int(lib().tc_workspace_bytes_plan(nu, nv, ctypes.byref(plan)))


def mul(u, v, plan: Optional[Plan] = None, out=None, stream=None):
    """w = u * v (GPU int32 limb tensors); returns w (nu+nv limbs).  Asynchronous."""
    _limbs(u, "u")
    _limbs(v, "v")
    nu, nv = u.numel(), v.numel()
    w = out if out is not None else empty(nu + nv, u.device)
    _limbs(w, "out")
    if w.numel() != nu + nv:
        raise ValueError("out must have nu+nv limbs")
    if plan is None:
        rc = lib().tc_mul(_ptr(w), _ptr(u), nu, _ptr(v), nv, _stream(stream))
    else:
        rc = lib().tc_mul_plan(_ptr(w), _ptr(u), nu, _ptr(v), nv, ctypes.byref(plan),
                               _stream(stream))
    _check(rc, "tc_mul")
    return w


def batch_descs(us, vs, outs):
    """The tc_mul_desc array of a batch (reusable while the tensors live)."""
    if len(us) != len(vs) or len(us) != len(outs) or not us:
        raise ValueError("need equally many u, v and outputs")
    descs = (MulDesc * len(us))()
    for i, (u, v, w) in enumerate(zip(us, vs, outs)):
        _limbs(u, "u")
        _limbs(v, "v")
        _limbs(w, "out")
        if w.numel() != u.numel() + v.numel():
            raise ValueError("each output must have nu+nv limbs")
        descs[i] = MulDesc(w.data_ptr(), u.data_ptr(), u.numel(), v.data_ptr(), v.numel())
    return descs


def mul_batch(us, vs, plans=None, outs=None, stream=None, descs=None, status=None):
    """Independent products u[i]*v[i] merged level by level; returns outputs.

    `descs` (from batch_descs over the same tensors) skips rebuilding the
    descriptor array on repeated calls.  `status`: None, or a 1-D int32
    tensor of len(us) entries (GPU, or pinned CPU memory) that receives each
    item's TC_OK / TC_ERR_INEXACT in stream order."""
    if len(us) != len(vs) or not us:
        raise ValueError("need equally many u and v")
    outs = outs if outs is not None else [empty(u.numel() + v.numel(), u.device)
                                          for u, v in zip(us, vs)]
    if descs is None:
        descs = batch_descs(us, vs, outs)
    elif len(descs) != len(us):
        raise ValueError("descs does not match the batch")
    sp = None
    if status is not None:
        torch = _torch()
        if status.dtype != torch.int32 or status.numel() != len(us) or not status.is_contiguous():
            raise TypeError("status: expected a contiguous int32 tensor with one entry per item")
        sp = _ptr(status)
    if plans is not None:
        parr = (Plan * len(us))(*plans)
        rc = lib().tc_mul_batch_plan(descs, len(us), parr, sp, _stream(stream))
    else:
        rc = lib().tc_mul_batch(descs, len(us), sp, _stream(stream))
    _check(rc, "tc_mul_batch")
    return outs


def sync(stream=None):
    """Waits for the stream; raises ToomError(TC_ERR_INEXACT) if a device check fired."""
    _check(lib().tc_sync(_stream(stream)), "tc_sync")


# ------------------------------------------------------------------ phases

def ntt_params(na: int, nb: int):
    """(bits, N, C): the piece width, transform length and row length the
    library takes for an na x nb transform leaf."""
    bits, N, C = ctypes.c_int(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().tc_ntt_params(na, nb, ctypes.byref(bits), ctypes.byref(N), ctypes.byref(C)),
           "tc_ntt_params")
    return bits.value, N.value, C.value


def measure_mad_rate() -> float:
    """32 x 32 + 32 -> 64 multiply-adds per second on this GPU (probe)."""
    r = ctypes.c_double()
    _check(lib().tc_measure_mad_rate(ctypes.byref(r)), "tc_measure_mad_rate")
    return r.value


def ntt_forward(u, bits: int, N: int, stream=None):
    """The forward transform of u's pieces in the library's order (int64
    tensor of N raw 64-bit field elements)."""
    torch = _torch()
    _limbs(u, "u")
    X = torch.empty(N, dtype=torch.int64, device=u.device)
    _check(lib().tc_ntt_forward(_ptr(X), _ptr(u), u.numel(), bits, N, _stream(stream)),
           "tc_ntt_forward")
    return X


def eval_points(u, B: int, variant: int, bl: int, nout: int, stream=None):
    torch = _torch()
    npts = 2 * B - 1
    out = empty(npts * nout, u.device)
    sign = torch.zeros(npts, dtype=torch.uint8, device=u.device)
    _check(lib().tc_eval(_ptr(out), _ptr(sign), _ptr(u), u.numel(), B, variant, bl, nout,
                         _stream(stream)), "tc_eval")
    return out.view(npts, nout), sign


def interp(y, sign, B: int, variant: int, nw: int, stream=None):
    npts = 2 * B - 1
    ny = y.numel() // npts
    w = empty(npts * nw, y.device)
    _check(lib().tc_interp(_ptr(w), nw, _ptr(y), _ptr(sign), ny, B, variant, _stream(stream)),
           "tc_interp")
    return w.view(npts, nw)


def recompose(w, B: int, bl: int, nout: int, stream=None):
    npts = 2 * B - 1
    nw = w.numel() // npts
    out = empty(nout, w.device)
    _check(lib().tc_recompose(_ptr(out), nout, _ptr(w), nw, B, bl, _stream(stream)),
           "tc_recompose")
    return out


def school(u, v, n: int, count: int, stream=None):
    p = empty(2 * n * count, u.device)
    _check(lib().tc_school(_ptr(p), _ptr(u), _ptr(v), n, count, _stream(stream)), "tc_school")
    return p.view(count, 2 * n)


def plan_cost(nu: int, nv: int, plan: Optional[Plan] = None) -> dict:
    """Algorithmic bytes and launches per kernel class, leaf limb products
    (plan None: of mul's own choice for these sizes)."""
    c = PlanCost()
    _check(lib().tc_plan_cost_get(nu, nv, ctypes.byref(plan) if plan is not None else None,
                                  ctypes.byref(c)), "tc_plan_cost_get")
    return {"launches": {KERNEL_NAMES[i]: int(c.launches[i]) for i in range(len(KERNEL_NAMES))},
            "bytes": {KERNEL_NAMES[i]: float(c.bytes[i]) for i in range(len(KERNEL_NAMES))},
            "leaf_limb_products": float(c.leaf_limb_products)}


def autotune(nu: int, nv: Optional[int] = None):
    """Times candidate plans for an nu x nv product on this GPU and makes the
    fastest the default for its size class; returns (plan, ms)."""
    nv = nu if nv is None else nv
    p = Plan()
    ms = ctypes.c_double()
    _check(lib().tc_autotune(nu, nv, 0, ctypes.byref(p), ctypes.byref(ms)), "tc_autotune")
    return p, ms.value


def autotune_clear():
    _check(lib().tc_autotune_clear(), "tc_autotune_clear")


def autotune_save(path: str):
    """Writes the tuned plans (JSON, keyed by device) to path."""
    _check(lib().tc_autotune_save(os.fsencode(path)), "tc_autotune_save")


def autotune_load(path: str) -> bool:
    """Loads a saved tuning table; False if it is missing or was tuned on
    another kind of device."""
    rc = lib().tc_autotune_load(os.fsencode(path))
    if rc in (-1, -7):
        return False
    _check(rc, "tc_autotune_load")
    return True


def autotune_count() -> int:
    return int(lib().tc_autotune_count())


def set_strict(on: bool):
    """Strict exactness checks: single-round levels compute every coefficient
    in its own exact step instead of one recomposing step (same results)."""
    _check(lib().tc_set_strict(1 if on else 0), "tc_set_strict")


def debug_fault(item: int):
    """Test hook: later products of batch item `item` (single products: 0)
    get one flipped bit in a top-level point product, which the kernels'
    exactness checks must report; -1 turns it off."""
    _check(lib().tc_debug_fault(int(item)), "tc_debug_fault")


# ------------------------------------------------------------------ timing

def timing_enable(on: bool = True):
    _check(lib().tc_timing_enable(1 if on else 0), "tc_timing_enable")


def timing_read() -> dict:
    k = len(KERNEL_NAMES)
    n = (ctypes.c_int64 * k)()
    ms = (ctypes.c_double * k)()
    _check(lib().tc_timing_read(n, ms), "tc_timing_read")
    return {KERNEL_NAMES[i]: (int(n[i]), float(ms[i])) for i in range(k)}


# ------------------------------------------------------------------ serving

class Server:
    """Continuous-batching request loop of libtoom.so on the current device.

    submit() queues w = u v and returns a ticket at once; poll() returns None
    while the request is queued or running, then its result record.  The
    tensors of a request are kept alive here until it has been reported."""

    def __init__(self, hbm_budget: int = 0, max_inflight: int = 0, max_queued: int = 0,
                 streams: int = 0, max_batch: int = 0):
        cfg = ServerCfg(hbm_budget, max_inflight, max_queued, streams, max_batch)
        h = ctypes.c_void_p()
        _check(lib().tc_server_create(ctypes.byref(cfg), ctypes.byref(h)), "tc_server_create")
        self._h = h
        self._live = {}

    def submit(self, u, v, out) -> int:
        _limbs(u, "u")
        _limbs(v, "v")
        _limbs(out, "out")
        if out.numel() != u.numel() + v.numel():
            raise ValueError("out must have nu+nv limbs")
        t = ctypes.c_uint64()
        _check(lib().tc_submit(self._h, _ptr(out), _ptr(u), u.numel(), _ptr(v), v.numel(),
                               ctypes.byref(t)), "tc_submit")
        self._live[t.value] = (u, v, out)
        return t.value

    def poll(self, ticket: int):
        r = Result()
        rc = lib().tc_poll(self._h, ticket, ctypes.byref(r))
        if rc == -5:
            return None
        _check(rc, "tc_poll")
        self._live.pop(ticket, None)
        return {"status": r.status, "submit_us": r.submit_us, "start_us": r.start_us,
                "finish_us": r.finish_us}

    def stats(self) -> dict:
        st = Stats()
        _check(lib().tc_server_stats(self._h, ctypes.byref(st)), "tc_server_stats")
        return {f: getattr(st, f) for f, _ in Stats._fields_}

    def reset_stats(self):
        _check(lib().tc_server_reset_stats(self._h), "tc_server_reset_stats")

    def close(self):
        if self._h:
            _check(lib().tc_server_destroy(self._h), "tc_server_destroy")
            self._h = None
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def set_cache_limit(nbytes: int):
    """Device bytes cached compiled plans may hold (least-recently-used beyond)."""
    _check(lib().tc_set_cache_limit(int(nbytes)), "tc_set_cache_limit")
