"""Small helpers shared by the tests (conversions only, no method arithmetic)."""
import numpy as np

from paper_1602_02740_amd.inputs import from_int, to_int


def signed_to_sm(values, nl):
    """Signed Python ints -> (magnitudes (k, nl) uint32, signs (k,) int8)."""
    mag = np.zeros((len(values), nl), dtype=np.uint32)
    sign = np.zeros(len(values), dtype=np.int8)
    for i, x in enumerate(values):
        mag[i] = from_int(abs(x), nl)
        sign[i] = 1 if x < 0 else 0
    return mag, sign


def sm_to_signed(mag, sign):
    return [(-1 if s else 1) * to_int(m) for m, s in zip(mag, sign)]


def residue(limbs, p):
    """limbs mod p by Horner from the top limb (independent of any product)."""
    r = 0
    for x in reversed(np.asarray(limbs, dtype=np.uint64).tolist()):
        r = (r * 4294967296 + int(x)) % p
    return r


def residue_np(limbs, p):
    """Vectorised limbs mod p for large vectors: sum of limb_i * (2^32)^i mod p."""
    a = np.asarray(limbs, dtype=np.uint64) % np.uint64(p)
    n = len(a)
    # powers of 2^32 mod p, by repeated squaring blocks (p < 2^32 keeps products < 2^64)
    pw = np.empty(n, dtype=np.uint64)
    base = (1 << 32) % p
    cur = 1
    blk = 1 << 12
    head = np.empty(min(blk, n), dtype=np.uint64)
    for i in range(len(head)):
        head[i] = cur
        cur = (cur * base) % p
    step = cur  # base^blk mod p
    m = 1
    for s in range(0, n, blk):
        e = min(blk, n - s)
        pw[s:s + e] = (head[:e] * np.uint64(m)) % np.uint64(p)
        m = (m * step) % p
    # each term < p < 2^32, so fewer than 2^32 terms cannot overflow uint64
    return int(np.sum((a * pw) % np.uint64(p), dtype=np.uint64)) % p
