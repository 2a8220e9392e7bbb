"""MI355X-native B-way Toom-Cook multiplication of 32-bit-limb integers.

The arithmetic runs in HIP kernels for gfx950 behind the C ABI declared in
include/toom.h (library ``libtoom.so`` in this directory); ``toom`` is the thin
ctypes binding, ``inputs`` the seeded operand generators.
"""
__all__ = ["inputs", "toom"]
