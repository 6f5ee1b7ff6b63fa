"""BF16 rounding helpers of the tests (round to nearest even, as the
kernels round)."""
import numpy as np


def bits(a):
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)
    return ((u + (((u >> 16) & 1) + 0x7FFF)) >> 16).astype(np.uint16)


def value(b):
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def round(a):
    return value(bits(a))
