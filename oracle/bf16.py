"""bfloat16 storage emulation (oracle).

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

bfloat16 keeps the sign, the 8-bit exponent and the top 7 fraction bits of an
IEEE binary32 value.  Values are first rounded to binary32 (round to nearest
even, NumPy's cast) and then to bfloat16 with round-to-nearest, ties to even,
on the 16 discarded bits.  NaN stays NaN.
"""
import numpy as np


def bf16_round(x):
    """Return x rounded to bfloat16 (RNE), as float64.
    Pinned by: exactly representable values, halfway cases (ties to even)
    and a brute-force nearest-neighbour search in tests."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out
