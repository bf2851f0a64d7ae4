"""Round-to-nearest-even emulation of float32 and bfloat16 storage.

Used to build the input-quantised oracle for the reduced-precision operator:
values are rounded float64 -> float32 -> bfloat16 (bfloat16 keeps the top 16
bits of the float32 pattern, rounded to nearest, ties to even), then the
operator is evaluated in float64 on the rounded inputs.
Pins: agreement with torch's CPU float32 -> bfloat16 cast on random and tie
cases (tests/test_oracle_quant.py).
"""
import numpy as np


def to_f32(a):
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def to_bf16(a):
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
