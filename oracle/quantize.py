"""Storage casts of coefficient tables: FP64 -> FP32 -> BF16, round to nearest even.

The paper fixes no storage precision; reduced-precision tables are the
precision form of the method.  FP64 -> FP32 is numpy's cast (IEEE round to
nearest even).  FP32 -> BF16 keeps the upper 16 bits of the FP32 pattern after
adding 0x7FFF plus the lowest kept bit (round half to even on the dropped 16
bits); NaNs stay NaN.
"""
import numpy as np


def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def f32_to_bf16_bits(x32):
    x32 = np.ascontiguousarray(x32, dtype=np.float32)
    u = x32.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    nan = np.isnan(x32)
    out = rounded.astype(np.uint16)
    out[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)      # quiet NaN, sign kept
    return out


def to_bf16_bits(x):
    return f32_to_bf16_bits(to_f32(x))


def bf16_bits_to_f64(bits):
    u = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def quantized(x, dtype):
    """The FP64 value of x after storage in ``dtype`` ('f64', 'f32' or 'bf16')."""
    if dtype == "f64":
        return np.asarray(x, dtype=np.float64)
    if dtype == "f32":
        return to_f32(x).astype(np.float64)
    if dtype == "bf16":
        return bf16_bits_to_f64(to_bf16_bits(x))
    raise ValueError(dtype)
