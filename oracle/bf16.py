"""Rounding of parameters to bfloat16 for the reduced-precision ansatz.

The BF16 ansatz stores every parameter as FP64 -> FP32 -> BF16 with
round-to-nearest-even at each step; the oracle then runs in FP64 on exactly those
values, so a GPU result in BF16 mode is compared with the FP64 answer for the same
parameters. (Rounding mode: IEEE round-to-nearest-even, the paper states none.)
"""
from __future__ import annotations

import numpy as np


def round_to_bf16(x: np.ndarray) -> np.ndarray:
    """FP64 -> FP32 (RNE) -> BF16 (RNE) -> back to FP64, exactly."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x: np.ndarray) -> np.ndarray:
    """Upper 16 bits of the rounded FP32 pattern (the BF16 encoding), uint16."""
    r = round_to_bf16(x).astype(np.float32)
    return (r.view(np.uint32) >> np.uint32(16)).astype(np.uint16)
