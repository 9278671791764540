"""Rounding emulator for the low-precision storage regime (Sections III-B, IV).

Test infrastructure only (see the package docstring).

The paper simulates floating-point types with a selectable number of stored
mantissa bits and applies them either to every arithmetic operation or only to
stored intermediates (Section IV, Methodology). A matrix product whose operands
are stored in a narrow type and whose products are accumulated in a wide type
is the storage regime: here the operands are rounded, the sum is formed in
float64, so the emulated product differs from an FP32-accumulating GPU product
only by the accumulation's own rounding.

Reading (listed in the design notes): round to nearest, ties to even; the
exponent range is that of the named format (gradual underflow below the
smallest normal, values above the largest finite clamp to it).
"""
from __future__ import annotations

import numpy as np

# name: (significand bits incl. the implicit one, smallest normal exponent, largest finite)
FORMATS = {
    "fp64": (53, -1022, np.finfo(np.float64).max),
    "fp32": (24, -126, float(np.finfo(np.float32).max)),
    "bf16": (8, -126, float.fromhex("0x1.fep127")),
    "fp16": (11, -14, 65504.0),
    "fp8_e4m3": (4, -6, 448.0),
}

# exponent of the power of two that places a tile's largest magnitude in
# [2^TOP, 2^(TOP+1)) before rounding; None = no per-tile scaling
TILE_TOP = {"bf16": None, "fp16": 14, "fp8_e4m3": 7, "fp64": None, "fp32": None}


def round_to_format(x: np.ndarray, fmt: str) -> np.ndarray:
    """Round float64 values to the named format, returned as float64."""
    t, emin, vmax = FORMATS[fmt]
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)                   # x = m 2^e, 0.5 <= |m| < 1
    e = np.maximum(e - 1, emin)          # exponent of the leading bit, floored at emin
    ulp = np.ldexp(1.0, e - (t - 1))
    y = np.rint(x / ulp) * ulp           # rint: round half to even
    return np.clip(y, -vmax, vmax)


def round_custom(x: np.ndarray, mantissa_bits: int) -> np.ndarray:
    """Round to a float with ``mantissa_bits`` stored bits and an unbounded
    exponent (the custom types of Section IV-B; "mantissa bits" counts stored
    bits, as in the footnotes of Section III-A)."""
    x = np.asarray(x, dtype=np.float64)
    _, e = np.frexp(x)
    ulp = np.ldexp(1.0, e - 1 - mantissa_bits)
    return np.rint(x / ulp) * ulp


def tile_exponents(x: np.ndarray, fmt: str, tile: int = 128) -> np.ndarray:
    """Per-tile power-of-two exponent e such that the tile's largest magnitude
    divided by 2^e lies in [2^TOP, 2^(TOP+1)); 0 for an all-zero tile or an
    unscaled format."""
    top = TILE_TOP[fmt]
    nr = -(-x.shape[0] // tile)
    nc = -(-x.shape[1] // tile)
    ex = np.zeros((nr, nc), dtype=np.int64)
    if top is None:
        return ex
    for bi in range(nr):
        for bj in range(nc):
            blk = x[bi * tile:(bi + 1) * tile, bj * tile:(bj + 1) * tile]
            amax = float(np.max(np.abs(blk))) if blk.size else 0.0
            if amax > 0:
                ex[bi, bj] = int(np.frexp(amax)[1] - 1) - top
    return ex


def quantize(x: np.ndarray, fmt: str, tile: int = 128):
    """Store x in ``fmt`` with per-tile power-of-two scales. Returns
    (codes, exponents): codes are the format's values (as float64) and
    x ~= codes * 2^exponent tile by tile."""
    ex = tile_exponents(x, fmt, tile)
    full = np.repeat(np.repeat(ex, tile, axis=0), tile, axis=1)[: x.shape[0], : x.shape[1]]
    codes = round_to_format(np.ldexp(x, -full), fmt)
    return codes, ex


def dequantize(codes: np.ndarray, ex: np.ndarray, tile: int = 128) -> np.ndarray:
    full = np.repeat(np.repeat(ex, tile, axis=0), tile, axis=1)[: codes.shape[0], : codes.shape[1]]
    return np.ldexp(codes, full)


def lowp_matmul(a: np.ndarray, b: np.ndarray, fmt: str, tile: int = 128) -> np.ndarray:
    """Product of the stored (rounded, tile-scaled) operands, summed in float64."""
    qa, ea = quantize(a, fmt, tile)
    qb, eb = quantize(b, fmt, tile)
    return dequantize(qa, ea, tile) @ dequantize(qb, eb, tile)
