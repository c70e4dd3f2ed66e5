"""Round-to-nearest-even emulation of reduced-precision operands (test infrastructure only).

The reduced-precision form of the proposal (random-walk increment eps * L * z
with the product in bfloat16 or float16 and float32 accumulation) rounds both
operands with round-to-nearest-even.  Because RNE is an odd function
(round(-x) = -round(x)) and z is symmetric, the rounded increment is still a
symmetric proposal, so the Metropolis ratio needs no Hastings term (the
proposal of App. A stays a random walk).

Operands reach the reduced format through float32: float64 -> float32 (RNE) ->
bfloat16 / float16 (RNE).  The oracle reproduces exactly that chain and then
computes the product in float64.

Pins (tests/test_oracle_precision.py): exhaustive agreement with numpy's
float16 conversion, the bfloat16 definition checked on hand-picked ties and
odd symmetry.
"""

import numpy as np


def to_f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def bf16_rne(x):
    """Round float32 values to bfloat16 (RNE), returned as float32 values.

    bfloat16 keeps the top 16 bits of the float32 pattern; the discarded low
    half is rounded to nearest, ties to the even kept pattern.  NaN stays NaN.
    """
    x = np.asarray(x, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = (r & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
    return np.where(np.isnan(x), x, out)


def f16_rne(x):
    """Round float32 values to float16 (RNE), returned as float32 values."""
    x = np.asarray(x, dtype=np.float32)
    return x.astype(np.float16).astype(np.float32)


def round_operand(x, precision):
    """float64 operand -> value the given proposal precision multiplies with.

    precision: 'fp64' (no rounding), 'fp32', 'bf16' or 'fp16'.
    """
    if precision == "fp64":
        return np.asarray(x, dtype=np.float64)
    x32 = to_f32(x)
    if precision == "fp32":
        return x32.astype(np.float64)
    if precision == "bf16":
        return bf16_rne(x32).astype(np.float64)
    if precision == "fp16":
        return f16_rne(x32).astype(np.float64)
    raise ValueError(f"unknown precision {precision!r}")
