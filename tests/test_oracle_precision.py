"""Pins of the round-to-nearest-even emulation of reduced-precision operands."""

import numpy as np
import pytest

from oracle import precision as pr


def _bf16_nearest(x):
    """Independent route: pick the nearest of the two neighbouring bf16 values."""
    x = np.float32(x)
    b = int(np.array([x]).view(np.uint32)[0])
    lo = b & 0xFFFF0000
    hi = lo + 0x10000
    vlo = float(np.array([lo], dtype=np.uint32).view(np.float32)[0])
    vhi = float(np.array([hi & 0xFFFFFFFF], dtype=np.uint32).view(np.float32)[0])
    dlo, dhi = abs(float(x) - vlo), abs(float(x) - vhi)
    if dlo < dhi or (dlo == dhi and ((lo >> 16) & 1) == 0):
        return vlo
    return vhi


def test_bf16_ties_to_even():
    assert pr.bf16_rne(np.float32(1 + 2 ** -8)) == 1.0
    assert pr.bf16_rne(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)
    assert pr.bf16_rne(np.float32(-(1 + 2 ** -8))) == -1.0


def test_bf16_matches_nearest_search():
    x = np.random.default_rng(0).standard_normal(3000).astype(np.float32) * 7
    got = pr.bf16_rne(x)
    want = np.array([_bf16_nearest(v) for v in x], dtype=np.float32)
    np.testing.assert_array_equal(got, want)


def test_odd_symmetry_and_nan():
    x = np.random.default_rng(1).standard_normal(10000).astype(np.float32)
    np.testing.assert_array_equal(pr.bf16_rne(-x), -pr.bf16_rne(x))
    np.testing.assert_array_equal(pr.f16_rne(-x), -pr.f16_rne(x))
    assert np.isnan(pr.bf16_rne(np.float32(np.nan)))


def test_round_operand_chain():
    x = np.array([1.0 + 2 ** -30, -0.1])
    assert np.array_equal(pr.round_operand(x, "fp64"), x)
    assert np.array_equal(pr.round_operand(x, "fp32"), x.astype(np.float32).astype(np.float64))
    assert pr.round_operand(x, "bf16")[0] == 1.0
    with pytest.raises(ValueError):
        pr.round_operand(x, "fp8")
