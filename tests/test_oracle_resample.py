"""Pins of the oracle's integer-CDF systematic resampling."""

from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import smc


def _ancestors_by_fractions(w, U):
    """Independent route: exact rationals, a_i = min{j: C_j/Q > (i + U/2^32)/N}."""
    n = len(w)
    k = smc.resample_bits(n)
    wmax = max(w)
    q = [int(Fraction(float(x) / float(wmax)) * 2 ** k) for x in w]
    Q = sum(q)
    out = []
    for i in range(n):
        pos = (Fraction(i) + Fraction(int(U), 2 ** 32)) / n * Q
        c = 0
        for j, qj in enumerate(q):
            c += qj
            if c > pos:
                out.append(j)
                break
    return np.array(out)


def test_bits():
    assert smc.resample_bits(16384) == 34
    assert smc.resample_bits(4096) == 38
    assert smc.resample_bits(4097) == 36
    assert smc.resample_bits(2) == 60


@pytest.mark.parametrize("n", [1, 2, 7, 64, 100])
@pytest.mark.parametrize("U", [0, 1, 0x7FFFFFFF, 0xFFFFFFFF])
def test_matches_exact_rationals(n, U):
    w = np.exp(synth.log_weights(n, n, spread=2.0))
    np.testing.assert_array_equal(smc.systematic_resample(w, U), _ancestors_by_fractions(w, U))


@pytest.mark.parametrize("U", [0, 12345, 0xFFFFFFFF])
def test_equal_weights_identity(U):
    np.testing.assert_array_equal(smc.systematic_resample(np.ones(1000), U), np.arange(1000))


def test_one_hot_is_constant():
    w = np.zeros(50)
    w[17] = 0.3
    assert np.all(smc.systematic_resample(w, 999) == 17)


def test_copy_counts_floor_or_ceil_and_sorted():
    n = 4096
    w = np.exp(synth.log_weights(3, n))
    k = smc.resample_bits(n)
    q = np.floor(np.ldexp(w / w.max(), k))
    W = q / q.sum()
    for U in (0, 0x9E3779B9, 0xFFFFFFFF):
        a = smc.systematic_resample(w, U)
        assert np.all(np.diff(a) >= 0)
        counts = np.bincount(a, minlength=n)
        lo, hi = np.floor(n * W), np.ceil(n * W)
        assert np.all((counts >= lo) & (counts <= hi))


def test_unbiased_copy_counts_over_offsets():
    n = 32
    w = np.exp(synth.log_weights(4, n))
    Us = np.linspace(0, 2 ** 32 - 1, 2001).astype(np.uint64)
    mean = np.mean([np.bincount(smc.systematic_resample(w, int(U)), minlength=n)
                    for U in Us], axis=0)
    np.testing.assert_allclose(mean, n * w / w.sum(), atol=2e-3 * n)


def test_empty_and_bad_weights():
    assert smc.systematic_resample(np.zeros(0), 5).shape == (0,)
    with pytest.raises(smc.DegenerateWeights):
        smc.systematic_resample(np.array([1.0, np.nan]), 5)
    with pytest.raises(smc.DegenerateWeights):
        smc.systematic_resample(np.zeros(3), 5)
