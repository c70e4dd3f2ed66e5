"""Pins of the oracle's Philox4x32-10 streams, uniforms and Box-Muller normals."""

import numpy as np
import pytest
from scipy import stats

from oracle import rng


# The published known-answer vectors are pinned in test_oracle_golden.py
# (tests/golden/philox4x32_10_kat.txt).


def test_philox_broadcasts_like_scalar_calls():
    c0 = np.arange(5)
    vec = rng.philox4x32_10(c0, 7, 3, 0x102, 11, 2)
    for i in range(5):
        one = rng.philox4x32_10(i, 7, 3, 0x102, 11, 2)
        assert all(int(v[i]) == int(o) for v, o in zip(vec, one))


def test_uniform_exact_grid_and_open_interval():
    w = np.array([0, 1, 511, 512, 0xFFFFFFFF, 0x80000000], dtype=np.uint32)
    u = rng.uniform(w)
    assert np.all(u > 0) and np.all(u < 1)
    # exactly representable in float32 and on the (k + 1/2) 2^-23 grid
    assert np.array_equal(u.astype(np.float32).astype(np.float64), u)
    k = u * 2 ** 23 - 0.5
    assert np.array_equal(k, np.floor(k))
    assert u[0] == 2.0 ** -24 and u[4] == 1.0 - 2.0 ** -24 and u[5] == 0.5 + 2.0 ** -24
    assert u[2] == u[0] and u[3] == 3 * 2.0 ** -24


def test_uniform_chi_square():
    w0, w1, w2, w3 = rng.philox4x32_10(np.arange(1 << 15), 1, 2, 3, 42, 0)
    u = rng.uniform(np.concatenate([w0, w1, w2, w3]))
    counts, _ = np.histogram(u, bins=64, range=(0, 1))
    chi2 = ((counts - u.size / 64) ** 2 / (u.size / 64)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4


def test_normal_moments_and_ks():
    z = rng.normals(5, 0, 1, 0, rng.PROPOSE, np.arange(2048), 64).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.kurtosis(z, fisher=False) - 3) < 5 * np.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4


def test_site_mapping_prefix_and_quads():
    full = rng.normals(3, 1, 2, 4, rng.PROPOSE, [0, 9], 8)
    part = rng.normals(3, 1, 2, 4, rng.PROPOSE, [0, 9], 6)
    assert np.array_equal(full[:, :6], part)
    # site 4q + w takes word w of call q: rebuild site 5 by hand
    w0, w1, w2, w3 = rng.philox4x32_10(1, 9, 4, (2 << 8) | rng.PROPOSE, 3, 1)
    z0, z1 = rng.box_muller(w0, w1)
    assert full[1, 5] == z1


def test_streams_differ_by_purpose_level_step_run():
    base = rng.normals(1, 0, 1, 0, rng.PROPOSE, [0], 16)
    for args in [(1, 0, 1, 0, rng.INIT), (1, 0, 2, 0, rng.PROPOSE),
                 (1, 0, 1, 1, rng.PROPOSE), (1, 1, 1, 0, rng.PROPOSE),
                 (2, 0, 1, 0, rng.PROPOSE)]:
        other = rng.normals(*args, [0], 16)
        assert not np.any(other == base)
