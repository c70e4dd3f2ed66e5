"""Stored reference values (tests/golden/) against the oracle and the exact
closed forms.

* philox4x32_10_kat.txt: the generator's published known-answer vectors
  (Salmon et al., SC'11);
* free_theory.txt: free-theory (lambda = 0, Sec. 2 Eq. (1)) log Z and <|M|>
  under N(0, s2 I), written by make_free_theory.py from dense determinants of
  the kinetic matrix read off the oracle's action, against the closed form
  over lattice momenta (tests/exact.py) and the float64 SMC sampler.
"""
import math
import os

import numpy as np
import pytest

import exact
from oracle import rng
from oracle import smc

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(HERE, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


KAT = [tuple(int(w, 16) for w in r) for r in _rows("philox4x32_10_kat.txt")]
FREE = [(int(r[0]), float(r[1]), float(r[2]), float(r[3]), float(r[4]))
        for r in _rows("free_theory.txt")]


@pytest.mark.parametrize("row", KAT)
def test_philox_known_answers(row):
    got = rng.philox4x32_10(*row[:6])
    assert tuple(int(x) for x in got) == row[6:]


@pytest.mark.parametrize("L,m2,s2,logz,absm", FREE)
def test_free_theory_closed_form(L, m2, s2, logz, absm):
    assert exact.free_logz(L, m2, s2) == pytest.approx(logz, rel=1e-12, abs=1e-12)
    assert exact.free_mean_abs_m(L, m2, s2) == pytest.approx(absm, rel=1e-12)


def test_free_theory_sampler_4x4():
    """The float64 SMC sampler on the stored L = 4 value (enough steps per
    level for the finite-mixing offset to sit inside the replica error)."""
    L, m2, s2, logz, _ = next(r for r in FREE if r[0] == 4 and r[2] == 1.0)
    z = np.array([smc.smc_run(L, m2, 0.0, 1024, 0.5, 50, seed=s)["logz"] for s in range(4)])
    se = z.std(ddof=1) / math.sqrt(len(z))
    assert abs(z.mean() - logz) < 3 * se + 0.1
