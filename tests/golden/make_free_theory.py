"""Writes free_theory.txt: exact free-theory (lambda = 0) evidence and mean
|magnetisation| under the Gaussian reference N(0, s2 I), through the oracle's
own action (Sec. 2 Eq. (1)).

With lambda = 0 the action is the quadratic form 1/2 phi^T A phi with
A = m2 I + K, K the periodic nearest-neighbour kinetic matrix.  K is read off
the oracle's action by polarisation (S(e_i + e_j) - S(e_i) - S(e_j) = K_ij at
m2 = 0), then
  log E[exp(-S)] = -1/2 log det(I + s2 A)     (Gaussian integral),
  M = mean of the sites ~ N(0, 1^T (I / s2 + A)^-1 1 / V^2),
  <|M|> = sqrt(2 / pi) * sd(M).
This route shares nothing with the closed form over lattice momenta that
tests/exact.py uses, so the two pin each other.

Run from the repository root:  python tests/golden/make_free_theory.py
"""
import math
import os
import sys

import numpy as np

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
from oracle import action  # noqa: E402

CASES = [(1, 1.0, 1.0), (2, 1.0, 1.0), (2, 1.0, 4.0), (3, 0.5, 1.0), (4, 1.0, 1.0),
         (4, 1.0, 4.0), (5, 2.0, 1.0), (8, 1.0, 1.0), (8, 1.0, 4.0), (16, 1.0, 1.0)]


def kinetic_matrix(L):
    d = L * L
    E = np.eye(d)
    s1 = action.action(E, L, 0.0, 0.0)            # S(e_i) = K_ii / 2
    K = np.empty((d, d))
    for i in range(d):
        K[i] = action.action(E + E[i], L, 0.0, 0.0) - s1 - s1[i]
    return K


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "free_theory.txt")
    lines = ["# Free theory (lambda = 0) under the reference N(0, s2 I): exact",
             "# log E[exp(-S)] and <|M|>, written by make_free_theory.py through the",
             "# oracle's action (Sec. 2 Eq. (1)) and dense determinants.",
             "# L m2 s2 logz mean_abs_m"]
    for L, m2, s2 in CASES:
        d = L * L
        A = m2 * np.eye(d) + kinetic_matrix(L)
        sign, logdet = np.linalg.slogdet(np.eye(d) + s2 * A)
        assert sign > 0
        prec = np.eye(d) / s2 + A
        var = np.ones(d) @ np.linalg.solve(prec, np.ones(d)) / d ** 2
        lines.append(f"{L} {m2!r} {s2!r} {-0.5 * logdet:.15e} {math.sqrt(2 / math.pi * var):.15e}")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


if __name__ == "__main__":
    main()
