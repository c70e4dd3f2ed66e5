"""Exact values the sampler's estimates are pinned to (independent of the oracle).

* free theory (lambda = 0): with prior N(0, s2 I) the evidence
  E[exp(-S)] factorises over the eigenmodes of the periodic lattice Laplacian,
  log Z = -1/2 sum_k log(1 + s2 (m^2 + lambda_k)),
  lambda_k = 4 sin^2(pi k0 / L) + 4 sin^2(pi k1 / L)  (Sec. 2 Eq. (1) with
  lambda = 0 is the quadratic form 1/2 phi^T (m^2 - Laplacian) phi);
* magnetisation of the free theory: M is the k = 0 mode, Gaussian with
  variance s2 / (V (1 + s2 m^2)), so <|M|> = sqrt(2/pi) * sd;
* 2 x 2 lattice at any coupling: the four sites form one cycle of bonds, each
  counted twice by Eq. (1), so Z is the trace of a product of four transfer
  matrices; on a uniform grid this is the 4D trapezoidal rule, which converges
  exponentially for this analytic, rapidly decaying integrand;
* 1 x 1 lattice: the kinetic term vanishes; one-dimensional adaptive
  quadrature (scipy).
"""

import math

import numpy as np


def free_eigs(L):
    k = np.arange(L)
    lk = 4.0 * np.sin(np.pi * k / L) ** 2
    return (lk[:, None] + lk[None, :]).ravel()


def free_logz(L, m2, s2=1.0):
    return float(-0.5 * np.sum(np.log(1.0 + s2 * (m2 + free_eigs(L)))))


def free_mean_abs_m(L, m2, s2=1.0):
    var = s2 / (L * L * (1.0 + s2 * m2))
    return math.sqrt(2.0 / math.pi) * math.sqrt(var)


def logz_2x2(m2, lam, s2=1.0, h=0.02, xmax=4.0):
    x = np.arange(-xmax, xmax + h / 2, h)
    on_site = 0.5 * x ** 2 / s2 + 0.5 * m2 * x ** 2 + lam * x ** 4
    D = h * np.exp(-on_site) / math.sqrt(2.0 * math.pi * s2)
    K = np.exp(-((x[:, None] - x[None, :]) ** 2))   # bond counted twice: 2 * 1/2
    T = D[:, None] * K
    return math.log(float(np.trace(np.linalg.matrix_power(T, 4))))


def logz_1x1(m2, lam, s2=1.0):
    from scipy.integrate import quad

    def f(x):
        return math.exp(-0.5 * x * x / s2 - 0.5 * m2 * x * x - lam * x ** 4) \
            / math.sqrt(2.0 * math.pi * s2)

    val, _ = quad(f, -math.inf, math.inf, epsabs=0, epsrel=1e-13, limit=200)
    return math.log(val)
