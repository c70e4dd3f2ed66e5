"""Seeded synthetic inputs shared by the oracle tests and the GPU parity tests.

Holds no arithmetic of the sampler: only reproducible random arrays with the
shapes and value ranges of the workloads (particle fields of a 2D lattice,
importance weights, covariance-like matrices).
"""

import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def fields(seed, n, L, scale=1.0, dtype=np.float32):
    """n lattice fields of d = L*L sites, N(0, scale^2), as float32 rows."""
    return (scale * rng(seed).standard_normal((n, L * L))).astype(dtype)


def broken_phase_fields(seed, n, L, v=0.35, noise=0.3, dtype=np.float32):
    """Fields fluctuating around +-v (both signs), like a double-well population."""
    g = rng(seed)
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)[:, None]
    return (sign * v + noise * g.standard_normal((n, L * L))).astype(dtype)


def log_weights(seed, n, spread=3.0):
    """float64 log-weights with a heavy spread, like -dbeta * S."""
    return spread * rng(seed).standard_normal(n)


def spd_matrix(seed, d, cond=10.0):
    """A symmetric positive-definite d x d float64 matrix of given condition."""
    g = rng(seed)
    q, _ = np.linalg.qr(g.standard_normal((d, d)))
    ev = np.geomspace(1.0, 1.0 / cond, d)
    return (q * ev) @ q.T


def lower_factor(seed, d, scale=1.0):
    """A lower-triangular factor with a positive diagonal (float64)."""
    g = rng(seed)
    Lm = np.tril(g.standard_normal((d, d))) * (scale / np.sqrt(d))
    Lm[np.diag_indices(d)] = scale * (0.5 + g.random(d))
    return Lm
