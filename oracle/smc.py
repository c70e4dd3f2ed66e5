"""Adaptive tempered SMC with covariance-preconditioned random-walk Metropolis
(SMC-RW) -- the FP64 oracle (test infrastructure only).

What the paper states (Sec. 2 "Particle-based Monte Carlo methods" (i); App. A):
particles are moved along the tempered family p_beta ~ exp(-[U0 + beta S])
(Sec. 2), beta goes from 0 to 1 adaptively so that each step keeps a target
effective sample size, particles are resampled, and each tempering transition
is followed by a fixed number of Gaussian random-walk Metropolis steps whose
proposal covariance is the particle covariance scaled by 2.38^2 / V (App. A).
The estimate of the normalising constant accumulates the mean incremental
weight of every tempering step.

Where the paper is silent the oracle takes these readings (each one is also
listed with its justification in the design notes of the repository):

* log Z is log E_{phi ~ N(0, I)}[exp(-S(phi))]: the tempered family always
  carries U0, and the estimator sums log mean_i exp(-dbeta S_i).
* Next beta: if ESS(1 - beta) >= alpha N take beta' = 1; otherwise bisect
  dbeta on [0, 1 - beta] for exactly 64 float64 iterations and keep the lower
  end, so ESS(dbeta) >= alpha N.  ESS(l) = exp(2 LSE(l) - LSE(2 l)).
* Order within a level: reweight -> log Z -> systematic resampling ->
  covariance and Cholesky -> n_s Metropolis steps at the new beta -> step-size
  adaptation; the level that reaches beta = 1 is also mutated.
* Systematic resampling on an integer CDF (bit-exact regardless of summation
  order): q_i = floor(2^k w_i / max_j w_j) with k = 62 - 2 ceil(log2 N),
  C = cumsum(q), Q = C[-1], T_i = floor((i Q + U Q / 2^32) / N) evaluated in
  exact integers, ancestor a_i = min{ j : C_j > T_i }.  This is textbook
  systematic resampling with offset u = U / 2^32 applied to the weights
  quantised at 2^-k of the largest.
* Covariance: unweighted, over the resampled particles, divisor N - 1; jitter
  tau = 1e-10 tr(Sigma) / d added to the diagonal, multiplied by 100 after each
  failed factorisation, at most five retries.
* Step size: eps0 = 2.38 / sqrt(d) (App. A); after each level
  log eps += (acceptance - target), clamped to [eps0 / 100, 10 eps0]; eps is
  fixed within a level.  Proposal: phi' = phi + eps * L z, z ~ N(0, I).
* Accept iff log u < log alpha (strict), with
  log alpha = -(U0(phi') - U0(phi)) - beta (S(phi') - S(phi)); NaN rejects.

Parity status: every function here is pinned by tests/test_oracle_smc.py and
tests/test_oracle_stats.py (closed forms, brute force on tiny inputs, library
routines, free-theory log Z from the lattice-Laplacian determinant and
Gauss-Hermite quadrature on a 2x2 lattice).  The full sampler at the
interacting couplings is pinned only statistically ("parity unpinned" beyond
that; see the design notes).
"""

import math

import numpy as np

from . import rng
from .action import action, magnetisation, u0
from .precision import round_operand


class CholeskyError(RuntimeError):
    """The jittered covariance could not be factorised."""


class DegenerateWeights(RuntimeError):
    """The beta solve made no progress (non-finite or degenerate weights)."""


# ---------------------------------------------------------------- reweighting

def lse(a):
    """log sum exp, float64."""
    a = np.asarray(a, dtype=np.float64)
    m = np.max(a)
    if not np.isfinite(m):
        return m
    return m + math.log(np.sum(np.exp(a - m)))


def ess(ell):
    """Effective sample size of log-weights ell: (sum w)^2 / sum w^2."""
    ell = np.asarray(ell, dtype=np.float64)
    return math.exp(2.0 * lse(ell) - lse(2.0 * ell))


def solve_dbeta(S, beta, target_ess):
    """Tempering increment that keeps ESS >= target_ess (64-step bisection)."""
    S = np.asarray(S, dtype=np.float64)
    room = 1.0 - beta
    if ess(-room * S) >= target_ess:
        return room
    lo, hi = 0.0, room
    for _ in range(64):
        mid = 0.5 * (lo + hi)
        if ess(-mid * S) >= target_ess:
            lo = mid
        else:
            hi = mid
    return lo


def reweight(S, beta, ess_frac):
    """One reweighting: returns (dbeta, new beta, log Z increment, weights).

    The weights are w_i = exp(l_i - max l) with l_i = -dbeta S_i.
    """
    S = np.asarray(S, dtype=np.float64)
    n = S.shape[0]
    dbeta = solve_dbeta(S, beta, ess_frac * n)
    if not dbeta > 0.0:
        raise DegenerateWeights("tempering increment is zero")
    new_beta = 1.0 if dbeta == 1.0 - beta else min(1.0, beta + dbeta)
    ell = -dbeta * S
    dlogz = lse(ell) - math.log(n)
    w = np.exp(ell - np.max(ell))
    return dbeta, new_beta, dlogz, w


# ----------------------------------------------------------------- resampling

def resample_bits(n):
    """k = 62 - 2 ceil(log2 N): quantisation bits of the integer CDF."""
    return 62 - 2 * (int(n) - 1).bit_length() if n > 1 else 62


def systematic_resample(w, U):
    """Ancestor indices of systematic resampling on the integer CDF."""
    w = np.asarray(w, dtype=np.float64)
    n = w.shape[0]
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    if not np.all(np.isfinite(w)) or np.any(w < 0) or not np.max(w) > 0:
        raise DegenerateWeights("weights must be finite, >= 0, not all zero")
    k = resample_bits(n)
    q = [int(math.floor(math.ldexp(float(x), k))) for x in (w / np.max(w))]
    C = []
    acc = 0
    for x in q:                       # exact integer prefix sum
        acc += x
        C.append(acc)
    Q = C[-1]
    U = int(U) & 0xFFFFFFFF
    anc = np.empty(n, dtype=np.int64)
    for i in range(n):
        T = (i * Q + U * (Q >> 32) + ((U * (Q & 0xFFFFFFFF)) >> 32)) // n
        anc[i] = _first_greater(C, T)
    return anc


def _first_greater(C, T):
    """min{ j : C[j] > T } by bisection over Python ints."""
    lo, hi = 0, len(C) - 1
    while lo < hi:
        mid = (lo + hi) // 2
        if C[mid] > T:
            hi = mid
        else:
            lo = mid + 1
    return lo


# ------------------------------------------------------- covariance and factor

def covariance(phi):
    """Unweighted particle covariance with divisor N - 1."""
    phi = np.asarray(phi, dtype=np.float64)
    n = phi.shape[0]
    if n < 2:
        raise ValueError("covariance needs at least two particles")
    c = phi - phi.mean(axis=0)
    return (c.T @ c) / (n - 1)


def cholesky_jitter(sigma, max_retries=5):
    """Lower Cholesky factor of sigma + tau I with the escalating jitter."""
    sigma = np.asarray(sigma, dtype=np.float64)
    d = sigma.shape[0]
    tau = 1e-10 * np.trace(sigma) / d
    eye = np.eye(d)
    for _ in range(max_retries + 1):
        try:
            return np.linalg.cholesky(sigma + tau * eye), tau
        except np.linalg.LinAlgError:
            tau *= 100.0
    raise CholeskyError("covariance not positive definite after jitter")


# ------------------------------------------------------------------ mutation

def propose(phi, B, seed, run, level, step, rows, precision="fp64", zsign=1.0):
    """phi' = phi + B z per particle (row form z B^T), z from the PROPOSE stream.

    ``B`` is the scaled factor eps * L; ``precision`` selects the rounding of
    z and B before the float64 product (see oracle.precision).
    """
    phi = np.asarray(phi, dtype=np.float64)
    d = phi.shape[1]
    z = zsign * rng.normals(seed, run, level, step, rng.PROPOSE, rows, d)
    zr = round_operand(z, precision)
    Br = round_operand(B, precision)
    return phi + zr @ Br.T


def tempered_log_alpha(phi, prop, beta, L, m2, lam):
    """log alpha = -dU0 - beta dS for p_beta ~ exp(-[U0 + beta S])."""
    dS = action(prop, L, m2, lam) - action(phi, L, m2, lam)
    dU = u0(prop) - u0(phi)
    return -dU - beta * dS


def accept(log_u, log_alpha):
    """Strict Metropolis test; NaN compares false and so rejects."""
    return np.asarray(log_u) < np.asarray(log_alpha)


def rwmh_step(phi, S, B, beta, L, m2, lam, seed, run, level, step,
              rows=None, precision="fp64"):
    """One random-walk Metropolis step at inverse temperature beta.

    Returns (new phi, new S, accepted mask).
    """
    phi = np.asarray(phi, dtype=np.float64)
    n = phi.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    prop = propose(phi, B, seed, run, level, step, rows, precision)
    log_alpha = tempered_log_alpha(phi, prop, beta, L, m2, lam)
    log_u = np.log(rng.accept_uniforms(seed, run, level, step, rows))
    acc = accept(log_u, log_alpha)
    new_phi = np.where(acc[:, None], prop, phi)
    new_S = np.where(acc, action(prop, L, m2, lam), S)
    return new_phi, new_S, acc


def adapt_eps(eps, n_acc, n_prop, eps0, acc_target):
    """log eps += (acceptance - target), clamped to [eps0/100, 10 eps0]."""
    abar = n_acc / n_prop if n_prop > 0 else acc_target
    new = eps * math.exp(abar - acc_target)
    return min(max(new, eps0 / 100.0), 10.0 * eps0)


# --------------------------------------------------------------- the sampler

def default_eps0(d):
    """eps0 = 2.38 / sqrt(d): the Roberts-Gelman-Gilks scaling of App. A."""
    return 2.38 / math.sqrt(d)


def init_particles(seed, run, n, d, scale=1.0):
    """phi_i ~ N(0, scale^2 I) from the INIT stream."""
    return scale * rng.normals(seed, run, 0, 0, rng.INIT, np.arange(n), d)


def smc_run(L, m2, lam, N, ess_frac=0.5, n_steps=10, seed=0, run=0,
            acc_target=0.3, eps0=None, precision="fp64", max_levels=100000,
            keep_particles=False):
    """Adaptive tempered SMC-RW from beta = 0 to beta = 1.

    Returns a dict with log Z, <|M|>, the per-level record and the final
    particles (if ``keep_particles``).
    """
    d = L * L
    eps0 = default_eps0(d) if eps0 is None or eps0 <= 0 else eps0
    eps = eps0
    phi = init_particles(seed, run, N, d)
    S = action(phi, L, m2, lam)
    beta = 0.0
    logz = 0.0
    levels = []
    level = 0
    while beta < 1.0:
        level += 1
        if level > max_levels:
            raise RuntimeError("too many tempering levels")
        dbeta, new_beta, dlogz, w = reweight(S, beta, ess_frac)
        ess_val = ess(-dbeta * S)
        logz += dlogz
        anc = systematic_resample(w, rng.resample_word(seed, run, level))
        phi = phi[anc]
        S = S[anc]
        chol, _ = cholesky_jitter(covariance(phi))
        B = eps * chol
        beta = new_beta
        n_acc = 0
        for s in range(n_steps):
            phi, S, acc = rwmh_step(phi, S, B, beta, L, m2, lam, seed, run,
                                    level, s, precision=precision)
            n_acc += int(acc.sum())
        levels.append(dict(beta=beta, dbeta=dbeta, ess=ess_val, dlogz=dlogz,
                           eps=eps, acc=n_acc / (N * n_steps) if n_steps else 0.0))
        eps = adapt_eps(eps, n_acc, N * n_steps, eps0, acc_target)
    out = dict(logz=logz, mean_abs_m=float(np.mean(np.abs(magnetisation(phi)))),
               n_levels=level, levels=levels, eps=eps)
    if keep_particles:
        out["phi"] = phi
        out["S"] = S
    return out
