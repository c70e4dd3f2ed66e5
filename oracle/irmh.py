"""Adaptive tempered SMC with an independent Metropolis-Hastings rejuvenation
(SMC-IRMH) -- the FP64 oracle (test infrastructure only).

What the paper states (Sec. 2 "Particle-based Monte Carlo methods" (ii);
App. A): the outer loop is the same adaptive tempered SMC as SMC-RW; the
inner kernel is a Metropolis-Hastings sampler whose proposal does not depend
on the current particle and is a Gaussian fitted to the particle population
at each outer step (its covariance is the particle covariance, like every
inner kernel of App. A), close to a plain annealed importance sampler.

Readings where the paper is silent (also listed in the design notes):

* Proposal: q = N(mu, L L^T), mu the mean and L the jittered Cholesky factor
  of the covariance of the resampled particles (the same covariance, divisor
  and jitter as SMC-RW); no 2.38^2 / V scaling, which App. A attaches to the
  random-walk proposal only, and no step-size adaptation.
* A proposal is phi' = mu + L z with z from the PROPOSE stream, so that
  log q(phi') = -|z|^2 / 2 + const; the current particle enters through its
  whitened residual r = |L^{-1}(phi - mu)|^2, computed once per level after
  the factor and replaced by |z|^2 when a proposal is accepted.
* Acceptance: log alpha = log p_beta(phi') - log p_beta(phi)
  + log q(phi) - log q(phi') = -dU0 - beta dS + (|z|^2 - r) / 2, strict
  test log u < log alpha with u from the ACCEPT stream (NaN rejects).

Everything else (reweighting, beta solve, resampling, covariance and
jitter, streams) is the SMC-RW oracle's.

Pins (tests/test_oracle_irmh.py): with the exact Gaussian target of the free
theory as proposal, log alpha vanishes for every pair of fields (closed
form); the whitened residual equals the Mahalanobis form through the
explicit inverse covariance; a mis-specified proposal leaves the exact
Gaussian target invariant (mean and variance after many steps); the full
sampler reproduces the free-theory log Z from the Laplacian determinant.
"""

import numpy as np

from . import rng
from .action import action, magnetisation, u0
from .smc import (cholesky_jitter, covariance, ess, init_particles, reweight,
                  systematic_resample)


def particle_mean(phi):
    """Mean field over the particles (float64)."""
    return np.asarray(phi, dtype=np.float64).mean(axis=0)


def whitened_sq(phi, mu, chol):
    """r_i = |L^{-1}(phi_i - mu)|^2 by forward substitution."""
    x = (np.asarray(phi, dtype=np.float64) - mu).T          # d x N
    d = chol.shape[0]
    w = np.empty_like(x)
    for i in range(d):                                      # L w = x, row by row
        w[i] = (x[i] - chol[i, :i] @ w[:i]) / chol[i, i]
    return np.sum(w * w, axis=0)


def propose(mu, chol, seed, run, level, step, rows):
    """phi' = mu + L z per particle; returns (phi', |z|^2)."""
    d = mu.shape[0]
    z = rng.normals(seed, run, level, step, rng.PROPOSE, rows, d)
    return mu + z @ chol.T, np.sum(z * z, axis=1)


def log_alpha(phi, prop, r_cur, zz, beta, L, m2, lam):
    """log alpha = -dU0 - beta dS + (|z|^2 - r) / 2 (independence sampler)."""
    dS = action(prop, L, m2, lam) - action(phi, L, m2, lam)
    dU = u0(prop) - u0(phi)
    return -dU - beta * dS + 0.5 * (np.asarray(zz) - np.asarray(r_cur))


def irmh_step(phi, S, r, mu, chol, beta, L, m2, lam, seed, run, level, step):
    """One independence-sampler step; returns (phi, S, r, accepted mask)."""
    phi = np.asarray(phi, dtype=np.float64)
    n = phi.shape[0]
    rows = np.arange(n)
    prop, zz = propose(mu, chol, seed, run, level, step, rows)
    la = log_alpha(phi, prop, r, zz, beta, L, m2, lam)
    lu = np.log(rng.accept_uniforms(seed, run, level, step, rows))
    acc = lu < la
    phi = np.where(acc[:, None], prop, phi)
    S = np.where(acc, action(prop, L, m2, lam), S)
    r = np.where(acc, zz, r)
    return phi, S, r, acc


def smc_run(L, m2, lam, N, ess_frac=0.5, n_steps=10, seed=0, run=0,
            max_levels=100000, keep_particles=False):
    """Adaptive tempered SMC-IRMH from beta = 0 to beta = 1.

    Same outer loop and streams as the SMC-RW oracle; returns a dict with
    log Z, <|M|>, the per-level record and (optionally) the particles.
    """
    d = L * L
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
        mu = particle_mean(phi)
        r = whitened_sq(phi, mu, chol)
        beta = new_beta
        n_acc = 0
        for s in range(n_steps):
            phi, S, r, acc = irmh_step(phi, S, r, mu, chol, beta, L, m2, lam,
                                       seed, run, level, s)
            n_acc += int(acc.sum())
        levels.append(dict(beta=beta, dbeta=dbeta, ess=ess_val, dlogz=dlogz,
                           acc=n_acc / (N * n_steps) if n_steps else 0.0))
    out = dict(logz=logz, mean_abs_m=float(np.mean(np.abs(magnetisation(phi)))),
               n_levels=level, levels=levels)
    if keep_particles:
        out["phi"] = phi
        out["S"] = S
    return out
