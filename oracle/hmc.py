"""Adaptive tempered SMC with a Hamiltonian Monte Carlo inner kernel
(SMC-HMC) -- the FP64 oracle (test infrastructure only).

What the paper states (Sec. 2 "Particle-based Monte Carlo methods" (iii);
App. A): the random-walk rejuvenation of the tempered SMC is replaced by
short HMC trajectories of a fixed 20 leapfrog steps with a diagonal mass
matrix; the inner kernels are based on Gaussian statistics of the particle
population at each outer step, and fewer MCMC steps per level are taken
than for the random walk.

Readings where the paper is silent (also listed in the design notes):

* Potential of the tempered target p_beta ~ exp(-[U0 + beta S]):
  V = U0 + beta S, gradient phi + beta dS/dphi with, from Sec. 2 Eq. (1),
  dS/dphi_x = sum_mu (2 phi_x - phi_{x+mu} - phi_{x-mu}) + m^2 phi_x
  + 4 lambda phi_x^3 (periodic neighbours).
* Mass matrix: M = diag(1 / v_x) with v_x the variance of site x over the
  resampled particles (the diagonal of the same covariance, divisor N - 1,
  as SMC-RW), fixed within a level.  Momentum p = z / sqrt(v) with z from
  the PROPOSE stream, kinetic energy K = sum_x v_x p_x^2 / 2.
* Leapfrog: p -= eps/2 grad V; then n_leap times phi += eps v p and
  p -= eps grad V, the last momentum update being a half step.
* Step size: eps0 = d^(-1/4) unless given; after each level
  log eps += (acceptance - target), clamped to [eps0/100, 10 eps0] (the
  random-walk rule); eps is fixed within a level.
* Accept iff log u < -(H(phi', p') - H(phi, p)) (strict; NaN rejects), u
  from the ACCEPT stream, H = V + K, the potential difference summed per
  site.

Everything else (reweighting, beta solve, resampling, streams) is the
SMC-RW oracle's.

Pins (tests/test_oracle_hmc.py): the gradient against central differences
of the action and the closed form of constant fields; leapfrog
reversibility (momentum flip returns to the start) and its second-order
energy error; stationarity of an exact Gaussian target; the full sampler
against the free-theory log Z and 2 x 2 quadrature.
"""

import numpy as np

from . import rng
from .action import action, magnetisation, u0
from .smc import adapt_eps, ess, init_particles, reweight, systematic_resample


def grad_action(phi, L, m2, lam):
    """dS/dphi per site, Sec. 2 Eq. (1); phi has shape (N, L*L)."""
    phi = np.asarray(phi, dtype=np.float64)
    n = phi.shape[0]
    f = phi.reshape(n, L, L)
    g = m2 * f + 4.0 * lam * f ** 3
    for axis in (1, 2):
        g = g + 2.0 * f - np.roll(f, -1, axis=axis) - np.roll(f, 1, axis=axis)
    return g.reshape(n, L * L)


def grad_potential(phi, beta, L, m2, lam):
    """grad (U0 + beta S)."""
    return np.asarray(phi, dtype=np.float64) + beta * grad_action(phi, L, m2, lam)


def leapfrog(phi, p, v, eps, n_leap, beta, L, m2, lam):
    """n_leap leapfrog steps of H = V + sum v p^2 / 2; returns (phi, p)."""
    phi = np.asarray(phi, dtype=np.float64)
    p = p - 0.5 * eps * grad_potential(phi, beta, L, m2, lam)
    for step in range(n_leap):
        phi = phi + eps * v * p
        g = grad_potential(phi, beta, L, m2, lam)
        p = p - (eps if step < n_leap - 1 else 0.5 * eps) * g
    return phi, p


def hamiltonian_change(phi, p, phi1, p1, v, beta, L, m2, lam):
    """H(phi1, p1) - H(phi, p)."""
    dV = (u0(phi1) - u0(phi)) + beta * (action(phi1, L, m2, lam) - action(phi, L, m2, lam))
    dK = 0.5 * np.sum(v * (p1 * p1 - p * p), axis=1)
    return dV + dK


def hmc_step(phi, S, v, eps, n_leap, beta, L, m2, lam, seed, run, level, step):
    """One HMC step per particle; returns (phi, S, accepted mask)."""
    phi = np.asarray(phi, dtype=np.float64)
    n, d = phi.shape
    rows = np.arange(n)
    z = rng.normals(seed, run, level, step, rng.PROPOSE, rows, d)
    p = z / np.sqrt(v)
    # a diverging trajectory (step too large for the quartic term) ends with a
    # non-finite H, which compares false and so rejects
    with np.errstate(over="ignore", invalid="ignore"):
        phi1, p1 = leapfrog(phi, p, v, eps, n_leap, beta, L, m2, lam)
        dH = hamiltonian_change(phi, p, phi1, p1, v, beta, L, m2, lam)
    lu = np.log(rng.accept_uniforms(seed, run, level, step, rows))
    acc = lu < -dH
    phi = np.where(acc[:, None], phi1, phi)
    with np.errstate(over="ignore", invalid="ignore"):
        S = np.where(acc, action(phi1, L, m2, lam), S)
    return phi, S, acc


def default_eps0(d):
    """eps0 = d^(-1/4), the dimension scaling of HMC step sizes."""
    return d ** -0.25


def smc_run(L, m2, lam, N, ess_frac=0.5, n_steps=5, seed=0, run=0, n_leap=20,
            acc_target=0.65, eps0=None, max_levels=100000, keep_particles=False,
            stop_after=None):
    """Adaptive tempered SMC-HMC from beta = 0 to beta = 1 (or, with
    `stop_after`, the state after that many levels)."""
    d = L * L
    eps0 = default_eps0(d) if eps0 is None or eps0 <= 0 else eps0
    eps = eps0
    phi = init_particles(seed, run, N, d)
    S = action(phi, L, m2, lam)
    beta = 0.0
    logz = 0.0
    levels = []
    level = 0
    while beta < 1.0 and (stop_after is None or level < stop_after):
        level += 1
        if level > max_levels:
            raise RuntimeError("too many tempering levels")
        dbeta, new_beta, dlogz, w = reweight(S, beta, ess_frac)
        ess_val = ess(-dbeta * S)
        logz += dlogz
        anc = systematic_resample(w, rng.resample_word(seed, run, level))
        phi = phi[anc]
        S = S[anc]
        v = phi.var(axis=0, ddof=1)   # the covariance's diagonal, divisor N - 1
        beta = new_beta
        n_acc = 0
        for s in range(n_steps):
            phi, S, acc = hmc_step(phi, S, v, eps, n_leap, beta, L, m2, lam, seed, run,
                                   level, s)
            n_acc += int(acc.sum())
        levels.append(dict(beta=beta, dbeta=dbeta, ess=ess_val, dlogz=dlogz, eps=eps,
                           acc=n_acc / (N * n_steps) if n_steps else 0.0))
        eps = adapt_eps(eps, n_acc, N * n_steps, eps0, acc_target)
    out = dict(logz=logz, mean_abs_m=float(np.mean(np.abs(magnetisation(phi)))),
               n_levels=level, levels=levels, eps=eps)
    if keep_particles:
        out["phi"] = phi
        out["S"] = S
    return out

