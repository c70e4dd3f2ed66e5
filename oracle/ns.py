"""Nested sampling with likelihood-constrained random-walk refill -- the FP64
oracle (test infrastructure only).

What the paper states (Sec. 2 "Particle-based Monte Carlo methods" (iv);
App. A): nested sampling keeps a population of live points, deletes a fraction
of them per iteration (0.5 in the paper's settings), and refills the deleted
slots with MCMC moves that must satisfy the current likelihood constraint; the
inner kernel is tuned by the particle covariance.  The paper's own refill is
slice sampling; here the refill is a likelihood-constrained Gaussian random
walk with the same covariance preconditioning (the paper's random-walk kernel
of App. A under the NS constraint).

Readings taken where the paper is silent:

* prior N(0, prior_var I) (prior_var = 4 in the d = 1024 workload),
  likelihood exp(-S), so log L = -S and the evidence is
  Z = E_{phi ~ N(0, prior_var I)}[exp(-S(phi))];
* deletion order: ascending (log L, row index); the j-th deleted point of an
  iteration (j = 0..k-1) gets log X_j = log X - sum_{m=0}^{j} 1/(n - m)
  (expected log shrinkage of the order statistics of n uniforms) and weight
  w_j = L_j (X_{j-1} - X_j), with X_{-1} the volume before the iteration;
* the constraint for new points is strict: S(phi') < S*, with S* the action of
  the last deleted point; the prior enters the Metropolis ratio as
  log alpha = -(|phi'|^2 - |phi|^2) / (2 prior_var);
* seeds: new point j copies survivor number floor(U_j (n - k) / 2^32) of the
  survivors listed in deletion order (ascending log L, then index), U_j a
  NS_PICK word; the covariance is taken over the survivors;
* termination, tested before each iteration: stop when
  log X + LSE(log L_live) - log n - log Z < log(term_frac); the final live
  points then each add weight X / n * L_i;
* error bar sqrt(H / n) with H the information of the posterior.

Parity status: pinned by tests/test_oracle_ns.py against the closed-form
free-theory evidence -1/2 sum_k log(1 + prior_var (m^2 + lambda_k)) and the
exact prior-volume sequence; at interacting couplings "parity unpinned" beyond
the statistical comparison (see the design notes).
"""

import math

import numpy as np

from . import rng
from .action import action, magnetisation, u0
from .precision import round_operand
from .smc import adapt_eps, cholesky_jitter, covariance, default_eps0, lse


def deletion_order(logL):
    """Row indices sorted by ascending log L, ties by ascending index."""
    logL = np.asarray(logL)
    return np.lexsort((np.arange(logL.shape[0]), logL))


def shrink_sequence(logX, n, k):
    """log X_j for the k deletions of one iteration (float64)."""
    out = np.empty(k)
    x = logX
    for j in range(k):
        x = x - 1.0 / (n - j)
        out[j] = x
    return out


def constrained_step(phi, B, S_star, prior_var, L, m2, lam, seed, run, it, step,
                     rows, precision="fp64"):
    """One likelihood-constrained random-walk Metropolis step of the rows given.

    Returns (new phi rows, new S rows, accepted mask).
    """
    phi = np.asarray(phi, dtype=np.float64)
    d = phi.shape[1]
    z = rng.normals(seed, run, it, step, rng.PROPOSE, rows, d)
    prop = phi + round_operand(z, precision) @ round_operand(B, precision).T
    S_prop = action(prop, L, m2, lam)
    log_alpha = -(u0(prop) - u0(phi)) / prior_var
    log_u = np.log(rng.accept_uniforms(seed, run, it, step, rows))
    acc = (S_prop < S_star) & (log_u < log_alpha)
    new_phi = np.where(acc[:, None], prop, phi)
    return new_phi, acc, S_prop


def ns_run(L, m2, lam, n_live, k_delete, n_steps, prior_var=4.0, term_frac=1e-3,
           seed=0, run=0, eps0=None, acc_target=0.3, precision="fp64",
           max_iter=1000000):
    """Nested sampling run; returns log Z, its error bar, <|M|> and counters."""
    d = L * L
    n, k = n_live, k_delete
    if not 0 < k < n:
        raise ValueError("need 0 < k_delete < n_live")
    eps0 = default_eps0(d) if eps0 is None or eps0 <= 0 else eps0
    eps = eps0
    phi = math.sqrt(prior_var) * rng.normals(seed, run, 0, 0, rng.INIT,
                                             np.arange(n), d)
    S = action(phi, L, m2, lam)
    logX = 0.0
    logZ = -math.inf
    dead_logw, dead_logL, dead_absm = [], [], []
    it = 0
    accs = []
    while True:
        logL = -S
        if logZ > -math.inf and \
                logX + lse(logL) - math.log(n) - logZ < math.log(term_frac):
            break
        it += 1
        if it > max_iter:
            raise RuntimeError("nested sampling did not terminate")
        order = deletion_order(logL)
        dead, surv = order[:k], order[k:]
        xs = shrink_sequence(logX, n, k)
        prev = np.concatenate([[logX], xs[:-1]])
        # log(X_{j-1} - X_j) = log X_{j-1} + log(1 - exp(log X_j - log X_{j-1}))
        logw = logL[dead] + prev + np.log(-np.expm1(xs - prev))
        absm = np.abs(magnetisation(phi[dead]))
        dead_logw.extend(logw)
        dead_logL.extend(logL[dead])
        dead_absm.extend(absm)
        for lw in logw:
            logZ = np.logaddexp(logZ, lw)
        logX = xs[-1]
        S_star = S[dead[-1]]
        picks = (rng.words(seed, run, it, 0, rng.NS_PICK, np.arange(k))
                 .astype(np.uint64) * np.uint64(n - k)) >> np.uint64(32)
        src = surv[picks.astype(np.int64)]
        phi[dead] = phi[src]
        S[dead] = S[src]
        chol, _ = cholesky_jitter(covariance(phi[surv]))
        B = eps * chol
        n_acc = 0
        for s in range(n_steps):
            new_rows, acc, S_prop = constrained_step(
                phi[dead], B, S_star, prior_var, L, m2, lam, seed, run, it, s,
                dead, precision)
            phi[dead] = new_rows
            S[dead] = np.where(acc, S_prop, S[dead])
            n_acc += int(acc.sum())
        accs.append(n_acc / (k * n_steps) if n_steps else 0.0)
        eps = adapt_eps(eps, n_acc, k * n_steps, eps0, acc_target)
    # final live points
    logL = -S
    live_logw = logX - math.log(n) + logL
    all_logw = np.concatenate([np.asarray(dead_logw), live_logw])
    all_logL = np.concatenate([np.asarray(dead_logL), logL])
    all_absm = np.concatenate([np.asarray(dead_absm),
                               np.abs(magnetisation(phi))])
    logZ = lse(all_logw)
    p = np.exp(all_logw - logZ)
    H = float(np.sum(p * all_logL) - logZ)
    mean_abs_m = float(np.sum(p * all_absm))
    return dict(logz=logZ, logz_err=math.sqrt(max(H, 0.0) / n), H=H,
                mean_abs_m=mean_abs_m, n_iter=it, logX=logX, acc=accs,
                eps=eps)
