"""Nested sampling with likelihood-constrained random-walk refill -- the FP64
oracle (test infrastructure only).

What the paper states (Sec. 2 "Particle-based Monte Carlo methods" (iv);
App. A): nested sampling keeps a population of live points, deletes a fraction
of them per iteration (0.5 in the paper's settings), and refills the deleted
slots with MCMC moves that must satisfy the current likelihood constraint; the
inner kernel is tuned by the particle covariance.  The paper's own refill is
slice sampling (``refill="slice"``: hit-and-run slice moves along directions
from the survivors' covariance, Neal's stepping-out and shrinkage); the
default refill is a likelihood-constrained Gaussian random walk with the same
covariance preconditioning (the paper's random-walk kernel of App. A under the
NS constraint).

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
exact prior-volume sequence; the slice refill by tests/test_oracle_ns_slice.py
(invariance of the prior and of the truncated-normal constrained prior at
L = 1, also with brackets ten times the slice, the constraint on a lattice,
free-theory and 2 x 2 quadrature evidences); at interacting couplings "parity unpinned" beyond
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


# Slice-sampling refill (Sec. 2 (iv); App. A: the paper's own NS kernel):
# hit-and-run slice sampling of the prior restricted to the likelihood
# constraint, along a direction drawn from the survivors' covariance, with
# Neal's stepping-out (limit m) and shrinkage procedures (Neal, "Slice
# sampling", Ann. Statist. 2003).
SLICE_WIDTH = 1.0       # w, in units of the direction L z
SLICE_MAX_STEPS = 32    # m: at most m - 1 expansions in total
SLICE_MAX_SHRINK = 64   # shrinkage draws; if all miss, the point stays


def slice_move(phi, u, S_cur, S_star, prior_var, L, m2, lam, uniforms):
    """One slice move of the field phi (1-D) along direction u.

    The slice of t -> N(phi + t u; 0, prior_var I) restricted to
    S(phi + t u) < S_star at the level log y = log prior(phi) + log U0;
    uniforms(j) is the j-th uniform of the move (U0, then the initial offset,
    the step-out split, then one per shrinkage draw).  Returns (phi', S')."""
    phi = np.asarray(phi, dtype=np.float64)
    log_y = -0.5 * float(phi @ phi) / prior_var + math.log(uniforms(0))

    def inside(t):
        x = phi + t * u
        if not -0.5 * float(x @ x) / prior_var > log_y:
            return False, None
        s = float(action(x[None, :], L, m2, lam)[0])
        return s < S_star, s

    w = SLICE_WIDTH
    lo = -w * uniforms(1)
    hi = lo + w
    J = int(math.floor(SLICE_MAX_STEPS * uniforms(2)))
    K = SLICE_MAX_STEPS - 1 - J
    while J > 0 and inside(lo)[0]:
        lo -= w
        J -= 1
    while K > 0 and inside(hi)[0]:
        hi += w
        K -= 1
    for i in range(SLICE_MAX_SHRINK):
        t = lo + uniforms(3 + i) * (hi - lo)
        ok, s = inside(t)
        if ok:
            return phi + t * u, s
        if t < 0.0:
            lo = t
        else:
            hi = t
    return phi, S_cur


def ns_run(L, m2, lam, n_live, k_delete, n_steps, prior_var=4.0, term_frac=1e-3,
           seed=0, run=0, eps0=None, acc_target=0.3, precision="fp64",
           max_iter=1000000, refill="rw"):
    """Nested sampling run; returns log Z, its error bar, <|M|> and counters.

    refill "rw": likelihood-constrained random walk (eps adapted per
    iteration); "slice": n_steps slice moves per refilled point along
    directions L z, L the factor of the survivors' covariance (no eps)."""
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
        if refill == "slice":
            n_moved = 0
            for s in range(n_steps):
                U = rng.normals(seed, run, it, s, rng.PROPOSE, dead, d) @ chol.T
                for j, row in enumerate(dead):
                    def uniforms(q, row=row, s=s):
                        return rng.slice_uniform(seed, run, it, s, int(row), q)
                    new, s_new = slice_move(phi[row], U[j], S[row], S_star, prior_var, L,
                                            m2, lam, uniforms)
                    n_moved += int(not np.array_equal(new, phi[row]))
                    phi[row] = new
                    S[row] = s_new
            accs.append(n_moved / (k * n_steps) if n_steps else 0.0)
            continue
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
