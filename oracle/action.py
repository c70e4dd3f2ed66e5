"""The lattice phi^4 action and observables (test infrastructure only).

Follows Sec. 2, Eq. (1): on the periodic D = 2 lattice {0..L-1}^2 with a = 1,

    S(phi) = sum_x [ 1/2 sum_mu (phi_{x+mu} - phi_x)^2 + 1/2 m^2 phi_x^2
                     + lambda phi_x^4 ],

the magnetisation M = (1/V) sum_x phi_x (Sec. 2) and the Gaussian reference
U0 = 1/2 sum_x phi_x^2 of the tempered family p_beta ~ exp(-[U0 + beta S])
(Sec. 2, "To incorporate annealing or tempering").

Layout convention (shared with the GPU path): a particle is a row of d = L^2
values; site (x0, x1) sits at x0 * L + x1, so the +1 neighbour in x1 is the
next element (wrapping inside the row of L) and the +1 neighbour in x0 is L
elements further on (wrapping modulo d).  Every forward bond is summed as the
equation writes it, so at L = 2 each bond appears twice and at L = 1 the
kinetic term vanishes.

Pins (tests/test_oracle_action.py): constant fields (closed form), Z2 symmetry
(bitwise), plane waves (lattice-Laplacian eigenvalues), an independent dense
quadratic-form route, L = 1 and L = 2.
"""

import numpy as np


def site_terms(phi, L, m2, lam):
    """Per-site summands s_x of Eq. (1); phi has shape (N, L*L), float64."""
    phi = np.asarray(phi, dtype=np.float64)
    n = phi.shape[0]
    f = phi.reshape(n, L, L)
    kin = 0.0
    for axis in (1, 2):                      # mu = x0 and x1 directions
        fwd = np.roll(f, -1, axis=axis)      # phi_{x + mu}
        diff = fwd - f
        kin = kin + diff * diff
    f2 = f * f
    s = 0.5 * kin + 0.5 * m2 * f2 + lam * (f2 * f2)
    return s.reshape(n, L * L)


def action(phi, L, m2, lam):
    """S(phi) per particle, Eq. (1)."""
    return site_terms(phi, L, m2, lam).sum(axis=1)


def abs_site_sum(phi, L, m2, lam):
    """sum_x |s_x|: the scale against which action errors are measured."""
    return np.abs(site_terms(phi, L, m2, lam)).sum(axis=1)


def magnetisation(phi):
    """M = (1/V) sum_x phi_x per particle (Sec. 2)."""
    phi = np.asarray(phi, dtype=np.float64)
    return phi.mean(axis=1)


def u0(phi):
    """Gaussian reference U0 = 1/2 sum_x phi_x^2 per particle (Sec. 2)."""
    phi = np.asarray(phi, dtype=np.float64)
    return 0.5 * (phi * phi).sum(axis=1)
