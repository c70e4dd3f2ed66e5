"""FP64 CPU oracle for the particle Monte Carlo samplers of "Particle Monte Carlo
methods for Lattice Field Theory" (arXiv 2511.15196).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call it; the product
path (the C-ABI library and its Python binding) never does, and shares no code
with it.

Everything here is numpy in float64 unless a function says otherwise (the
precision-emulation helpers round to float32 / bfloat16 / float16 on purpose).
Each function cites the passage of the paper it follows:

* ``rng``       -- counter-based Philox4x32-10 streams, uniforms, Box-Muller
                   normals (the paper draws Gaussian proposals, App. A; the
                   generator is Salmon et al., SC'11).
* ``action``    -- the periodic-lattice phi^4 action, Sec. 2 Eq. (1), the
                   magnetisation order parameter and the Gaussian reference U0
                   of the tempered family (Sec. 2).
* ``smc``       -- adaptive tempered SMC with covariance-preconditioned
                   random-walk Metropolis rejuvenation (Sec. 2 "Particle-based
                   Monte Carlo methods" (i), App. A).
* ``irmh``      -- the same tempered SMC with an independent Metropolis-Hastings
                   proposal fitted to the particles (Sec. 2 (ii), App. A).
* ``hmc``       -- the same tempered SMC with Hamiltonian Monte Carlo
                   trajectories, diagonal mass (Sec. 2 (iii), App. A).
* ``ns``        -- nested sampling with likelihood-constrained random-walk
                   refill (Sec. 2 (iv), App. A).
* ``precision`` -- round-to-nearest-even emulation of the reduced-precision
                   proposal product.

Parity status of every function is listed in each module's header.
"""

from . import rng, action, precision, smc, irmh, hmc, ns  # noqa: F401
