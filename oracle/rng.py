"""Counter-based random streams for the oracle (test infrastructure only).

The paper's samplers draw Gaussian random-walk proposals and Metropolis
uniforms (Sec. 2 "Particle-based Monte Carlo methods" (i); App. A).  To make
the oracle and the GPU path consume identical randomness without passing
billions of numbers around, both sides implement the same counter-based
generator from its published definition: Philox4x32-10 (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).

Definition used here (written from the published description):

* state: a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1), all
  32-bit words;
* one round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 as 64-bit products with
  M0 = 0xD2511F53, M1 = 0xCD9E8D57; the new counter is
  (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
* ten rounds; between consecutive rounds the key is bumped by the Weyl
  constants (0x9E3779B9, 0xBB67AE85) modulo 2^32.

Stream map (shared convention of the oracle and the GPU path):

* key = (seed, run), both 32-bit;
* counter = (c0, c1, c2, c3) = (group, particle, step, level << 8 | purpose);
* purposes: INIT = 1, PROPOSE = 2, ACCEPT = 3, RESAMPLE = 4, NS_PICK = 5,
  SLICE = 6 (the j-th uniform of a slice move is word j mod 4 of the call
  with group j // 4);
* normals for the d sites of a particle: site x takes word (x mod 4) of the
  call with group = x // 4; Box-Muller pairs words (0, 1) and (2, 3);
* uniform from a word w: u = ((w >> 9) + 1/2) * 2^-23, i.e. the odd
  multiples of 2^-24 strictly inside (0, 1); 24 significant bits, so exact
  in float32 and float64;
* Box-Muller: r = sqrt(-2 ln u_a), z_a = r cos(2 pi u_b), z_b = r sin(2 pi u_b).

Pins (tests/test_oracle_rng.py): the three Philox4x32-10 known-answer vectors
distributed with the generator's publication; chi-square uniformity of the
uniforms; normal moments; exactness of the uniform conversion.
"""

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85

INIT = 1
PROPOSE = 2
ACCEPT = 3
RESAMPLE = 4
NS_PICK = 5
SLICE = 6

_MASK32 = np.uint64(0xFFFFFFFF)
_SHIFT32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 of counter words (c0..c3) under key (k0, k1).

    Arguments broadcast as numpy integer arrays; returns four uint32 arrays.
    """
    c = [np.asarray(x, dtype=np.uint64) & _MASK32 for x in (c0, c1, c2, c3)]
    k0 = np.asarray(k0, dtype=np.uint64) & _MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & _MASK32
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & _MASK32
            k1 = (k1 + np.uint64(PHILOX_W1)) & _MASK32
        p0 = m0 * c[0]          # < 2^64: exact in uint64
        p1 = m1 * c[2]
        c = [(p1 >> _SHIFT32) ^ c[1] ^ k0,
             p1 & _MASK32,
             (p0 >> _SHIFT32) ^ c[3] ^ k1,
             p0 & _MASK32]
    return tuple(x.astype(np.uint32) for x in c)


def uniform(w):
    """uint32 word -> float64 uniform ((w >> 9) + 1/2) * 2^-23 in (0, 1)."""
    w = np.asarray(w, dtype=np.uint32)
    return ((w >> np.uint32(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(wa, wb):
    """Two uint32 words -> two float64 standard normals (Box-Muller)."""
    ua = uniform(wa)
    ub = uniform(wb)
    r = np.sqrt(-2.0 * np.log(ua))
    t = 2.0 * np.pi * ub
    return r * np.cos(t), r * np.sin(t)


def counter3(level, purpose):
    return (int(level) << 8) | int(purpose)


def normals(seed, run, level, step, purpose, particles, d):
    """Standard normals z[i, x] for the given particle indices and d sites.

    ``particles`` is an integer array of particle (row) indices; the result has
    shape (len(particles), d) in float64.
    """
    particles = np.asarray(particles, dtype=np.int64)
    n_groups = (d + 3) // 4
    g = np.arange(n_groups, dtype=np.uint64)[None, :]
    p = particles.astype(np.uint64)[:, None]
    w0, w1, w2, w3 = philox4x32_10(g, p, step, counter3(level, purpose), seed, run)
    z0, z1 = box_muller(w0, w1)
    z2, z3 = box_muller(w2, w3)
    z = np.stack([z0, z1, z2, z3], axis=-1).reshape(len(particles), 4 * n_groups)
    return z[:, :d]


def words(seed, run, level, step, purpose, particles):
    """Word 0 of the call (group 0, particle i, step, level/purpose) per particle."""
    particles = np.asarray(particles, dtype=np.uint64)
    w0, _, _, _ = philox4x32_10(0, particles, step, counter3(level, purpose), seed, run)
    return w0


def accept_uniforms(seed, run, level, step, particles):
    """Metropolis uniforms u_i (float64) for one step."""
    return uniform(words(seed, run, level, step, ACCEPT, particles))


def slice_uniform(seed, run, level, step, particle, j):
    """The j-th uniform of a slice-sampling move (float64): word j mod 4 of
    the call (group j // 4, particle, step, level/SLICE)."""
    w = philox4x32_10(j // 4, particle, step, counter3(level, SLICE), seed, run)[j % 4]
    return float(uniform(w))


def resample_word(seed, run, level):
    """The single uint32 U that drives systematic resampling at a level."""
    return int(words(seed, run, level, 0, RESAMPLE, [0])[0])
