"""Counter-based random numbers for the oracle (test infrastructure only).

The paper draws its Gaussian white noise with cuRAND on the GPU and the C++
standard library on the CPU (Sec. "What cuPSS calculates", the paragraph after
the six-step list) and fixes no generator.  Both the oracle and the GPU path
therefore implement one published counter-based generator from its
definition, so that a noise value is a pure function of (seed, step, mode):

* Philox4x32 with 10 rounds, from J. K. Salmon, M. A. Moraes, R. O. Dror and
  D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 3.3.
  One round maps the counter (c0, c1, c2, c3) with key (k0, k1) to
      (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
  where hi/lo are the two 32-bit halves of the 64-bit product; between rounds
  the key is bumped by the Weyl constants (W0, W1).  The first round uses the
  key as given.
* uniforms u = (floor(w / 2^9) + 1/2) * 2^-23 from a 32-bit word w: an odd
  multiple of 2^-24 in (0, 1), exactly representable in IEEE binary32, so the
  FP32 GPU path and this FP64 oracle hold the same value.
* Box-Muller: g1 = sqrt(-2 ln u0) cos(2 pi u1), g2 = sqrt(-2 ln u0) sin(2 pi u1)
  (G. E. P. Box and M. E. Muller, Ann. Math. Stat. 29, 610 (1958)).

Everything is vectorised over numpy uint64 arrays holding 32-bit values, so a
32x32-bit product never overflows.
"""

import numpy as np

# Multipliers and key increments of Philox4x32 (Salmon et al. SC'11, Sec. 3.3).
PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

# Stream tags: the fourth counter word separates noise draws from initial
# fields (a reading of the paper's silence on how noise is keyed).
TAG_NOISE = 0
TAG_INIT = 1


def _u32(x):
    return np.asarray(x, dtype=np.uint64) & np.uint64(MASK32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds on broadcastable arrays of 32-bit words.

    Returns a tuple of four uint64 arrays holding the 32-bit output words.
    """
    c0, c1, c2, c3 = _u32(c0), _u32(c1), _u32(c2), _u32(c3)
    k0, k1 = _u32(k0), _u32(k1)
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    mask = np.uint64(MASK32)
    sh = np.uint64(32)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(PHILOX_W0)) & mask
            k1 = (k1 + np.uint64(PHILOX_W1)) & mask
        p0 = m0 * c0          # < 2^64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & mask
        hi1, lo1 = p1 >> sh, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def seed_key(seed):
    """Split a 64-bit seed into the Philox key (low word, high word)."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK32, seed >> 32


def uniform23(w):
    """(floor(w/2^9) + 1/2) * 2^-23: exact in binary32, strictly inside (0,1)."""
    w = _u32(w)
    return ((w >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(u0, u1):
    """Two independent standard normals from two uniforms (Box & Muller 1958)."""
    r = np.sqrt(-2.0 * np.log(u0))
    ang = 2.0 * np.pi * u1
    return r * np.cos(ang), r * np.sin(ang)


def gaussian_pair(counter, step, field, seed, tag=TAG_NOISE):
    """(g1, g2) for Philox counter (counter, step, field, tag) and a 64-bit seed."""
    k0, k1 = seed_key(seed)
    w0, w1, _, _ = philox4x32_10(counter, step, field, tag, k0, k1)
    return box_muller(uniform23(w0), uniform23(w1))


def uniform_site(counter, field, seed, tag=TAG_INIT):
    """First uniform of Philox counter (counter, 0, field, tag) for initial fields."""
    k0, k1 = seed_key(seed)
    w0, _, _, _ = philox4x32_10(counter, 0, field, tag, k0, k1)
    return uniform23(w0)
