"""Philox4x32-10 and the Gaussian sketch, CPU reference (test infrastructure).

The paper only says that the sketching matrix has independent entries drawn
from a Gaussian with mean 0 and variance 1 (Sec. 4.2, Alg. 1 step 1). To make
GPU and CPU draw the *same* sketch, both sides implement one counter-based
generator from its published definition:

* Philox4x32 with 10 rounds, J. K. Salmon, M. A. Moraes, R. O. Dror,
  D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11.
  Round function on a 4x32-bit counter (c0,c1,c2,c3) and a 2x32-bit key
  (k0,k1), multipliers M0=0xD2511F53, M1=0xCD9E8D57, Weyl key increments
  W0=0x9E3779B9, W1=0xBB67AE85.
* Box-Muller (G. E. P. Box, M. E. Muller, 1958) on two 53-bit uniforms.

Sketch definition (shared reading, also stated in the library header):
  entry (j, c) of the n x l sketch, j < n, c < l, uses one Philox call with
  key = (seed mod 2^32, seed div 2^32) and counter = (j mod 2^32, j div 2^32,
  c div 2, stream), stream = 0 for the sketch.  With outputs x0..x3:
      a  = (x0 >> 5) * 2^26 + (x1 >> 6)          (53 bits)
      b  = (x2 >> 5) * 2^26 + (x3 >> 6)
      u1 = (a + 0.5) * 2^-53    in (0, 1)
      u2 =  b        * 2^-53    in [0, 1)
      rho = sqrt(-2 ln u1),  theta = 6.283185307179586 * u2
      even c -> rho cos(theta),  odd c -> rho sin(theta).
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)
SH32 = np.uint64(32)

TWO_PI = 6.283185307179586  # the double nearest to 2*pi


def _mulhilo(a, b):
    """32x32 -> 64-bit product split into (hi, lo) 32-bit words."""
    p = a * b  # both < 2^32, so the product fits in uint64 exactly
    return p >> SH32, p & MASK32


def philox4x32_10(ctr, key):
    """Apply Philox4x32-10.

    ctr: uint array of shape (..., 4) with 32-bit words; key: (..., 2).
    Returns a uint64 array of shape (..., 4) holding 32-bit outputs.
    """
    ctr = np.asarray(ctr, dtype=np.uint64) & MASK32
    key = np.asarray(key, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = key[..., 0].copy(), key[..., 1].copy()
    for rnd in range(10):
        if rnd > 0:  # key schedule: bump between rounds
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return np.stack([c0, c1, c2, c3], axis=-1)


def sketch_bits(seed, n, l, stream=0):
    """Raw Philox outputs used for the sketch: uint32 array (n, ceil(l/2), 4)."""
    seed = int(seed)
    npairs = (l + 1) // 2
    j = np.arange(n, dtype=np.uint64)[:, None]
    t = np.arange(npairs, dtype=np.uint64)[None, :]
    ctr = np.empty((n, npairs, 4), dtype=np.uint64)
    ctr[..., 0] = j & MASK32
    ctr[..., 1] = j >> SH32
    ctr[..., 2] = t
    ctr[..., 3] = np.uint64(stream)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    out = philox4x32_10(ctr, np.broadcast_to(key, (n, npairs, 2)))
    return out.astype(np.uint32)


def bits_to_gaussian(bits, l):
    """Box-Muller map from sketch_bits() to the n x l FP64 sketch."""
    x = bits.astype(np.uint64)
    a = (x[..., 0] >> np.uint64(5)) * np.uint64(1 << 26) + (x[..., 1] >> np.uint64(6))
    b = (x[..., 2] >> np.uint64(5)) * np.uint64(1 << 26) + (x[..., 3] >> np.uint64(6))
    u1 = (a.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    rho = np.sqrt(-2.0 * np.log(u1))
    theta = TWO_PI * u2
    n, npairs = bits.shape[:2]
    out = np.empty((n, 2 * npairs), dtype=np.float64)
    out[:, 0::2] = rho * np.cos(theta)
    out[:, 1::2] = rho * np.sin(theta)
    return out[:, :l]


def gaussian_sketch(seed, n, l, stream=0):
    """The n x l FP64 Gaussian sketch (Sec. 4.2, Alg. 1 step 1) for `seed`."""
    return bits_to_gaussian(sketch_bits(seed, n, l, stream), l)
