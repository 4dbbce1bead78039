"""Reference sparse embedding W (n x w) for the sketch A D W.

The paper only asks for a random sparse embedding with a few non-zeros per row
(Sec. 2, the sparse-embedding result quoted before Sec. 3; Sec. 5 lists other
admissible constructions).  This module fixes one concrete, counter-based
construction so that two independent implementations can agree bit for bit:

  mix(z)      SplitMix64 output function (Steele, Lea and Flood, "Fast
              splittable pseudorandom number generators", OOPSLA 2014):
                z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
                z ^= z >> 27; z *= 0x94D049BB133111EB;
                z ^= z >> 31            (all arithmetic mod 2^64)
  base(k, r)  mix(seed + 0x9E3779B97F4A7C15 * (1 + k*s + r))
  h(j, r)     mix(base(k, r) XOR j)
  bucket      r*(w/s) + (((h >> 32) * (w/s)) >> 32)
  sign        -1 if h is odd else +1

Row j of W has exactly one entry per block r = 0..s-1 of w/s columns
(block CountSketch; s = 1 is the plain CountSketch), with value +-1.  k is a
salt (the IPM iteration when a fresh W is drawn every iteration, as step (a) of
Alg. 2 does).  Entries are not scaled by 1/sqrt(s): scaling W by a constant
changes neither the preconditioned CG iterates nor the correction vector v.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MASK = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB


def mix_int(z: int) -> int:
    """SplitMix64 output function on one Python integer (mod 2^64)."""
    z &= MASK
    z ^= z >> 30
    z = (z * M1) & MASK
    z ^= z >> 27
    z = (z * M2) & MASK
    z ^= z >> 31
    return z


def mix_array(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output function, elementwise on a uint64 array (numpy uint64
    multiplication wraps mod 2^64)."""
    z = np.asarray(z, dtype=np.uint64).copy()
    z ^= z >> np.uint64(30)
    z *= np.uint64(M1)
    z ^= z >> np.uint64(27)
    z *= np.uint64(M2)
    z ^= z >> np.uint64(31)
    return z


def splitmix64_stream(state: int, count: int):
    """The SplitMix64 generator itself: state += golden gamma; output mix(state)."""
    out = []
    for _ in range(count):
        state = (state + GOLDEN) & MASK
        out.append(mix_int(state))
    return out


def sketch_hash(seed: int, k: int, s: int, n: int, w: int):
    """Bucket and sign of every (row j, block r) pair: arrays of shape (n, s)."""
    if s < 1 or w % s != 0:
        raise ValueError("s must divide w")
    blk = w // s
    j = np.arange(n, dtype=np.uint64)
    bucket = np.empty((n, s), dtype=np.int64)
    sign = np.empty((n, s), dtype=np.int8)
    for r in range(s):
        base = mix_int((seed + GOLDEN * (1 + k * s + r)) & MASK)
        h = mix_array(np.uint64(base) ^ j)
        hi = h >> np.uint64(32)
        bucket[:, r] = r * blk + ((hi * np.uint64(blk)) >> np.uint64(32)).astype(np.int64)
        sign[:, r] = np.where((h & np.uint64(1)) == 1, -1, 1).astype(np.int8)
    return bucket, sign


def sketch_matrix(seed: int, k: int, s: int, n: int, w: int) -> sp.csr_matrix:
    """Explicit W (n x w) with the entries of `sketch_hash`."""
    bucket, sign = sketch_hash(seed, k, s, n, w)
    rows = np.repeat(np.arange(n), s)
    return sp.csr_matrix((sign.ravel().astype(np.float64), (rows, bucket.ravel())),
                         shape=(n, w))


# ----------------------------------------------------------------------------
# Gaussian sketching matrix (Sec. 5: W_G with N(0, 1) entries; the paper's
# experiments use it)
# ----------------------------------------------------------------------------
#
# Entries (j, c) and (j, c + 1), c even, of the n x w matrix, with salt k
# (one Box-Muller pair; Box and Muller, 1958):
#   base      mix(seed + 0x9E3779B97F4A7C15 * (1 + k))
#   q         j w + c
#   h1, h2    mix(base XOR 2 q), mix(base XOR (2 q + 1))
#   u1        ((h1 >> 11) + 1) 2^-53   in (0, 1]
#   u2        (h2 >> 11) 2^-53         in [0, 1)
#   r, t      sqrt(-2 ln u1), 2 pi u2
#   W_jc      r cos t,  W_j,c+1  r sin t   (when c + 1 < w)
# each rounded to 8 significant bits, ties to even.
# The last step makes the entry exactly representable in bfloat16 and makes two
# implementations agree even where their log / cos differ in the last bit of
# the FP64 result (they disagree only when z lies within an FP64 rounding error
# of a tie of the 8-bit rounding).

def round_to_8_bits(z: np.ndarray) -> np.ndarray:
    """Round to the nearest value with an 8-bit significand, ties to even."""
    m, e = np.frexp(z)                      # z = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)


def gaussian_sketch_matrix(seed: int, k: int, n: int, w: int) -> np.ndarray:
    """The dense n x w Gaussian sketching matrix with salt k (see above)."""
    base = mix_int(seed + GOLDEN * (1 + k))
    c = np.arange(w, dtype=np.uint64)
    even = c & ~np.uint64(1)
    q = np.arange(n, dtype=np.uint64)[:, None] * np.uint64(w) + even[None, :]
    h1 = mix_array(np.uint64(base) ^ (q * np.uint64(2)))
    h2 = mix_array(np.uint64(base) ^ (q * np.uint64(2) + np.uint64(1)))
    u1 = ((h1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (h2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    z = np.where((c % np.uint64(2) == 0)[None, :], r * np.cos(t), r * np.sin(t))
    return round_to_8_bits(z)
