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
