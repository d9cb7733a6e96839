"""Philox4x32-10 counter-based generator and Box-Muller normals (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper asks only that every noise mode be drawn independently on every site
from a Gaussian (Sec. VI, first paragraph); it names a fast generator but does
not fix one.  This build fixes the draw as follows, on both sides:

* generator: Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw
  ("Parallel random numbers: as easy as 1, 2, 3", SC'11): one round maps
  (x0, x1, x2, x3) with key (k0, k1) to
      (hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)),
  M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by the Weyl constants
  (0x9E3779B9, 0xBB67AE85) between rounds; 10 rounds.
* counter (site, step, block | tag << 16, replica), key (seed mod 2^32,
  seed >> 32), site = x + nx*(y + ny*z).
* Box-Muller pairs: pair p takes a full 32-bit word r for its radius,
  R = sqrt(-2 ln u), u = (r + 1) 2^-32 in (0, 1], and 16 bits h for its angle,
  theta = 2 pi v, v = (h + 1) 2^-16; (z_2p, z_2p+1) = R (cos theta, sin theta).
  With P = ceil(K/2) pairs for K normals, the words w_0, w_1, ... are the
  outputs of blocks 0, 1, ... in order; pair p uses w_p for its radius and
  w_{P + p//2} for its angle (high half for even p, low half for odd p).  A
  D3Q19 site (K = 15) thus needs 12 words (3 blocks), a D2Q9 site (K = 6) 5
  words (2 blocks).  Normal number k drives the k-th non-conserved mode in
  basis order.

Pinned by: an independent library implementation of the same bijection
(rocRAND's host-callable ``ten_rounds``) compared word for word in the tests,
and by moment/KS statistics of the normals.
"""

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Apply Philox4x32-10 to counters and keys (uint32 values, scalars or
    arrays that broadcast together).

    Returns four uint32 arrays.  Arithmetic is done in uint64 so the 32x32->64
    products are exact.
    """
    x0 = np.asarray(c0, dtype=np.uint64) & MASK32
    x1 = np.asarray(c1, dtype=np.uint64) & MASK32
    x2 = np.asarray(c2, dtype=np.uint64) & MASK32
    x3 = np.asarray(c3, dtype=np.uint64) & MASK32
    k0 = np.asarray(k0, dtype=np.uint64) & MASK32
    k1 = np.asarray(k1, dtype=np.uint64) & MASK32
    x0, x1, x2, x3, k0, k1 = np.broadcast_arrays(x0, x1, x2, x3, k0, k1)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
        p0 = M0 * x0
        p1 = M1 * x2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        x0, x1, x2, x3 = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def key_of(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def block_words(sites, step, block, seed, tag=0, replica=0):
    """The four Philox words of noise block ``block`` for every site in ``sites``
    at time step ``step``: array of shape (4, len(sites)), uint32."""
    k0, k1 = key_of(seed)
    sites = np.asarray(sites, dtype=np.uint64)
    c2 = (int(block) | (int(tag) << 16)) & 0xFFFFFFFF
    return np.stack(philox4x32_10(sites, int(step) & 0xFFFFFFFF, c2, int(replica), k0, k1))


def uniform(r):
    """u = (r + 1) 2^-32 in (0, 1], FP64."""
    return (np.asarray(r, dtype=np.float64) + 1.0) * 2.0 ** -32


def pair_normals(r, h):
    """Box-Muller on a radius word r (uint32 array) and 16-bit angles h:
    returns (R cos theta, R sin theta), FP64."""
    R = np.sqrt(-2.0 * np.log(uniform(r)))
    theta = 2.0 * np.pi * ((np.asarray(h, dtype=np.float64) + 1.0) * 2.0 ** -16)
    return R * np.cos(theta), R * np.sin(theta)


def normals(nsites, step, count, seed, tag=0, replica=0, sites=None):
    """``count`` standard normals per site for sites 0..nsites-1 (or for the
    given linear site indices ``sites``): shape (count, number of sites)."""
    sites = np.arange(nsites, dtype=np.uint64) if sites is None else np.asarray(sites, np.uint64)
    npair = (count + 1) // 2
    nword = npair + (npair + 1) // 2
    nblk = (nword + 3) // 4
    words = np.concatenate([block_words(sites, step, b, seed, tag, replica) for b in range(nblk)])
    out = []
    for p in range(npair):
        a = words[npair + p // 2]
        h = (a >> np.uint32(16)) if p % 2 == 0 else (a & np.uint32(0xFFFF))
        c, s = pair_normals(words[p], h)
        out += [c, s]
    return np.stack(out)[:count]
