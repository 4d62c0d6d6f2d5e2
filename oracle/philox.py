"""Philox4x32-10 counter-based generator and the random streams built on it.

Test infrastructure only (see ``oracle/__init__``).

The generator is the one published by Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4x32-bit counter,
a 2x32-bit key, ten rounds of two 32x32->64 multiplies with a Weyl key
schedule.  The device implements the same published definition on its own;
the two agree bit for bit on the integer outputs.

Random streams (the paper draws Gaussian fields for its bootstrap, Sec. 3.5,
and the log-determinant alternative it names in Sec. 3.3 -- stochastic trace
estimation -- needs probe vectors):

* Rademacher probe entry (index i, probe k):
      counter = (i, k, DOMAIN_PROBE, 0), key = (seed_lo, seed_hi)
      value = +1 if bit 0 of output word 0 is 0, else -1.
* Standard normal (index i, stream s):
      counter = (i, s, domain, 0), key = (seed_lo, seed_hi)
      u1 = ((w0 >> 5) * 2^26 + (w1 >> 6) + 0.5) / 2^53   in (0, 1)
      u2 = ((w2 >> 5) * 2^26 + (w3 >> 6)) / 2^53         in [0, 1)
      z  = sqrt(-2 ln u1) * cos(2 pi u2)                  (Box-Muller)
"""
import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

DOMAIN_PROBE = 1      # Rademacher / coloured probe signs
DOMAIN_FIELD = 2      # white noise driving a Gaussian-field sample
DOMAIN_NOISE = 3      # measurement (nugget) noise
DOMAIN_TARGET = 4     # noise of a simulated observation at a prediction cell


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on uint32 arrays (broadcast together); returns 4 arrays.

    Each round: (hi0, lo0) = M0*c0, (hi1, lo1) = M1*c2,
    c <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); then the key takes one
    Weyl step (k0 += W0, k1 += W1) before the next round.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK32 for c in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & MASK32)
    k1 = np.uint64(int(k1) & MASK32)
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    sh = np.uint64(32)
    msk = np.uint64(MASK32)
    for r in range(10):
        if r:
            k0 = np.uint64((int(k0) + W0) & MASK32)
            k1 = np.uint64((int(k1) + W1) & MASK32)
        p0 = c0 * m0
        p1 = c2 * m1
        hi0, lo0 = p0 >> sh, p0 & msk
        hi1, lo1 = p1 >> sh, p1 & msk
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def _key(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & MASK32, seed >> 32


def rademacher(index, probe, seed):
    """Rademacher signs (+1/-1, float64) for the given index and probe arrays."""
    k0, k1 = _key(seed)
    index = np.asarray(index)
    w0, _, _, _ = philox4x32_10(index, np.broadcast_to(probe, index.shape), DOMAIN_PROBE, 0, k0, k1)
    return 1.0 - 2.0 * (w0 & 1).astype(np.float64)


def normals(index, stream, seed, domain):
    """Standard normals for the given index array, stream id and domain."""
    k0, k1 = _key(seed)
    index = np.asarray(index)
    w0, w1, w2, w3 = philox4x32_10(index, np.broadcast_to(stream, index.shape), domain, 0, k0, k1)
    w0, w1, w2, w3 = (w.astype(np.float64) for w in (w0, w1, w2, w3))
    two26 = 67108864.0
    two53 = 9007199254740992.0
    u1 = (np.floor(w0 / 32.0) * two26 + np.floor(w1 / 64.0) + 0.5) / two53
    u2 = (np.floor(w2 / 32.0) * two26 + np.floor(w3 / 64.0)) / two53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def probe_matrix(rows, cols, num_probes, seed, colour_period=0):
    """Probe vectors (p, N) on the observed cells (rows, cols in compact
    order).

    colour_period == 0: Rademacher entries for probe k = 0..N-1.
    colour_period == c > 0 (reading of a lattice-coloured probing scheme):
    cell (r, col) has colour (r mod c) + c (col mod c); probe k (k < c^2)
    carries the Rademacher sign of that cell on colour-k cells and zero
    elsewhere, so that sum_k z_k z_k^T has unit diagonal and the estimate of
    tr log K stays unbiased.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    p = rows.size
    idx = np.arange(p)
    if colour_period <= 0:
        return np.stack([rademacher(idx, k, seed) for k in range(num_probes)], axis=1)
    c = colour_period
    colour = (rows % c) + c * (cols % c)
    Z = np.zeros((p, c * c))
    for k in range(c * c):
        Z[:, k] = np.where(colour == k, rademacher(idx, k, seed), 0.0)
    return Z
