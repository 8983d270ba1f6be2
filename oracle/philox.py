"""Philox-4x32-10 counter-based generator (oracle side).

Written from the published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): ten rounds of the
4x32 Philox S-box with multipliers 0xD2511F53 / 0xCD9E8D57 and key
schedule increments 0x9E3779B9 / 0xBB67AE85.  The GPU library carries its own
independent implementation of the same definition.

Sampling keys: the random number for sample ``j`` at chain site ``k`` is
philox((k, j_lo, j_hi, 0x5A4D5053), (seed_lo, seed_hi)) word 0 and 1 combined
into a 53-bit uniform in [0, 1).
"""
from __future__ import annotations

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF
SAMPLE_TAG = 0x5A4D5053


def _mulhilo(a: int, b: int):
    p = a * b
    return (p >> 32) & MASK, p & MASK


def philox4x32_10(ctr, key):
    c0, c1, c2, c3 = [int(v) & MASK for v in ctr]
    k0, k1 = [int(v) & MASK for v in key]
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniform(seed: int, sample: int, site: int) -> float:
    """53-bit uniform in [0, 1) for (seed, sample, site)."""
    out = philox4x32_10((site, sample & MASK, (sample >> 32) & MASK, SAMPLE_TAG),
                        (seed & MASK, (seed >> 32) & MASK))
    bits53 = ((out[0] << 21) | (out[1] >> 11)) & ((1 << 53) - 1)
    return bits53 / float(1 << 53)
