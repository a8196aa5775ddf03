"""Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011) on Python integers, the reference that the
deblocking initialisation on the GPU is checked against (test infrastructure).

A round multiplies counter words 0 and 2 by 0xD2511F53 and 0xCD9E8D57 (32 x 32
-> 64 bits) and forms (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); the key grows by
the Weyl constants 0x9E3779B9 and 0xBB67AE85 between rounds.  All arithmetic is
on Python ints (NumPy integer scalars would wrap at 64 bits in the products).
"""

MASK = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """Four 32-bit output words of counter (4 words) under key (2 words)."""
    c = [int(v) & MASK for v in counter]
    k0, k1 = int(key[0]) & MASK, int(key[1]) & MASK
    for r in range(10):
        if r:
            k0, k1 = (k0 + 0x9E3779B9) & MASK, (k1 + 0xBB67AE85) & MASK
        p0, p1 = 0xD2511F53 * c[0], 0xCD9E8D57 * c[2]
        c = [(p1 >> 32) ^ c[1] ^ k0, p1 & MASK, (p0 >> 32) ^ c[3] ^ k1, p0 & MASK]
    return c
