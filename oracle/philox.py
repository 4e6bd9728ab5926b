"""Philox4x32-10 counter-based generator (oracle side).

TEST INFRASTRUCTURE ONLY: nothing in the product path imports this package.

Written from the published definition of Philox (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11, Sec. 3): four 32-bit
counter words, two 32-bit key words, ten rounds; each round multiplies words 0
and 2 by fixed odd constants, mixes the high halves with words 1/3 and the key,
and the key is bumped by the Weyl constants between rounds.  The paper itself
draws its random quantities (payload bits, channels, noise, SNR; training
section and Eq. (1)) without naming a generator; this one is the project's choice,
implemented independently on the GPU side.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

# stream identifiers (third counter word)
STREAM_WEIGHTS = 0
STREAM_BITS = 1
STREAM_CHANNEL = 2
STREAM_NOISE = 3
STREAM_SLOT = 4


def philox4x32_10(ctr, key):
    """ctr: (..., 4) integer array (values < 2**32); key: (2,) integers.
    Returns (..., 4) uint32."""
    c = [np.asarray(ctr, dtype=np.uint64)[..., i].copy() for i in range(4)]
    k0 = int(key[0]) & 0xFFFFFFFF
    k1 = int(key[1]) & 0xFFFFFFFF
    for rnd in range(10):
        p0 = _M0 * c[0]
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c = [hi1 ^ c[1] ^ np.uint64(k0), lo1, hi0 ^ c[3] ^ np.uint64(k1), lo0]
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return np.stack(c, axis=-1).astype(np.uint32)


def seed_key(seed):
    seed = int(seed)
    return (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)


def draw(seed, batch_index, slot, stream, element):
    """Words for counter (batch_index, slot, stream, element); element may be an array."""
    element = np.asarray(element, dtype=np.uint64)
    ctr = np.zeros(element.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = int(batch_index) & 0xFFFFFFFF
    ctr[..., 1] = int(slot) & 0xFFFFFFFF
    ctr[..., 2] = int(stream)
    ctr[..., 3] = element
    return philox4x32_10(ctr, seed_key(seed))


def uniform(w):
    """Map a 32-bit word to an odd multiple of 2**-24 in (0, 1) (exact in fp32 and fp64)."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(9)).astype(np.float64) * 2.0 + 1.0) * 2.0 ** -24
