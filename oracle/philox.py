"""Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as
1, 2, 3", SC'11), written from its published definition in exact integer arithmetic.

The paper draws one uniform variate u_i per pixel for stochastic rounding (Sec. 4.2,
eq. holdout) and does not fix the generator; this implementation keys Philox with the 64-bit
scene seed and counts with (pixel div 4, frame, stream, j): the four output words of one
block serve four consecutive pixels (word pixel mod 4).  u = (word >> 8) * 2^-24 lies in
[0, 1 - 2^-24] and is exact in binary32 and binary64.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_LO = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten rounds; round r uses the key bumped r times by the Weyl constants."""
    c = [np.asarray(x, dtype=np.uint64) & _LO for x in (c0, c1, c2, c3)]
    c = list(np.broadcast_arrays(*c))
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for _ in range(10):
        p0 = _M0 * c[0]               # < 2^64, exact in uint64
        p1 = _M1 * c[2]
        hi0, lo0 = p0 >> _S32, p0 & _LO
        hi1, lo1 = p1 >> _S32, p1 & _LO
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + _W0) & _LO
        k1 = (k1 + _W1) & _LO
    return c


STREAM_U = 0


def uniform24(seed: int, pixel, frame: int, stream: int = STREAM_U, j: int = 0):
    """u in [0, 1): 24 high bits of output word (pixel mod 4) of the block with counter
    (pixel div 4, frame, stream, j)."""
    seed = int(seed)
    pixel = np.asarray(pixel, dtype=np.uint64)
    words = philox4x32_10(pixel >> np.uint64(2), np.uint64(frame), np.uint64(stream), np.uint64(j),
                          seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w = np.choose((pixel & np.uint64(3)).astype(np.int64), words)
    return (w >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
