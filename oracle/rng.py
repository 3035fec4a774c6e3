"""Random streams of the method, drawn from NumPy's Philox4x64-10 generator.

Every stream is keyed [seed, key1(stream, cfg, i)]; the j-th 64-bit word of a
stream is NumPy's j-th raw output for that key with counter 0, and a uniform is
u = (word >> 11) * 2^-53, a double in [0, 1).  Algorithm 1 draws its random
numbers with a library generator (cuRAND); here the library is NumPy's Philox.
"""

import numpy as np

TWO_M53 = 1.0 / 9007199254740992.0


def key1(stream, cfg, i):
    return (int(stream) << 56) | (int(cfg) << 48) | int(i)


def words(seed, k1, count):
    bg = np.random.Philox(key=np.array([seed, k1], dtype=np.uint64))
    return bg.random_raw(int(count)).astype(np.uint64)


def uniforms(seed, k1, count):
    w = words(seed, k1, count)
    return (w >> np.uint64(11)).astype(np.float64) * TWO_M53
