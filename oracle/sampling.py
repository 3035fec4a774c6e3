"""Shot sampling from a prepared state (Sec. 2.1 shots; Sec. 3 bulk draws of m_alpha shots).

p_x = |psi_x|^2 / ||psi||^2 (||psi||^2 by math.fsum); CDF = np.cumsum(p), an
inclusive prefix sum in float64.  Shot j of trajectory alpha uses
u_j = (word_j >> 11) 2^-53 from the stream [seed, key1(SAMPLER, cfg, alpha)]
(or caller-given uniforms).  Uniforms are sorted within consecutive chunks of
``chunk`` shots and each is mapped to idx_j = min(searchsorted(CDF,
u_j * CDF[-1], side='right'), N - 1): the inverse-CDF reading of
index(r, {p}) in Algorithm 1, which never selects a zero-probability x.
Shots come out chunk by chunk, ascending in u within a chunk.
`distinct` lists a trajectory's distinct shot values with their counts and
`expected_distinct` gives the closed-form expectation of their number.
"""

import math

import numpy as np

from .rng import key1, uniforms

STREAM_SAMPLER = 2


def probabilities(psi):
    w = psi.real ** 2 + psi.imag ** 2
    return w / math.fsum(w)


def cdf(psi):
    return np.cumsum(probabilities(psi))


def chunk_sorted(u, chunk):
    out = np.array(u, dtype=np.float64, copy=True)
    for a in range(0, out.size, chunk):
        out[a:a + chunk] = np.sort(out[a:a + chunk])
    return out


def draw(c, u):
    """Upper-bound search of u * total in the inclusive CDF, clamped to N - 1."""
    total = c[-1]
    idx = np.searchsorted(c, u * total, side="right")
    return np.minimum(idx, c.size - 1)


def sample(psi, m, seed, cfg, alpha, chunk=4096, u=None):
    """Return (idx, sorted uniforms) for m shots of trajectory ``alpha``."""
    if u is None:
        u = uniforms(seed, key1(STREAM_SAMPLER, cfg, alpha), m)
    us = chunk_sorted(u, chunk)
    return draw(cdf(psi), us), us


def boundary_distance(c, u):
    """Distance in u-space from u to the nearest CDF boundary (normalised CDF)."""
    total = c[-1]
    cn = c / total
    pos = np.searchsorted(cn, u, side="right")
    lo = np.where(pos > 0, cn[np.maximum(pos - 1, 0)], 0.0)
    hi = np.where(pos < cn.size, cn[np.minimum(pos, cn.size - 1)], 1.0)
    return np.minimum(np.abs(u - lo), np.abs(hi - u))


def distinct(shots):
    """Distinct values of one trajectory's shots (Sec. 4, Fig. 4: the unique
    fraction is len(values) / len(shots)), in order of first appearance, with
    how often each occurs: written out as a loop over the shots."""
    first = {}
    values, counts = [], []
    for x in np.asarray(shots).tolist():
        j = first.get(x)
        if j is None:
            first[x] = len(values)
            values.append(x)
            counts.append(1)
        else:
            counts[j] += 1
    return np.asarray(values, dtype=np.int64), np.asarray(counts, dtype=np.int64)


def expected_distinct(p, m):
    """E[#distinct values among m iid draws from p] = sum_x 1 - (1 - p_x)^m
    (each x is missed by all m draws with probability (1 - p_x)^m)."""
    p = np.asarray(p, dtype=np.float64)
    if m == 0:
        return 0.0
    with np.errstate(divide="ignore"):
        return float(np.sum(-np.expm1(m * np.log1p(-p))))
