"""Shared helpers of the GPU parity tests: oracle-side references and comparisons."""

import math
import sys

import numpy as np

from oracle.noise import expand, site_channels
from oracle.sampling import boundary_distance, cdf, sample
from oracle.statevector import run_record


def log(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def oracle_states(circ, records, params=None):
    ss = expand(circ)
    ch = site_channels(circ)
    out = []
    bits = []
    for rec in records:
        psi, b = run_record(circ, rec, params=params, steps_sites=ss, chans=ch)
        out.append(psi / math.sqrt(math.fsum(np.abs(psi) ** 2)))
        bits.append(b)
    return out, bits


def compare_shots(psi, gpu_bits, m, seed, cfg, alpha, chunk=4096, u=None, tol=1e-6):
    """Shot indices of one trajectory vs the oracle: equal except where the sorted
    uniform lies within ``tol`` of a CDF boundary.  Returns (mismatches, excused)."""
    idx, us = sample(psi, m, seed, cfg, alpha, chunk=chunk, u=u)
    g = np.asarray(gpu_bits, dtype=np.int64)
    bad = np.flatnonzero(g != idx)
    if bad.size == 0:
        return 0, 0
    d = boundary_distance(cdf(psi), us[bad])
    unexcused = int(np.sum(d >= tol))
    return unexcused, int(bad.size - unexcused)
