"""Seeded synthetic workloads for the PTSBE hot path.

This package only *describes* inputs: circuits as symbolic op lists (gate names,
qubits, angles), noise channels by name and probability, and the sampling
options of each workload.  It holds none of the method's arithmetic (no gate
matrices, no Kraus operators, no sampling), so the oracle and the HIP path can
both consume it without sharing any computation.

Qubit convention: basis index x = sum_q x_q 2^q (qubit 0 is the least
significant bit).
"""

from .circuits import (  # noqa: F401
    brick_circuit,
    c1_workload,
    c2_workload,
    c3_workload,
    c4_workload,
    c5_workload,
    product_circuit,
    random_small_circuit,
    surface_code_d3,
    hea_circuit,
    STREAM_PTS,
    STREAM_SAMPLER,
    STREAM_BASELINE,
    key1,
)
