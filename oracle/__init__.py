"""FP64 CPU oracle for the PTSBE hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct NumPy (complex128 / float64) implementations of
what Pre-Trajectory Sampling with Batched Execution computes:

* ``gates``        gate matrices and the full-unitary Kronecker builder (pins).
* ``channels``     Kraus channels, the CPTP condition and unitary-mixture
                   detection (Sec. 2.2, noise-channel paragraph and feature 2).
* ``noise``        expansion of a circuit + noise model into an ordered list of
                   steps and noise sites (Algorithm 1's ``lookUp``).
* ``rng``          the Philox4x64-10 streams, via NumPy's own Philox generator.
* ``pts``          pre-trajectory sampling: proportional, Algorithm 2 as
                   printed, most-likely-first enumeration, shot allocation
                   (Sec. 3.1).
* ``statevector``  fixed-Kraus trajectory preparation (Sec. 3, batched
                   execution) and mid-circuit measure-reset.
* ``sampling``     norm, probabilities, CDF and sorted-uniform shot draws
                   (Sec. 2.1 shots; Sec. 3 bulk sampling).
* ``densitymatrix`` exact channel evolution for <= 8 qubits (Sec. 2.1).
* ``adjoint``      expectation values and adjoint gradients of the
                   probability-weighted trajectory ensemble.
* ``baseline``     conventional per-shot trajectories (Algorithm 1).
* ``stabilizer``   Pauli-frame propagation used to pin measure-reset records.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It imports nothing from the GPU package
and shares no code with it.
"""
