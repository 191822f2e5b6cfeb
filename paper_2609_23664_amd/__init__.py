"""MI355X-native prefix-reuse statevector path (gfx950).

The hot path -- gate passes, boundary snapshots, batched suffix replay,
Pauli-sum expectations and Z-basis sampling -- runs in the HIP kernels of
``libqw.so`` behind the C ABI declared in ``include/qw.h``; ``binding``
marshals arguments to it and ``planner`` decides reuse (Eq. (1)
fingerprints, Table II legality, Eq. (2) cost rule).
"""
__all__ = ["binding", "planner"]
