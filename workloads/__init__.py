"""Seeded synthetic workload generators.

This package is the only code shared by the CPU oracle and the GPU path. It
produces gate lists, Pauli terms and random draws (angles, noise patterns,
suffix lengths); it holds none of the simulation arithmetic.
"""
from .gen import (  # noqa: F401
    GATE_NAMES,
    Workload,
    TrieWorkload,
    NoisyWorkload,
    hea_layer,
    cz_layer,
    random_angles,
    config1,
    config2,
    config3,
    config4,
    config5_specs,
    config5_workload,
    random_pauli_terms,
    zz_terms,
    pauli_string,
    small_vqe,
    small_trie,
    small_noisy,
)
