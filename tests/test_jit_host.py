"""Generated pass kernels compile on the host (hipRTC, no GPU needed).

Covers every op form the generator emits (register, lane, thread and global
operands; diagonal sets with and without a register table; both kernel
forms) for several tile sizes.
"""
import numpy as np
import pytest

from paper_2609_23664_amd import binding as B
from workloads import gen


@pytest.fixture(autouse=True)
def _cache(tmp_path, monkeypatch):
    monkeypatch.setenv("QW_JIT_CACHE", str(tmp_path / "jit"))


def _random_gates(n, seed, count):
    g = np.random.default_rng(seed)
    names1 = ["X", "Y", "Z", "H", "S", "SDG", "T", "TDG", "RX", "RY", "RZ", "P"]
    gates = []
    for _ in range(count):
        if g.random() < 0.6:
            gates.append((names1[g.integers(len(names1))], (int(g.integers(n)),), float(g.uniform(0, 6.3))))
        else:
            a, b = g.choice(n, 2, replace=False)
            gates.append((("CNOT", "CZ")[int(g.integers(2))], (int(a), int(b)), 0.0))
    gates.append(("RENORM", (), 0.0))
    return gates


@pytest.mark.parametrize("n,tile", [(11, 10), (13, 12), (16, 14)])
def test_random_circuit_kernels_compile(n, tile):
    B.jit_precompile(n, _random_gates(n, 100 + n, 70), tile)


def test_vqe_suffix_kernels_compile_and_cache():
    w = gen.config2()
    s0 = B.jit_stats()
    B.jit_precompile(24, w.suffixes[0])
    s1 = B.jit_stats()
    assert s1["compiled"] + s1["disk_hits"] > s0["compiled"] + s0["disk_hits"]
    # same structure, other angles: no new kernels
    B.jit_precompile(24, w.suffixes[1])
    assert B.jit_stats()["compiled"] == s1["compiled"]


@pytest.mark.parametrize("n,tile", [(12, 10), (24, 14)])
def test_reducer_kernels_compile(n, tile):
    g = np.random.default_rng(n)
    terms = gen.random_pauli_terms(g, n, 30) + gen.zz_terms(g, n, 10)
    B.jit_precompile_terms(n, terms, tile)


@pytest.mark.parametrize("n,tile,seed", [(16, 10, 1), (18, 12, 2), (22, 14, 4)])
def test_relabel_kernels_compile(n, tile, seed):
    from tests.test_gpu_relabel import _ladder_circuit
    gates = _ladder_circuit(n, np.random.default_rng(7100 + seed), 3)
    assert any(p["out_cx"] for p in B.plan_describe(n, gates, tile)["passes"])
    B.jit_precompile(n, gates, tile)


@pytest.mark.parametrize("n,tile,layers", [(16, 12, 2), (18, 14, 3)])
def test_persistent_kernel_compiles(n, tile, layers):
    """The persistent kernel of a suffix batch (every pass structure of the
    batch, with the fused epilogue, in one code object) compiles on the host
    together with the per-pass kernels; a second request is served from the
    caches."""
    w = gen.small_vqe(n, 1, layers, 2, 12, seed=900 + n)
    s0 = B.jit_stats()
    B.jit_precompile_suffix(n, w.suffixes[0], w.terms, tile)
    s1 = B.jit_stats()
    assert s1["compiled"] + s1["disk_hits"] > s0["compiled"] + s0["disk_hits"]
    B.jit_precompile_suffix(n, w.suffixes[1], w.terms, tile)
    assert B.jit_stats()["compiled"] == s1["compiled"]
