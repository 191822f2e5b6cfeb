"""Seeded generators for the synthetic workloads.

A gate record is a tuple ``(name, qubits, param)``:

* ``name``  one of :data:`GATE_NAMES`;
* ``qubits`` a tuple of qubit indices (control first for ``CNOT``);
* ``param`` a Python float (binary64), the rotation angle for ``RX/RY/RZ/P``
  and ``0.0`` otherwise.

``RENORM`` is a marker with no qubits: the state is renormalised at that
point of the gate list (used after inserted noise jumps).

``MEASURE`` and ``RESET`` act on one qubit; their ``param`` is the uniform
draw u in [0, 1) that decides the outcome (1 iff u < P(qubit = 1)); RESET
then flips the qubit back to 0 when the outcome is 1.

A Pauli term is ``(coeff, x_mask, z_mask)``: bit q of ``x_mask`` is set when
the term has X or Y on qubit q, bit q of ``z_mask`` when it has Z or Y.

Qubit q is bit q of the basis index (little-endian).

Every random draw comes from numpy's PCG64 seeded through
``SeedSequence(entropy=base, spawn_key=path)``; the base seeds of the five
workload families are 101, 202, 303, 404 and 505. Nothing here simulates
anything: these functions only list gates and draw numbers.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

GATE_NAMES = (
    "X", "Y", "Z", "H", "S", "SDG", "T", "TDG",
    "RX", "RY", "RZ", "P",
    "CNOT", "CZ",
    "RENORM",
    "MEASURE", "RESET",
)

Gate = Tuple[str, Tuple[int, ...], float]
Term = Tuple[float, int, int]

TWO_PI = 2.0 * math.pi


def rng(base: int, *path: int) -> np.random.Generator:
    """PCG64 stream for (base seed, path)."""
    ss = np.random.SeedSequence(entropy=base, spawn_key=tuple(int(p) for p in path))
    return np.random.Generator(np.random.PCG64(ss))


def random_angles(g: np.random.Generator, count: int) -> List[float]:
    """``count`` angles uniform on [0, 2*pi)."""
    return [float(a) for a in g.uniform(0.0, TWO_PI, size=count)]


def hea_layer(n: int, angles: Sequence[float]) -> List[Gate]:
    """Hardware-efficient layer: RY(theta_q) then RZ(phi_q) on every qubit,
    then CNOT(q -> q+1) for q = 0..n-2 in ascending order.

    ``angles`` holds 2n values: theta_0, phi_0, theta_1, phi_1, ...
    """
    assert len(angles) == 2 * n
    gates: List[Gate] = []
    for q in range(n):
        gates.append(("RY", (q,), float(angles[2 * q])))
        gates.append(("RZ", (q,), float(angles[2 * q + 1])))
    for q in range(n - 1):
        gates.append(("CNOT", (q, q + 1), 0.0))
    return gates


def cz_layer(n: int, angles: Sequence[float]) -> List[Gate]:
    """RY(theta_q) on every qubit, then CZ(q, q+1) for q = 0..n-2."""
    assert len(angles) == n
    gates: List[Gate] = [("RY", (q,), float(angles[q])) for q in range(n)]
    gates += [("CZ", (q, q + 1), 0.0) for q in range(n - 1)]
    return gates


def pauli_string(term: Term, n: int) -> str:
    """Readable form, qubit 0 leftmost: e.g. 'XIZY'."""
    _, x, z = term
    out = []
    for q in range(n):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        out.append("IXZY"[xb | (zb << 1)])
    return "".join(out)


def random_pauli_terms(g: np.random.Generator, n: int, count: int,
                       max_weight: int = 4) -> List[Term]:
    """``count`` distinct Pauli strings: weight uniform on {1..max_weight},
    positions uniform without replacement, each non-identity factor uniform
    over {X, Y, Z}; coefficients N(0, 1)."""
    seen = set()
    terms: List[Term] = []
    while len(terms) < count:
        w = int(g.integers(1, max_weight + 1))
        pos = g.choice(n, size=w, replace=False)
        kinds = g.integers(0, 3, size=w)
        x = z = 0
        for q, k in zip(pos, kinds):
            if k == 0:      # X
                x |= 1 << int(q)
            elif k == 1:    # Y
                x |= 1 << int(q)
                z |= 1 << int(q)
            else:           # Z
                z |= 1 << int(q)
        if (x, z) in seen:
            continue
        seen.add((x, z))
        terms.append((float(g.standard_normal()), x, z))
    return terms


def zz_terms(g: np.random.Generator, n: int, count: int) -> List[Term]:
    """Each term is Z_i (probability 1/2, i uniform on 0..n-1) or
    Z_i Z_{i+1} (i uniform on 0..n-2); coefficients N(0, 1)."""
    terms: List[Term] = []
    for _ in range(count):
        if g.random() < 0.5:
            i = int(g.integers(0, n))
            z = 1 << i
        else:
            i = int(g.integers(0, n - 1))
            z = (1 << i) | (1 << (i + 1))
        terms.append((float(g.standard_normal()), 0, z))
    return terms


@dataclass
class Workload:
    """Tasks that share one prefix and differ in their suffixes."""
    name: str
    n: int
    prefix: List[Gate]
    suffixes: List[List[Gate]]
    terms: List[Term] = field(default_factory=list)
    shots: int = 0
    seed: int = 0

    @property
    def n_tasks(self) -> int:
        return len(self.suffixes)

    def task_gates(self, t: int) -> List[Gate]:
        return list(self.prefix) + list(self.suffixes[t])


@dataclass
class TrieWorkload:
    """A prefix tree: ``levels[d]`` lists the nodes at depth d+1 as
    ``(parent_index, gates)`` where the parent index refers to
    ``levels[d-1]`` (and is -1 at depth 1, whose parent is |0...0>).
    ``leaves`` lists ``(parent_index_in_last_level, gates)``."""
    name: str
    n: int
    levels: List[List[Tuple[int, List[Gate]]]]
    leaves: List[Tuple[int, List[Gate]]]
    shots: int = 0
    seed: int = 0

    def leaf_path(self, k: int) -> List[Gate]:
        """All gates from |0...0> to leaf k, in order."""
        parent, gates = self.leaves[k]
        chain = [gates]
        for d in range(len(self.levels) - 1, -1, -1):
            p, g = self.levels[d][parent]
            chain.append(g)
            parent = p
        out: List[Gate] = []
        for g in reversed(chain):
            out += g
        return out


@dataclass
class NoisyWorkload:
    """A shared noiseless prefix and one suffix per trajectory; each
    trajectory's suffix is the common suffix with Pauli jumps inserted."""
    name: str
    n: int
    prefix: List[Gate]
    suffix: List[Gate]
    trajectories: List[List[Gate]]
    p: float
    shots: int = 0
    seed: int = 0


def insert_jumps(g: np.random.Generator, suffix: Sequence[Gate], p: float) -> List[Gate]:
    """For every gate and every qubit it touches, with probability p insert a
    Pauli uniform over {X, Y, Z} on that qubit right after the gate, each
    followed by a RENORM marker."""
    out: List[Gate] = []
    for gate in suffix:
        out.append(gate)
        for q in gate[1]:
            if g.random() < p:
                kind = ("X", "Y", "Z")[int(g.integers(0, 3))]
                out.append((kind, (q,), 0.0))
                out.append(("RENORM", (), 0.0))
    return out


def _hea_layers(g: np.random.Generator, n: int, layers: int) -> List[Gate]:
    out: List[Gate] = []
    for _ in range(layers):
        out += hea_layer(n, random_angles(g, 2 * n))
    return out


# ---------------------------------------------------------------- families

def small_vqe(n: int, prefix_layers: int, suffix_layers: int, n_tasks: int,
              n_terms: int, seed: int, layer: str = "hea",
              weight: int = 4) -> Workload:
    """A VQE-shaped workload of any size (the configurations below are
    instances of it)."""
    g = rng(seed, 0)
    if layer == "hea":
        prefix = _hea_layers(g, n, prefix_layers)
    else:
        prefix = []
        for _ in range(prefix_layers):
            prefix += cz_layer(n, random_angles(g, n))
    suffixes = []
    for t in range(n_tasks):
        gt = rng(seed, 1, t)
        if layer == "hea":
            suffixes.append(_hea_layers(gt, n, suffix_layers))
        else:
            s: List[Gate] = []
            for _ in range(suffix_layers):
                s += cz_layer(n, random_angles(gt, n))
            suffixes.append(s)
    gh = rng(seed, 2)
    if layer == "hea":
        terms = random_pauli_terms(gh, n, n_terms, max_weight=min(weight, n))
    else:
        terms = zz_terms(gh, n, n_terms)
    return Workload(f"vqe_{layer}_{n}q", n, prefix, suffixes, terms, seed=seed)


def config1() -> Workload:
    """10 qubits, RY + CZ-ladder layers: 3 shared layers, 16 tasks with one
    own layer each, 10 random Z_i / Z_i Z_{i+1} terms."""
    w = small_vqe(10, 3, 1, 16, 10, seed=101, layer="cz")
    w.name = "vqe_cz_10q_16t"
    return w


def config2() -> Workload:
    """24 qubits, 8 hardware-efficient layers: 6 shared, 2 per task,
    64 tasks, 50 random Pauli strings of weight <= 4."""
    w = small_vqe(24, 6, 2, 64, 50, seed=202, layer="hea")
    w.name = "vqe_hea_24q_64t"
    return w


def small_trie(n: int, depth: int, branching: int, layers_per_level: int,
               max_extra: int, seed: int, shots: int) -> TrieWorkload:
    levels: List[List[Tuple[int, List[Gate]]]] = []
    prev = 1
    for d in range(depth - 1):
        nodes = []
        for k in range(prev * branching):
            gk = rng(seed, 10 + d, k)
            nodes.append(((k // branching) if d > 0 else -1,
                          _hea_layers(gk, n, layers_per_level)))
        levels.append(nodes)
        prev = len(nodes)
    leaves = []
    for k in range(prev * branching):
        gk = rng(seed, 20, k)
        extra = int(gk.integers(1, max_extra + 1))
        gates = _hea_layers(gk, n, layers_per_level + extra)
        leaves.append(((k // branching) if depth > 1 else -1, gates))
    return TrieWorkload(f"trie_{n}q", n, levels, leaves, shots=shots, seed=seed)


def config3() -> TrieWorkload:
    """20 qubits; prefix tree of depth 3 and branching 8, two HEA layers per
    level; each of the 512 leaves adds 1..12 more layers; 1024 shots."""
    w = small_trie(20, 3, 8, 2, 12, seed=303, shots=1024)
    w.name = "trie_hea_20q_512leaves"
    return w


def small_noisy(n: int, prefix_layers: int, suffix_layers: int, n_traj: int,
                p: float, seed: int, shots: int) -> NoisyWorkload:
    g = rng(seed, 0)
    prefix = _hea_layers(g, n, prefix_layers)
    suffix = _hea_layers(g, n, suffix_layers)
    trajs = [insert_jumps(rng(seed, 3, t), suffix, p) for t in range(n_traj)]
    return NoisyWorkload(f"noisy_{n}q", n, prefix, suffix, trajs, p,
                         shots=shots, seed=seed)


def config4() -> NoisyWorkload:
    """22 qubits; 10 shared noiseless layers; 256 trajectories of a 4-layer
    suffix with single-qubit Pauli jumps at p = 1e-3 per (gate, qubit);
    1024 shots per trajectory."""
    w = small_noisy(22, 10, 4, 256, 1e-3, seed=404, shots=1024)
    w.name = "noisy_hea_22q_256traj"
    return w


@dataclass
class Config5Spec:
    index: int
    n: int
    total_layers: int
    prefix_layers: int
    n_tasks: int
    spread: int
    negative: bool


def config5_specs(count: int = 2000) -> List[Config5Spec]:
    """Workload shapes for the cost-model study: qubits 12..26, prefix
    fraction 0..0.95, 1..256 tasks (log-uniform), suffix spread 0..10 layers,
    10% negative controls (no shared prefix)."""
    specs = []
    for i in range(count):
        g = rng(505, 0, i)
        n = int(g.integers(12, 27))
        total = int(g.integers(2, 17))
        frac = float(g.uniform(0.0, 0.95))
        prefix_layers = min(total - 1, int(round(frac * total)))
        tasks = int(round(math.exp(g.uniform(0.0, math.log(256.0)))))
        tasks = max(1, min(256, tasks))
        spread = int(g.integers(0, 11))
        negative = bool(g.random() < 0.10)
        if negative:
            prefix_layers = 0
        specs.append(Config5Spec(i, n, total, prefix_layers, tasks, spread, negative))
    return specs


def config5_workload(spec: Config5Spec, max_tasks: int | None = None) -> Workload:
    """Materialise one cost-model workload. Task t's suffix has
    (total - prefix) + U{0..spread} layers. Negative controls have no
    shared layer at all (every task draws its own angles from layer 0)."""
    n = spec.n
    g = rng(505, 1, spec.index)
    prefix = _hea_layers(g, n, spec.prefix_layers)
    tasks = spec.n_tasks if max_tasks is None else min(spec.n_tasks, max_tasks)
    suffixes = []
    for t in range(tasks):
        gt = rng(505, 2, spec.index, t)
        extra = int(gt.integers(0, spec.spread + 1))
        suffixes.append(_hea_layers(gt, n, spec.total_layers - spec.prefix_layers + extra))
    terms = random_pauli_terms(rng(505, 3, spec.index), n, 8)
    return Workload(f"cm_{spec.index}", n, prefix, suffixes, terms, seed=505)


def syndrome_round(d: int, draws: Sequence[float]) -> List[Gate]:
    """One syndrome-extraction round of a distance-d bit-flip repetition code:
    data qubits 0..d-1, ancilla d+i measures Z_i Z_{i+1} through CNOT(i, d+i)
    and CNOT(i+1, d+i), then a RESET of the ancilla with draw draws[i]."""
    g: List[Gate] = []
    for i in range(d - 1):
        g += [("CNOT", (i, d + i), 0.0), ("CNOT", (i + 1, d + i), 0.0),
              ("RESET", (d + i,), float(draws[i]))]
    return g


def qec_repetition(d: int = 12, n_tasks: int = 64, seed: int = 606) -> Workload:
    """Repetition-code memory experiment with mid-circuit measurements
    (2d - 1 qubits). Shared prefix: encode cos(t/2)|0..0> + sin(t/2)|1..1>
    on the data (RY on qubit 0 and a CNOT chain), then one syndrome round.
    Task k: a coherent error RX(e_k) on data qubit k mod d (e_k uniform on
    [0.05, 0.3]), then one more syndrome round with its own draws. Terms: the
    data parities Z_i Z_{i+1} and Z_0, coefficient 1."""
    n = 2 * d - 1
    g = rng(seed, 0)
    theta = float(g.uniform(0.3, 1.2))
    prefix: List[Gate] = [("RY", (0,), theta)] + [("CNOT", (i, i + 1), 0.0) for i in range(d - 1)]
    prefix += syndrome_round(d, g.uniform(0.0, 1.0, size=d - 1))
    suffixes = []
    for k in range(n_tasks):
        gk = rng(seed, 1, k)
        e = float(gk.uniform(0.05, 0.3))
        suffixes.append([("RX", (k % d,), e)] + syndrome_round(d, gk.uniform(0.0, 1.0, size=d - 1)))
    terms = [(1.0, 0, (1 << i) | (1 << (i + 1))) for i in range(d - 1)] + [(1.0, 0, 1)]
    return Workload(name=f"qec_repetition_d{d}_{n}q_{n_tasks}t", n=n, prefix=prefix,
                    suffixes=suffixes, terms=terms)


CLIFFORD_1Q = ("H", "S", "SDG", "X", "Y", "Z")


def clifford_prefix_vqe(n: int = 24, layers: int = 12, n_tasks: int = 64, seed: int = 707) -> Workload:
    """A Clifford prefix (layers of one random single-qubit Clifford per
    qubit, then the CNOT ladder) shared by n_tasks tasks whose suffixes and
    terms are those of the 24-qubit VQE configuration (2 HEA layers, 50
    Pauli terms)."""
    g = rng(seed, 0)
    prefix: List[Gate] = []
    for _ in range(layers):
        for q in range(n):
            prefix.append((CLIFFORD_1Q[int(g.integers(len(CLIFFORD_1Q)))], (q,), 0.0))
        prefix += [("CNOT", (q, q + 1), 0.0) for q in range(n - 1)]
    base = config2()
    return Workload(name=f"clifford_prefix_{n}q_{layers}l_{n_tasks}t", n=n, prefix=prefix,
                    suffixes=[list(s) for s in base.suffixes[:n_tasks]], terms=list(base.terms))
