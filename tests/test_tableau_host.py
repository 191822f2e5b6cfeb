"""Stabilizer tableau of the library (host side, no GPU) against the
oracle's dense statevector: after random Clifford circuits every stabilizer
row (x, z, r) is a +1 eigenoperator of the oracle's state, i.e.
<P(x, z)> = (-1)^r with P = i^{|x & z|} X^x Z^z; the rows keep the symplectic
relations of a tableau (stabilizers commute pairwise, destabilizer i
anticommutes exactly with stabilizer i); a non-Clifford gate is refused and
leaves the tableau unchanged; the tableau artifact passes Table II's
STAB -> SV rule and fails STAB -> STAB on a statevector backend."""
import numpy as np
import pytest

import oracle
from paper_2609_23664_amd import binding as B

CLIFF1 = ["X", "Y", "Z", "H", "S", "SDG"]


def random_clifford(n, g, count):
    gates = []
    for _ in range(count):
        u = g.random()
        if u < 0.3 and n > 1:
            a, b = (int(v) for v in g.choice(n, 2, replace=False))
            gates.append(("CNOT" if u < 0.2 else "CZ", (a, b), 0.0))
        else:
            gates.append((CLIFF1[int(g.integers(len(CLIFF1)))], (int(g.integers(n)),), 0.0))
    return gates


def _anti(x1, z1, x2, z2):
    return (bin(int(x1) & int(z2)).count("1") + bin(int(z1) & int(x2)).count("1")) & 1


@pytest.mark.parametrize("n,count,seed", [(1, 10, 1), (3, 30, 2), (6, 80, 3), (10, 200, 4)])
def test_stabilizers_fix_the_oracle_state(n, count, seed):
    g = np.random.default_rng(seed)
    for _ in range(4):
        gates = random_clifford(n, g, count)
        tb = B.Tableau(n)
        tb.apply(gates)
        x, z, r = tb.rows()
        psi = oracle.simulate(n, gates)
        vals = oracle.expect_terms(psi, n, [(1.0, int(x[n + i]), int(z[n + i])) for i in range(n)])
        assert np.allclose(vals, [(-1.0) ** int(r[n + i]) for i in range(n)], atol=1e-12), (gates, vals, r)
        for i in range(2 * n):
            for j in range(2 * n):
                a = _anti(x[i], z[i], x[j], z[j])
                if i >= n and j >= n:
                    assert a == 0
                elif i < n and j >= n:
                    assert a == (1 if j == i + n else 0)
        tb.free()


def test_non_clifford_is_refused_and_leaves_tableau():
    tb = B.Tableau(3)
    tb.apply([("H", (0,), 0.0), ("CNOT", (0, 1), 0.0)])
    before = [a.copy() for a in tb.rows()]
    with pytest.raises(B.QwError) as ei:
        tb.apply([("H", (2,), 0.0), ("RY", (1,), 0.3)])
    assert ei.value.code == 5  # QW_E_UNSUPPORTED
    for a, b in zip(before, tb.rows()):
        assert np.array_equal(a, b)
    with pytest.raises(B.QwError):
        tb.apply([("CNOT", (1, 1), 0.0)])


def test_tableau_artifact_legality():
    tb = B.Tableau(4)
    art = tb.artifact(b"t" * 32)
    assert art["kind"] == 2 and art["exactness"] == 1 and art["backend"] == 2 and art["n_qubits"] == 4
    rc, js = B.legality_check(art["kind"], art["exactness"], art["backend"], 4, 1, 1)
    assert rc == 0 and js == ""
    rc, js = B.legality_check(art["kind"], art["exactness"], art["backend"], 4, 2, 1)
    assert rc == 4 and "FORBIDDEN_CONVERSION" in js
