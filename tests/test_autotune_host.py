"""Host checks of the autotuner's workload signature: it follows the pass
structure (gate kinds, qubits, task shape, outputs), not the angles."""
from paper_2609_23664_amd import autotune as A


def _tasks(a):
    return [[("RY", (0,), a), ("CNOT", (0, 1), 0.0)], [("RZ", (1,), 2 * a)]]


def test_signature_ignores_angles():
    assert A.signature(4, _tasks(0.1), 0, True) == A.signature(4, _tasks(2.3), 0, True)


def test_signature_follows_structure():
    base = A.signature(4, _tasks(0.1), 0, True)
    assert A.signature(5, _tasks(0.1), 0, True) != base
    assert A.signature(4, _tasks(0.1), 16, True) != base
    assert A.signature(4, _tasks(0.1), 0, False) != base
    t = _tasks(0.1)
    t[0][1] = ("CNOT", (1, 0), 0.0)
    assert A.signature(4, t, 0, True) != base
    t = _tasks(0.1)
    t[1][0] = ("RY", (1,), 0.2)
    assert A.signature(4, t, 0, True) != base
    assert A.signature(4, _tasks(0.1)[:1], 0, True) != base
