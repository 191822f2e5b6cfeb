"""Host side of measured gate lists in the library (no GPU): plan cost by
segments (each measurement one state read, its projector folded into the next
segment) and the refusal of a measurement inside a pass plan."""
import pytest

from paper_2609_23664_amd import binding as B


def test_plan_cost_by_segments():
    from paper_2609_23664_amd import binding as B
    n = 16
    a = [("RY", (q,), 0.1 * q) for q in range(n)] + [("CNOT", (q, q + 1), 0.0) for q in range(n - 1)]
    b = [("RX", (q,), 0.2) for q in range(n)]
    pa, _ = B.plan_cost(n, a, 12)
    pb, _ = B.plan_cost(n, [("PROJ0", (3,), 1.0)] + b, 12)
    passes, by = B.plan_cost(n, a + [("MEASURE", (3,), 0.25)] + b, 12)
    sb = 8.0 * 2 ** n
    assert passes == pa + pb
    assert by == passes * 2 * sb + sb
    with pytest.raises(B.QwError):
        B.plan_describe(n, a + [("MEASURE", (3,), 0.25)], 12)
    with pytest.raises(B.QwError):
        B.plan_cost(n, a + [("MEASURE", (3,), 1.5)], 12)
