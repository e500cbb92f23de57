"""Flop bookkeeping against hand-worked values of eq. sumfactcost."""
import os

from oracle.cost import sumfact_cost

HERE = os.path.dirname(os.path.abspath(__file__))


def test_sumfact_cost_golden():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "sumfact_cost.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) >= 5
    for r in rows:
        m, n, c = tuple(map(int, r[:3])), tuple(map(int, r[3:6])), int(r[6])
        assert sumfact_cost(m, n) == c, r


def test_sumfact_cost_scaling():
    """Linear in m_0 (the property behind the over-integration factor of Section 3.2)."""
    for m0 in range(1, 9):
        assert sumfact_cost((2 * m0, 5, 5), (5, 5, 5)) == 2 * sumfact_cost((m0, 5, 5), (5, 5, 5))
