"""The paper's operation count of one sum-factorization kernel (test infrastructure;
oracle only): checks the library's flop model, which uses the same count for
its non-collocated contractions."""
from __future__ import annotations


def sumfact_cost(m, n) -> int:
    """Flops of one sum-factorization kernel (Section 3.2, eq. sumfactcost):
    2 * sum_k prod_{i<=k} m_i * prod_{j>=k} n_j for d = len(m) directions."""
    d = len(m)
    total = 0
    for k in range(d):
        a = 1
        for i in range(k + 1):
            a *= m[i]
        b = 1
        for j in range(k, d):
            b *= n[j]
        total += a * b
    return 2 * total
