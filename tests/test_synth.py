"""Seeded input generators: the structure the paper's workloads prescribe
(shapes, patterns, value ranges); no method arithmetic is involved."""
import numpy as np

from paper_2506_06258_amd import synth


def test_table2_market_structure():
    """Sec. 5.1 generator: every buyer values each good with probability q,
    u ~ U(0, 1), w ~ U(0, 1); rows hold distinct sorted goods and every good
    has a buyer (Assumption 1)."""
    n, m, q = 3000, 400, 0.05
    mk = synth.table2_market(n, m, q, 3)
    deg = np.diff(mk.row_ptr)
    assert mk.n == n and mk.m == m and deg.min() >= 1
    # Binomial(m, q) degrees: mean m q, variance m q (1 - q)
    assert abs(deg.mean() - m * q) < 4 * np.sqrt(m * q * (1 - q) / n)
    assert abs(deg.var() / (m * q * (1 - q)) - 1.0) < 0.15
    for i in range(0, n, 97):
        row = mk.col[mk.row_ptr[i]:mk.row_ptr[i + 1]]
        assert np.all(np.diff(row) > 0)
    assert np.bincount(mk.col, minlength=m).min() >= 1
    assert mk.u.dtype == np.float32 and 0.0 < mk.u.min() and mk.u.max() < 1.0
    assert 0.0 < mk.w.min() and mk.w.max() < 1.0
    # goods are uniform: every good's share of the entries near 1/m
    share = np.bincount(mk.col, minlength=m) / mk.nnz
    assert np.abs(share * m - 1.0).max() < 0.5
    # seeded: the same seed gives the same market, another seed another
    again = synth.table2_market(n, m, q, 3)
    assert np.array_equal(again.col, mk.col) and np.array_equal(again.u, mk.u)
    assert not np.array_equal(synth.table2_market(n, m, q, 4).col[:50], mk.col[:50])
