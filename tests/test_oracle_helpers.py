"""Pins of the oracle's Python-side helpers that the GPU parity tests use as
references: the row normalisation of the Sec. 5 preprocessing
(``oracle.normalize_rows``) and the exact prox of every row with its prices
gathered through the CSR pattern (``oracle.row_prox_all``, Sec. 2.2).

Each pin checks what the definition fixes independently of how the helper
computes it: a hand-worked example, per-row maxima, ratios inside a row, the
row subproblem's optimality conditions with prices gathered here entry by
entry, and the closed form of a one-good row."""
import numpy as np
import pytest

import oracle


def test_normalize_rows_hand_example():
    # rows: [2, 4, 1], empty, [0, 5] (an explicit zero), [3]
    row_ptr = np.array([0, 3, 3, 5, 6])
    u = np.array([2.0, 4.0, 1.0, 0.0, 5.0, 3.0])
    uh, mx = oracle.normalize_rows(row_ptr, u)
    np.testing.assert_array_equal(uh, [0.5, 1.0, 0.25, 0.0, 1.0, 1.0])
    np.testing.assert_array_equal(mx, [4.0, 0.0, 5.0, 3.0])


@pytest.mark.parametrize("seed", range(6))
def test_normalize_rows_properties(seed):
    """Every non-empty row's maximum becomes exactly 1, the row's ratios are
    kept, u_hat * rowmax restores u, and explicit zeros stay zero; rows of
    every length, including empty ones and rows whose maximum is a middle or
    last entry."""
    rng = np.random.default_rng(seed)
    n = 200
    lens = rng.integers(0, 12, n)
    lens[rng.integers(0, n, 10)] = 0
    row_ptr = np.concatenate([[0], np.cumsum(lens)])
    u = np.exp(rng.standard_normal(row_ptr[-1]) * 2.0)
    u[rng.random(u.size) < 0.1] = 0.0
    for i in range(n):  # Assumption 1: every buyer values some good
        a, b = row_ptr[i], row_ptr[i + 1]
        if a < b and u[a:b].max() == 0.0:
            u[a + (b - a) // 2] = 1.5
    uh, mx = oracle.normalize_rows(row_ptr, u)
    assert uh.shape == u.shape and mx.shape == (n,)
    for i in range(n):
        a, b = row_ptr[i], row_ptr[i + 1]
        if a == b:
            continue
        row, rh = u[a:b], uh[a:b]
        assert mx[i] == row.max()
        assert rh.max() == 1.0
        assert rh[np.argmax(row)] == 1.0
        np.testing.assert_allclose(rh * mx[i], row, rtol=1e-15, atol=0)
        k = int(np.argmax(row))
        np.testing.assert_allclose(rh * row[k], row * rh[k], rtol=1e-15)
        assert np.all(rh[row == 0.0] == 0.0)
        assert np.all(rh >= 0.0)


def _market(rng, n, m, dmax):
    lens = rng.integers(1, dmax + 1, n)
    cols = [np.sort(rng.choice(m, size=int(d), replace=False)) for d in lens]
    row_ptr = np.concatenate([[0], np.cumsum(lens)])
    col = np.concatenate(cols).astype(np.int32)
    u = rng.uniform(0.01, 1.0, col.size)
    uh, _ = oracle.normalize_rows(row_ptr, u)
    w = rng.uniform(0.5, 1.5, n)
    x = rng.uniform(0.0, 0.05, col.size) * (rng.random(col.size) < 0.7)
    p = rng.uniform(0.3, 3.0, m)
    return row_ptr, col, uh, w, x, p


@pytest.mark.parametrize("seed", range(4))
def test_row_prox_all_satisfies_every_row_kkt(seed):
    """For every row i, with p_j gathered here as p[col[k]] entry by entry:
    s_i = u_hat_i^T x_i, x >= 0, and the row subproblem's optimality
    conditions -w u_j/s + p_j + (x_j - x^k_j)/tau = 0 on x_j > 0, >= 0 on
    x_j = 0 (Sec. 2.2)."""
    rng = np.random.default_rng(50 + seed)
    n, m = 120, 40
    row_ptr, col, uh, w, xk, p = _market(rng, n, m, 30)
    tau = [0.01, 0.3, 2.0, 20.0][seed]
    x, s = oracle.row_prox_all(row_ptr, col, uh, w, xk, p, tau)
    assert x.shape == xk.shape and s.shape == (n,)
    assert np.all(x >= 0.0)
    for i in range(n):
        a, b = row_ptr[i], row_ptr[i + 1]
        pj = np.array([p[int(col[k])] for k in range(a, b)])
        ui, xi, xki = uh[a:b], x[a:b], xk[a:b]
        assert s[i] > 0
        assert abs(ui @ xi - s[i]) <= 1e-12 * max(1.0, s[i])
        grad = -w[i] * ui / s[i] + pj + (xi - xki) / tau
        scale = pj + np.abs(xki) / tau + w[i] * ui / s[i]
        pos = xi > 0
        assert np.all(np.abs(grad[pos]) <= 1e-9 * scale[pos])
        assert np.all(grad[~pos] >= -1e-9 * scale[~pos])


def test_row_prox_all_one_good_rows_closed_form():
    """Rows with one good: s solves s = u (a + tau w u / s) with
    a = x^k - tau p_j, i.e. s = (u a + sqrt(u^2 a^2 + 4 tau w u^2)) / 2 and
    x = s / u (cf. eq. update:t)."""
    rng = np.random.default_rng(7)
    n, m = 50, 9
    row_ptr = np.arange(n + 1)
    col = rng.integers(0, m, n).astype(np.int32)
    uh = np.ones(n)
    w = rng.uniform(0.5, 1.5, n)
    xk = rng.uniform(0.0, 1.0, n)
    p = rng.uniform(0.2, 4.0, m)
    tau = 0.7
    x, s = oracle.row_prox_all(row_ptr, col, uh, w, xk, p, tau)
    a = xk - tau * p[col]
    s_ref = (a + np.sqrt(a * a + 4 * tau * w)) / 2
    np.testing.assert_allclose(s, s_ref, rtol=1e-13)
    np.testing.assert_allclose(x, s_ref, rtol=1e-13)


def test_row_prox_all_uses_each_rows_own_prices_and_budget():
    """Permuting the goods (relabelling col and p together) and permuting the
    buyers (rows with their budgets) permutes the result the same way."""
    rng = np.random.default_rng(11)
    n, m = 60, 25
    row_ptr, col, uh, w, xk, p = _market(rng, n, m, 12)
    tau = 0.5
    x, s = oracle.row_prox_all(row_ptr, col, uh, w, xk, p, tau)
    # relabel goods: good j becomes perm[j]; keep each row sorted
    perm = rng.permutation(m)
    inv = np.argsort(perm)
    p2 = p[inv]
    col2 = perm[col]
    x2 = np.empty_like(x)
    uh2, xk2 = np.empty_like(uh), np.empty_like(xk)
    order = np.empty(col.size, np.int64)
    for i in range(n):
        a, b = row_ptr[i], row_ptr[i + 1]
        o = a + np.argsort(col2[a:b])
        order[a:b] = o
    col2, uh2, xk2 = col2[order], uh[order], xk[order]
    x2, s2 = oracle.row_prox_all(row_ptr, col2.astype(np.int32), uh2, w, xk2, p2, tau)
    np.testing.assert_allclose(s2, s, rtol=1e-13)
    np.testing.assert_allclose(x2, x[order], rtol=1e-12, atol=1e-15)
    # reverse the buyers
    lens = np.diff(row_ptr)[::-1]
    rp3 = np.concatenate([[0], np.cumsum(lens)])
    idx = np.concatenate([np.arange(row_ptr[i], row_ptr[i + 1]) for i in range(n - 1, -1, -1)])
    x3, s3 = oracle.row_prox_all(rp3, col[idx], uh[idx], w[::-1], xk[idx], p, tau)
    np.testing.assert_allclose(s3, s[::-1], rtol=1e-13)
    np.testing.assert_allclose(x3, x[idx], rtol=1e-12, atol=1e-15)
