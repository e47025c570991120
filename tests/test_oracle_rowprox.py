"""Pins of the oracle's row subproblem (Sec. 2.2) against what the paper and
the mathematics fix: the subproblem's own optimality conditions, a generic
bound-constrained optimiser, the closed form of a one-good row, the
bracketing lemma of Alg. 3 and the interval shrink of the k-section search."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle


def random_row(rng, d, scale_tau=1.0, negative_a=False):
    u = rng.uniform(0.01, 1.0, d)
    u /= u.max()
    xk = rng.uniform(0.0, 0.05, d) * (rng.random(d) < 0.7)
    p = rng.uniform(0.5, 2.0, d)
    w = rng.uniform(0.5, 1.5)
    tau = scale_tau * rng.uniform(1e-3, 5e-2)
    if negative_a:
        tau *= 50.0
    return u, xk, p, w, tau


def row_objective(x, u, xk, p, w, tau):
    s = u @ x
    return -w * np.log(s) + p @ x + np.sum((x - xk) ** 2) / (2 * tau)


@pytest.mark.parametrize("seed", range(30))
def test_exact_prox_satisfies_row_kkt(seed):
    """x >= 0 with  -w u_j/s + p_j + (x_j - xk_j)/tau = 0 where x_j > 0 and
    >= 0 where x_j = 0 (the row KKT system, with the u_ij factor)."""
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 60))
    u, xk, p, w, tau = random_row(rng, d, negative_a=(seed % 3 == 0))
    x, s = oracle.row_prox_exact(u, xk, p, w, tau)
    assert s > 0 and np.all(x >= 0)
    assert abs(u @ x - s) <= 1e-12 * max(1.0, s)
    grad = -w * u / s + p + (x - xk) / tau
    scale = np.abs(p) + np.abs(xk) / tau + w * u / s
    pos = x > 0
    assert np.all(np.abs(grad[pos]) <= 1e-9 * scale[pos])
    assert np.all(grad[~pos] >= -1e-9 * scale[~pos])


@pytest.mark.parametrize("seed", range(12))
def test_exact_prox_matches_generic_optimizer(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(2, 12))
    u, xk, p, w, tau = random_row(rng, d)
    x, s = oracle.row_prox_exact(u, xk, p, w, tau)
    x0 = np.full(d, max(xk.mean(), 1e-3))
    res = minimize(row_objective, x0, args=(u, xk, p, w, tau), method="L-BFGS-B",
                   bounds=[(0, None)] * d, options=dict(ftol=1e-15, gtol=1e-12, maxiter=10000))
    f_exact = row_objective(x, u, xk, p, w, tau)
    assert f_exact <= res.fun + 1e-10 * abs(res.fun) + 1e-12
    assert np.allclose(x, res.x, atol=2e-5 * max(1.0, x.max()))


def test_paper_printed_update_is_not_the_prox():
    """The update printed in Sec. 2.2 without the u_ij factor does not solve
    the row subproblem when the row's utilities differ (reading A1)."""
    rng = np.random.default_rng(7)
    u, xk, p, w, tau = random_row(rng, 8)
    x, s = oracle.row_prox_exact(u, xk, p, w, tau)
    # root of s = sum_j u_j [xk_j - tau p_j + tau w / s]_+ by bisection
    lo, hi = 1e-12, 1e6
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        g = u @ np.maximum(xk - tau * p + tau * w / mid, 0)
        lo, hi = (mid, hi) if mid < g else (lo, mid)
    x_lit = np.maximum(xk - tau * p + tau * w / lo, 0)
    assert row_objective(x, u, xk, p, w, tau) < row_objective(x_lit, u, xk, p, w, tau) - 1e-8


@pytest.mark.parametrize("seed", range(10))
def test_one_good_closed_form(seed):
    """d = 1: s = u (a + b/s) with a = xk - tau p, b = tau w u, so
    s = (u a + sqrt(u^2 a^2 + 4 tau w u^2)) / 2 (cf. eq. update:t)."""
    rng = np.random.default_rng(200 + seed)
    u = np.array([rng.uniform(0.1, 1.0)])
    xk = np.array([rng.uniform(0, 0.1)])
    p = np.array([rng.uniform(0.1, 5.0)])
    w, tau = rng.uniform(0.5, 2.0), rng.uniform(1e-3, 1.0)
    a = xk[0] - tau * p[0]
    s_ref = (u[0] * a + np.sqrt((u[0] * a) ** 2 + 4 * tau * w * u[0] ** 2)) / 2
    x, s = oracle.row_prox_exact(u, xk, p, w, tau)
    assert s == pytest.approx(s_ref, rel=1e-13)
    assert x[0] == pytest.approx(s_ref / u[0], rel=1e-12)


@pytest.mark.parametrize("seed", range(20))
def test_bisection_and_ksection_match_exact(seed):
    rng = np.random.default_rng(300 + seed)
    d = int(rng.integers(1, 80))
    u, xk, p, w, tau = random_row(rng, d, negative_a=(seed % 2 == 0))
    x, s = oracle.row_prox_exact(u, xk, p, w, tau)
    xb, sb, _ = oracle.row_prox_bisect(u, xk, p, w, tau, eps=1e-14)
    xs, ss, _, L, U = oracle.row_prox_ksection(u, xk, p, w, tau, K=32, eps=1e-14)
    assert sb == pytest.approx(s, rel=1e-11)
    assert ss == pytest.approx(s, rel=1e-11)
    assert np.allclose(xb, x, rtol=1e-8, atol=1e-12)
    assert np.allclose(xs, x, rtol=1e-8, atol=1e-12)


@pytest.mark.parametrize("K", [2, 4, 8, 16, 32])
def test_ksection_bracket_and_shrink(K):
    """The bracket contains s* after every round (Sec. 2.2 bracketing), and
    each K-section round shrinks it at least (K+1)-fold: s* lies between two
    neighbouring candidates, which then bound it."""
    rng = np.random.default_rng(400 + K)
    for _ in range(20):
        d = int(rng.integers(2, 50))
        u, xk, p, w, tau = random_row(rng, d)
        _, s = oracle.row_prox_exact(u, xk, p, w, tau)
        _, _, _, L0, U0 = oracle.row_prox_ksection(u, xk, p, w, tau, K=K, max_rounds=0)
        assert L0 <= s * (1 + 1e-14) and s <= U0 * (1 + 1e-14)
        width = U0 - L0
        for r in range(1, 4):
            _, _, _, L, U = oracle.row_prox_ksection(u, xk, p, w, tau, K=K, max_rounds=r,
                                                     eps=0.0)
            assert L <= s * (1 + 1e-13) and s <= U * (1 + 1e-13)
            if width > 1e-9 * s:
                assert (U - L) <= width / (K + 1) * (1 + 1e-9) + 1e-15 * s
            width = U - L


def test_zero_trial_uses_positive_lower_bound():
    """x^k = 0 makes the Alg. 3 trial u^T x^k zero; the search still returns
    the exact prox."""
    rng = np.random.default_rng(9)
    u, _, p, w, tau = random_row(rng, 20)
    xk = np.zeros(20)
    x, s = oracle.row_prox_exact(u, xk, p, w, tau)
    xb, sb, _ = oracle.row_prox_bisect(u, xk, p, w, tau, eps=1e-14)
    assert sb == pytest.approx(s, rel=1e-11)
    assert np.allclose(xb, x, rtol=1e-8, atol=1e-14)


def test_zero_utility_entries_are_plain_projection():
    """An explicit zero utility leaves x_ij = [x^k_ij - tau p_j]_+."""
    u = np.array([1.0, 0.0, 0.5, 0.0])
    xk = np.array([0.1, 0.3, 0.0, 0.01])
    p = np.array([1.0, 2.0, 1.5, 0.5])
    x, s = oracle.row_prox_exact(u, xk, p, 1.0, 0.1)
    assert x[1] == pytest.approx(max(0.3 - 0.2, 0.0))
    assert x[3] == pytest.approx(0.0)
    assert s == pytest.approx(u @ x, rel=1e-14)
