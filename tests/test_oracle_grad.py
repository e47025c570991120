"""Pins of the oracle's implicit derivatives of equilibrium prices
(``oracle.implicit_grad``) against what fixes them independently:

* closed forms: one good (p = sum w), a diagonal market (p_j = w_j) and a
  two-buyer market whose second buyer splits spending over both goods
  (p_1 / p_2 = u_21 / u_22 and p_1 + p_2 = w_1 + w_2);
* central finite differences of exact equilibria found by support
  enumeration (tests/brute.py) on random 3 x 3 markets;
* central finite differences of tightly solved oracle equilibria on a
  6 x 5 market, for active and inactive utilities and for budgets.
A degenerate support (a cycle of bought goods, so x is not unique) must be
reported as singular, not given a gradient.

The reverse-mode oracle through the unrolled fixed-step iteration
(``oracle.unrolled_grad``) is pinned by central finite differences of the
unrolled map itself (start point held fixed, away from equilibrium) and by
its limit: started at an equilibrium it tends to the implicit derivative.
"""
import numpy as np
import pytest

import oracle
from brute import dense_to_csr, equilibria_by_support


def _grad(U, w, g, x=None, p=None, tol=1e-13):
    rp, col, u = dense_to_csr(U)
    n, m = U.shape
    if x is None:
        s = oracle.solve(n, m, rp, col, u, w, tol=tol, max_iter=2000000)
        assert s.status == oracle.OK
        x, p = s.x, s.p
    st, du, dw, dim = oracle.implicit_grad(n, m, rp, col, u, w, x, p, g)
    return st, du, dw, (rp, col, u), x, p


def test_single_good():
    U = np.array([[0.3], [2.0], [0.7]])
    w = np.array([1.0, 2.0, 0.5])
    g = np.array([1.7])
    st, du, dw, _, _, _ = _grad(U, w, g)
    assert st == oracle.OK
    np.testing.assert_allclose(dw, g[0] * np.ones(3), rtol=1e-9)
    np.testing.assert_allclose(du, 0.0, atol=1e-9)


def test_diagonal():
    U = np.diag([0.5, 1.5, 3.0])
    w = np.array([1.0, 2.0, 3.0])
    g = np.array([0.3, -1.0, 2.0])
    st, du, dw, _, _, _ = _grad(U, w, g)
    assert st == oracle.OK
    np.testing.assert_allclose(dw, g, rtol=1e-9)
    np.testing.assert_allclose(du, 0.0, atol=1e-9)


def test_two_by_two_closed_form():
    # buyer 1 wants only good 1; buyer 2 values both and buys both:
    # p1/p2 = u21/u22, p1 + p2 = w1 + w2
    u11, u21, u22 = 1.0, 1.0, 1.6
    w = np.array([1.0, 3.0])
    U = np.array([[u11, 0.0], [u21, u22]])
    S = w.sum()
    p = S * np.array([u21, u22]) / (u21 + u22)
    x = np.array([w[0] / p[0], 1.0 - w[0] / p[0], 1.0])  # CSR order (0,0),(1,0),(1,1)
    assert np.all(x > 0)
    g = np.array([0.8, -0.4])
    st, du, dw, _, _, _ = _grad(U, w, g, x=x, p=p)
    assert st == oracle.OK
    d = (u21 + u22) ** 2
    dp_du21 = S * np.array([u22, -u22]) / d
    dp_du22 = S * np.array([-u21, u21]) / d
    dp_dw = np.array([u21, u22]) / (u21 + u22)
    np.testing.assert_allclose(du, [0.0, g @ dp_du21, g @ dp_du22], atol=1e-12)
    np.testing.assert_allclose(dw, [g @ dp_dw, g @ dp_dw], rtol=1e-12)


def _exact_price(U, w):
    found = equilibria_by_support(U, w)
    assert len(found) == 1
    return found[0]


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4, 5])
def test_finite_differences_of_exact_equilibria(seed):
    rng = np.random.default_rng(100 + seed)
    U = rng.uniform(0.1, 1.0, (3, 3))
    w = rng.uniform(0.5, 1.5, 3)
    g = rng.normal(size=3)
    st, du, dw, (rp, col, u), x, p = _grad(U, w, g)
    if st != oracle.OK:
        pytest.skip("degenerate support for this seed")
    np.testing.assert_allclose(p, _exact_price(U, w), rtol=1e-8)
    h = 1e-6
    rows = np.repeat(np.arange(3), np.diff(rp))
    for q in range(len(u)):
        Up, Um = U.copy(), U.copy()
        Up[rows[q], col[q]] += h
        Um[rows[q], col[q]] -= h
        fd = g @ (_exact_price(Up, w) - _exact_price(Um, w)) / (2 * h)
        assert abs(fd - du[q]) <= 1e-6 * (1 + abs(fd)), (q, fd, du[q])
    for i in range(3):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = g @ (_exact_price(U, wp) - _exact_price(U, wm)) / (2 * h)
        assert abs(fd - dw[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, dw[i])


def test_finite_differences_of_oracle_solves():
    rng = np.random.default_rng(7)
    n, m = 6, 5
    U = rng.uniform(0.05, 1.0, (n, m)) * (rng.uniform(size=(n, m)) < 0.7)
    for i in range(n):
        if not U[i].any():
            U[i, rng.integers(m)] = 0.5
    for j in range(m):
        if not U[:, j].any():
            U[rng.integers(n), j] = 0.5
    w = rng.uniform(0.5, 1.5, n)
    g = rng.normal(size=m)
    st, du, dw, (rp, col, u), x, p = _grad(U, w, g)
    assert st == oracle.OK
    active = x > 1e-9
    assert active.any() and (~active).any()  # both kinds of entries are checked
    rows = np.repeat(np.arange(n), np.diff(rp))

    def price(Ux, wx):
        rpx, cx, ux = dense_to_csr(Ux)
        s = oracle.solve(n, m, rpx, cx, ux, wx, tol=1e-14, max_iter=4000000)
        assert s.status == oracle.OK
        return s.p

    h = 1e-5
    for q in range(len(u)):
        Up, Um = U.copy(), U.copy()
        Up[rows[q], col[q]] += h
        Um[rows[q], col[q]] -= h
        fd = g @ (price(Up, w) - price(Um, w)) / (2 * h)
        assert abs(fd - du[q]) <= 1e-5 * (1 + abs(fd)), (q, bool(active[q]), fd, du[q])
    for i in range(n):
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = g @ (price(U, wp) - price(U, wm)) / (2 * h)
        assert abs(fd - dw[i]) <= 1e-5 * (1 + abs(fd)), (i, fd, dw[i])


def test_degenerate_support_is_singular():
    # two identical buyers and two goods valued equally: any split of the
    # goods is an equilibrium allocation, the support has a cycle
    U = np.ones((2, 2))
    w = np.ones(2)
    x = np.full(4, 0.5)
    p = np.ones(2)
    st, _, _, _, _, _ = _grad(U, w, np.array([1.0, 0.0]), x=x, p=p)
    assert st == oracle.ERR_NUMERIC


def test_prices_sum_gradient_is_budget_sum():
    # sum_j p_j = sum_i w_i at every equilibrium (Sec. 3): the gradient of
    # sum p is one per budget and zero per utility
    rng = np.random.default_rng(11)
    U = rng.uniform(0.1, 1.0, (5, 4))
    w = rng.uniform(0.5, 1.5, 5)
    st, du, dw, _, _, _ = _grad(U, w, np.ones(4))
    assert st == oracle.OK
    np.testing.assert_allclose(dw, 1.0, rtol=1e-9)
    np.testing.assert_allclose(du, 0.0, atol=1e-9)


# ---------------------------------------------------------------------------
# Reverse mode through the unrolled fixed-step iteration (oracle.unrolled_grad)


def _market(seed, n, m, q):
    rng = np.random.default_rng(seed)
    U = rng.uniform(0.05, 1.0, (n, m)) * (rng.uniform(size=(n, m)) < q)
    for i in range(n):
        if not U[i].any():
            U[i, rng.integers(m)] = 0.5
    for j in range(m):
        if not U[:, j].any():
            U[rng.integers(n), j] = 0.5
    w = rng.uniform(0.5, 1.5, n)
    return U, w, rng


def _steps(rp, col, m, omega):
    deg = np.bincount(col, minlength=m)
    eta = 0.9 / np.sqrt(deg.max())
    return eta / omega, eta * omega


def test_unrolled_grad_matches_finite_differences_of_the_unrolled_map():
    # reverse mode must equal the derivative of p_K(u, w) with the start
    # point held fixed, for any K (here a start away from equilibrium)
    U, w, rng = _market(21, 7, 5, 0.6)
    rp, col, u = dense_to_csr(U)
    n, m = U.shape
    x0 = rng.uniform(0.05, 0.3, len(u))
    p0 = rng.uniform(0.5, 1.5, m)
    tau, sigma = _steps(rp, col, m, 0.7)
    g = rng.normal(size=m)
    K = 6
    st, du, dw, pK = oracle.unrolled_grad(n, m, rp, col, u, w, x0, p0, tau, sigma, K, g)
    assert st == oracle.OK

    def loss(uu, ww):
        _, _, _, p = oracle.unrolled_grad(n, m, rp, col, uu, ww, x0, p0, tau, sigma, K,
                                          np.zeros(m))
        return g @ p

    h = 1e-6
    for q in range(len(u)):
        e = np.zeros(len(u))
        e[q] = h
        fd = (loss(u + e, w) - loss(u - e, w)) / (2 * h)
        assert abs(fd - du[q]) <= 1e-6 * (1 + abs(fd)), (q, fd, du[q])
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        fd = (loss(u, w + e) - loss(u, w - e)) / (2 * h)
        assert abs(fd - dw[i]) <= 1e-6 * (1 + abs(fd)), (i, fd, dw[i])


def test_unrolled_grad_tends_to_implicit_grad():
    U, w, rng = _market(3, 30, 10, 0.5)
    rp, col, u = dense_to_csr(U)
    n, m = U.shape
    s = oracle.solve(n, m, rp, col, u, w, tol=1e-13, max_iter=2000000)
    assert s.status == oracle.OK
    g = rng.normal(size=m)
    st, du_i, dw_i, _ = oracle.implicit_grad(n, m, rp, col, u, w, s.x, s.p, g)
    assert st == oracle.OK
    tau, sigma = _steps(rp, col, m, s.omega)
    errs = []
    for K in (50, 2000):
        st, du, dw, pK = oracle.unrolled_grad(n, m, rp, col, u, w, s.x, s.p, tau, sigma, K, g)
        assert st == oracle.OK
        np.testing.assert_allclose(pK, s.p, rtol=1e-9)  # the start is a fixed point
        errs.append(max(np.max(np.abs(du - du_i)) / np.max(np.abs(du_i)),
                        np.max(np.abs(dw - dw_i)) / np.max(np.abs(dw_i))))
    assert errs[1] <= 1e-9 and errs[1] < errs[0]
