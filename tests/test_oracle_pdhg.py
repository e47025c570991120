"""Pins of the oracle's restarted PDHG (Alg. 1 with the Sec. 5
enhancements), independent of its own formulas:

* one iteration: (p', y') maximises and (x', t') minimises the proximal
  subproblems of eq. update-rule, written out from the Lagrangian of eq.
  primal-dual-formulation and solved numerically by scipy;
* the relative KKT error of Sec. 5 Criteria for (x, t, p, y): reduces to
  the PDHCG form when t = Ux and y = w/t (the reduction the paper states),
  a hand-computed point, and zero at hand-worked equilibria;
* the solve: hand-worked equilibria (tests/golden), brute-force support
  enumeration, closed forms, sum(p) = sum(w), and the PDHCG oracle's
  prices (prices are unique, Sec. 3 Fact 1)."""
import json
import os

import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
from brute import dense_to_csr, equilibria_by_support
from paper_2506_06258_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def lagrangian(rp, col, u, w, x, t, p, y):
    """L(x, t; p, y) of eq. primal-dual-formulation on the stored pattern."""
    n, m = len(rp) - 1, len(p)
    rows = np.repeat(np.arange(n), np.diff(rp))
    c = np.bincount(col, weights=x, minlength=m)
    r = np.bincount(rows, weights=u * x, minlength=n)
    return -np.sum(w * np.log(t)) + p @ (c - 1.0) + y @ (t - r)


def random_state(rng, n, m, q=0.5):
    U = rng.uniform(0.05, 1.0, (n, m)) * (rng.random((n, m)) < q)
    for i in range(n):
        if not U[i].any():
            U[i, rng.integers(m)] = 0.5
    for j in range(m):
        if not U[:, j].any():
            U[rng.integers(n), j] = 0.5
    rp, col, u = dense_to_csr(U)
    nnz = len(col)
    w = rng.uniform(0.5, 1.5, n)
    x = rng.uniform(0.0, 0.5, nnz)
    xp = rng.uniform(0.0, 0.5, nnz)
    t = rng.uniform(0.2, 1.0, n)
    tp = rng.uniform(0.2, 1.0, n)
    p = rng.uniform(0.5, 2.0, m)
    y = rng.uniform(0.5, 2.0, n)
    return rp, col, u, w, x, xp, t, tp, p, y


@pytest.mark.parametrize("seed", range(4))
def test_pdhg_step_solves_the_proximal_subproblems(seed):
    rng = np.random.default_rng(seed)
    n, m = 5, 4
    rp, col, u, w, x, xp, t, tp, p, y = random_state(rng, n, m)
    tau, sigma = 0.3, 0.7
    rows = np.repeat(np.arange(n), np.diff(rp))
    c_prev = np.bincount(col, weights=xp, minlength=m)
    g_prev = tp - np.bincount(rows, weights=u * xp, minlength=n)
    x2, t2, p2, y2 = oracle.pdhg_step(n, m, rp, col, u, w, x, t, p, y, c_prev, g_prev, tau, sigma)

    # dual step: argmax over (p, y) of L(2x - x_prev, 2t - t_prev; p, y)
    # - (|y - y^k|^2 + |p - p^k|^2) / (2 sigma)
    xe, te = 2 * x - xp, 2 * t - tp

    def neg_dual(z):
        pp, yy = z[:m], z[m:]
        n_ = len(te)
        c = np.bincount(col, weights=xe, minlength=m)
        r = np.bincount(rows, weights=u * xe, minlength=n_)
        lin = pp @ (c - 1.0) + yy @ (te - r)  # the log term does not depend on (p, y)
        return -(lin - (np.sum((yy - y) ** 2) + np.sum((pp - p) ** 2)) / (2 * sigma))

    res = minimize(neg_dual, np.concatenate([p, y]), method="BFGS", options={"gtol": 1e-12})
    assert np.allclose(res.x[:m], p2, rtol=1e-7, atol=1e-8)
    assert np.allclose(res.x[m:], y2, rtol=1e-7, atol=1e-8)

    # primal step: argmin over x >= 0, t > 0 of L(x, t; p', y')
    # + (|x - x^k|^2 + |t - t^k|^2) / (2 tau)
    nnz = len(col)

    def prim(z):
        xx, tt = z[:nnz], z[nnz:]
        return (lagrangian(rp, col, u, w, xx, tt, p2, y2)
                + (np.sum((xx - x) ** 2) + np.sum((tt - t) ** 2)) / (2 * tau))

    bounds = [(0.0, None)] * nnz + [(1e-9, None)] * n
    res = minimize(prim, np.concatenate([np.maximum(x, 0.0), t]), method="L-BFGS-B",
                   bounds=bounds, options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 10000})
    assert np.allclose(res.x[:nnz], x2, atol=1e-6)
    assert np.allclose(res.x[nnz:], t2, rtol=1e-6, atol=1e-7)
    assert (x2 >= 0).all() and (t2 > 0).all()


def test_t_update_root_is_the_one_dimensional_minimiser():
    """eq. update:t on its own: a single buyer with no goods' influence,
    compared with a bounded scalar minimisation of
    -w log t + y t + (t - t0)^2 / (2 tau) over a range of y (both signs)."""
    from scipy.optimize import minimize_scalar
    rp, col, u = dense_to_csr([[1.0]])
    for y0 in (-3.0, -0.2, 0.0, 0.4, 5.0):
        for tau in (0.05, 1.0, 20.0):
            w, t0 = np.array([1.3]), np.array([0.7])
            # sigma = 0 keeps y' = y0 and p' = p
            _, t2, _, y2 = oracle.pdhg_step(1, 1, rp, col, u, w, np.array([0.5]), t0,
                                            np.array([1.0]), np.array([y0]), np.array([0.5]),
                                            np.array([0.2]), tau, 0.0)
            assert y2[0] == y0
            f = lambda s: -w[0] * np.log(s) + y0 * s + (s - t0[0]) ** 2 / (2 * tau)
            ref = minimize_scalar(f, bounds=(1e-12, 1e3), method="bounded",
                                  options={"xatol": 1e-13})
            assert t2[0] == pytest.approx(ref.x, rel=1e-7)


@pytest.mark.parametrize("seed", range(3))
def test_kkt_ty_reduces_to_the_pdhcg_form(seed):
    """Sec. 5 Criteria: for PDHCG, t = Ux and y = w/t."""
    rng = np.random.default_rng(100 + seed)
    rp, col, u, w, x, _, _, _, p, _ = random_state(rng, 6, 5)
    n, m = 6, 5
    rows = np.repeat(np.arange(n), np.diff(rp))
    t = np.bincount(rows, weights=u * x, minlength=n)
    a, pa = oracle.kkt(n, m, rp, col, u, w, x, p)
    b, pb = oracle.kkt_ty(n, m, rp, col, u, w, x, t, p, w / t)
    assert np.allclose(pa, pb, rtol=1e-13, atol=1e-15)


def test_kkt_ty_hand_example():
    """One buyer, two goods, u = (1, 0.5), w = 2; x = (0.5, 1.5) so the
    column sums are (0.5, 1.5) and Ux = 1.25; t = 1, y = 1.5, p = (1, 1).
      primal: max(|0.5-1|, |1.5-1|, |1-1.25|) = 0.5, over 1 + max(1.5, 0.25, 1)
              = 2.5  -> 0.2
      dual:   |w/t - y| = 0.5; M = (1.5, 0.75), p - M = (-0.5, 0.25): max
              (p - M)_- = 0.5; denominator 1 + max(2, 1.5, 0.25) = 3
              -> 1/6
      gap:    p - u y = (-0.5, 0.25); x (p - u y)_+ = (0, 0.375) -> 0.375
              over 1 + max(1.5, 0.25) = 2.5 -> 0.15"""
    rp, col, u = dense_to_csr([[1.0, 0.5]])
    r, parts = oracle.kkt_ty(1, 2, rp, col, u, np.array([2.0]), np.array([0.5, 1.5]),
                             np.array([1.0]), np.array([1.0, 1.0]), np.array([1.5]))
    assert parts == pytest.approx([0.2, 1.0 / 6.0, 0.15], rel=1e-14)
    assert r == pytest.approx(0.2, rel=1e-14)


def solve_dense(U, w, tol=1e-10, **kw):
    rp, col, u = dense_to_csr(U)
    n, m = np.asarray(U).shape
    return oracle.pdhg_solve(n, m, rp, col, u, np.asarray(w, float), tol=tol, max_iter=2000000,
                             **kw)


def rel_err(p, q):
    return np.max(np.abs(p - q)) / np.max(np.abs(q))


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "fisher_tiny.json")))["cases"],
                         ids=lambda c: c["name"])
def test_pdhg_golden_tiny_markets(case):
    sol = solve_dense(case["U"], case["w"])
    assert sol.status == oracle.OK
    assert rel_err(sol.p, np.array(case["p"], float)) < 1e-7


@pytest.mark.parametrize("seed", range(12))
def test_pdhg_random_tiny_markets_match_support_enumeration(seed):
    rng = np.random.default_rng(seed)
    n, m = int(rng.integers(1, 4)), int(rng.integers(1, 4))
    while True:
        U = rng.uniform(0.05, 1.0, (n, m)) * (rng.random((n, m)) < 0.75)
        if (U > 0).any(axis=1).all() and (U > 0).any(axis=0).all():
            break
    w = rng.uniform(0.2, 2.0, n)
    found = equilibria_by_support(U, w)
    assert len(found) == 1
    sol = solve_dense(U, w)
    assert sol.status == oracle.OK
    assert rel_err(sol.p, found[0]) < 1e-6


def test_pdhg_closed_forms():
    w = np.array([0.3, 1.2, 0.5, 2.0])
    s = solve_dense([[0.4], [1.0], [0.2], [0.7]], w)
    assert s.p[0] == pytest.approx(w.sum(), rel=1e-8)
    w5 = np.array([0.3, 1.2, 0.5, 2.0, 0.9])
    s = solve_dense(np.diag([0.5, 1.0, 0.2, 0.8, 0.3]), w5)
    assert rel_err(s.p, w5) < 1e-8
    a = np.array([1.0, 2.0, 0.5, 1.5])
    v = np.array([0.3, 0.9, 0.6])
    w4 = np.array([1.0, 2.0, 3.0, 0.5])
    s = solve_dense(np.outer(a, v), w4)
    assert rel_err(s.p, v * w4.sum() / v.sum()) < 1e-7


def test_pdhg_small_market_agrees_with_pdhcg():
    """The same unique prices as the PDHCG oracle (Sec. 3 Fact 1) on the
    1000 x 500 market, with sum(p) = sum(w) and the PDHCG-form KKT of the
    returned (x, p) small."""
    mk = synth.fisher_small(0).as_float32()
    u, w = mk.u.astype(np.float64), mk.w.astype(np.float64)
    a = oracle.pdhg_solve(mk.n, mk.m, mk.row_ptr, mk.col, u, w, tol=1e-9, max_iter=400000)
    b = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u, w, tol=1e-10, max_iter=400000)
    assert a.status == oracle.OK and b.status == oracle.OK
    assert rel_err(a.p, b.p) < 1e-7
    assert abs(a.p.sum() - w.sum()) / w.sum() < 1e-7
    uh, _ = oracle.normalize_rows(mk.row_ptr, u)
    r, _ = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, w, a.x, a.p)
    assert r < 1e-7
    # more iterations than PDHCG on the same market (the motivation of Sec. 2.2)
    assert a.iters > b.iters
