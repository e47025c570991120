"""Pins of the oracle's Alg. 2 in the setting of its analysis (Sec. 3:
fixed sigma = tau = eta, fixed restart length K, restarts to the average;
oracle.fixed_restart):

* its restart points are those of chained runs of the oracle's main solver
  (a separately written loop) with the same fixed step, no adaptive
  restarts and primal weight one, each warm-started from the previous
  average: the inner loop, the average and the restart bookkeeping;
* the starting distance has its closed form (p0 = sum(w)/m);
* with K long enough the distance to p* contracts at every restart and the
  restart points converge to the hand-worked equilibria (Theorem 1)."""
import json
import os

import numpy as np
import pytest

import oracle
from brute import dense_to_csr
from paper_2506_06258_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_restart_points_match_chained_solver_runs():
    mk = synth.bernoulli_market(200, 80, 0.1, 7, w_mode="uniform")
    u, w = mk.u.astype(np.float64), mk.w.astype(np.float64)
    deg = np.bincount(mk.col, minlength=mk.m)
    eta = 1.0 / (2.0 * np.sqrt(deg.max()))
    K, R = 24, 3
    st, p, x, _, kk = oracle.fixed_restart(mk.n, mk.m, mk.row_ptr, mk.col, u, w, K, R)
    assert st == oracle.OK
    common = dict(tol=0.0, max_iter=K, eval_every=10**6, step_mode=0, restart=0, eta0=eta,
                  omega0=1.0, output=2)
    s = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u, w, **common)
    for _ in range(R - 1):
        s = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u, w, p0=s.p, x0=s.x, **common)
    assert np.allclose(s.p, p, rtol=1e-12, atol=1e-14)
    assert np.allclose(s.x, x, rtol=1e-12, atol=1e-14)
    assert kk[-1] == pytest.approx(s.rel_kkt, rel=1e-10)


def test_starting_distance_closed_form():
    mk = synth.bernoulli_market(50, 20, 0.3, 8, w_mode="uniform")
    u, w = mk.u.astype(np.float64), mk.w.astype(np.float64)
    ref = np.linspace(0.5, 1.5, mk.m)
    st, _, _, d, _ = oracle.fixed_restart(mk.n, mk.m, mk.row_ptr, mk.col, u, w, 4, 0, p_ref=ref)
    assert st == oracle.OK
    assert d[0] == pytest.approx(np.linalg.norm(w.sum() / mk.m - ref), rel=1e-14)


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLDEN, "fisher_tiny.json")))["cases"],
                         ids=lambda c: c["name"])
def test_contracts_to_golden_equilibria(case):
    rp, col, u = dense_to_csr(case["U"])
    n, m = np.asarray(case["U"]).shape
    p_star = np.array(case["p"], float)
    st, p, _, d, _ = oracle.fixed_restart(n, m, rp, col, u, np.array(case["w"], float), 200, 40,
                                          p_ref=p_star)
    assert st == oracle.OK
    scale = max(d[0], np.max(p_star))  # d[0] is 0 when p0 = sum(w)/m is p*
    assert d[-1] <= 1e-6 * scale
    assert np.all(np.diff(d[1:]) <= 1e-12 * scale)
