"""Independent references used to pin the oracle (tests only).

* ``equilibria_by_support`` - linear Fisher equilibrium prices of a tiny
  market by enumerating every candidate maximum-bang-per-buck (MBB) graph:
  on a graph G the conditions p_j = u_ij * beta_i for (i, j) in G fix the
  prices of each connected component up to scale; money conservation inside
  the component fixes the scale; the candidate is an equilibrium when every
  stored edge satisfies u_ij * beta_i <= p_j (MBB) and some spending b >= 0
  on G has row sums w and column sums p (a transportation feasibility LP).
  These are the equilibrium conditions of the PDHCG KKT system (Sec. 3,
  eq. KKT-system-pdhcg) written with spending b_ij = p_j x_ij.
* ``proportional_response`` - proportional-response dynamics for linear
  Fisher markets (bids b_ij <- w_i u_ij x_ij / u_i^T x_i, p_j = sum_i b_ij,
  x_ij = b_ij / p_j), a different algorithm with the same fixed point.
* ``eg_duality_gap`` - the Lagrangian duality gap of the Eisenberg-Gale
  program at (x, p): with alpha_i = max_j u_ij/p_j,
  g(p) = sum_j p_j + sum_i w_i (log w_i + log alpha_i - 1) bounds every
  feasible objective sum_i w_i log(u_i^T x_i) from above.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.optimize import linprog


def _components(n, m, edges):
    parent = list(range(n + m))

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, j in edges:
        ra, rb = find(i), find(n + j)
        if ra != rb:
            parent[ra] = rb
    comp = {}
    for v in range(n + m):
        comp.setdefault(find(v), []).append(v)
    return list(comp.values())


def equilibria_by_support(U: np.ndarray, w: np.ndarray, rtol: float = 1e-9):
    """All distinct equilibrium price vectors found by support enumeration."""
    U = np.asarray(U, dtype=float)
    w = np.asarray(w, dtype=float)
    n, m = U.shape
    edges = [(i, j) for i in range(n) for j in range(m) if U[i, j] > 0]
    found = []
    for r in range(1, len(edges) + 1):
        for G in itertools.combinations(edges, r):
            if {i for i, _ in G} != set(range(n)) or {j for _, j in G} != set(range(m)):
                continue
            p = np.zeros(m)
            beta = np.zeros(n)
            ok = True
            for comp in _components(n, m, G):
                buyers = [v for v in comp if v < n]
                goods = [v - n for v in comp if v >= n]
                cedges = [(i, j) for (i, j) in G if i in buyers]
                # propagate p_j = u_ij beta_i from beta_root = 1
                beta_c = {buyers[0]: 1.0}
                p_c = {}
                frontier = [buyers[0]]
                while frontier and ok:
                    nxt = []
                    for v in frontier:
                        for (i, j) in cedges:
                            if i == v and j not in p_c:
                                p_c[j] = U[i, j] * beta_c[i]
                                for (i2, j2) in cedges:
                                    if j2 == j and i2 not in beta_c:
                                        beta_c[i2] = p_c[j] / U[i2, j]
                                        nxt.append(i2)
                    frontier = nxt
                if len(beta_c) != len(buyers) or len(p_c) != len(goods):
                    ok = False
                    break
                for (i, j) in cedges:
                    if abs(p_c[j] - U[i, j] * beta_c[i]) > rtol * p_c[j]:
                        ok = False
                        break
                if not ok:
                    break
                scale = w[buyers].sum() / sum(p_c.values())
                for j, v in p_c.items():
                    p[j] = v * scale
                for i, v in beta_c.items():
                    beta[i] = v * scale
            if not ok:
                continue
            # MBB on every stored edge: u_ij beta_i <= p_j
            if any(U[i, j] * beta[i] > p[j] * (1 + 1e-9) for (i, j) in edges):
                continue
            # spending b >= 0 on G with row sums w and column sums p
            k = len(G)
            A = np.zeros((n + m, k))
            for e, (i, j) in enumerate(G):
                A[i, e] = 1.0
                A[n + j, e] = 1.0
            res = linprog(np.zeros(k), A_eq=A, b_eq=np.concatenate([w, p]),
                          bounds=[(0, None)] * k, method="highs")
            if res.status != 0:
                continue
            if not any(np.allclose(p, q, rtol=1e-9, atol=1e-12) for q in found):
                found.append(p.copy())
    return found


def proportional_response(U_csr, w, iters=20000):
    """Proportional-response dynamics on a CSR market; returns prices."""
    row_ptr, col, u = U_csr
    n = len(row_ptr) - 1
    m = int(col.max()) + 1
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    deg = np.diff(row_ptr)
    b = (np.asarray(w, float) / deg)[rows]  # equal split of each budget
    for _ in range(iters):
        p = np.bincount(col, weights=b, minlength=m)
        x = b / p[col]
        ux = u * x
        t = np.bincount(rows, weights=ux, minlength=n)
        b = np.asarray(w, float)[rows] * ux / t[rows]
    return np.bincount(col, weights=b, minlength=m)


def eg_duality_gap(row_ptr, col, u, w, x, p):
    """g(p) - sum_i w_i log(u_i^T xt_i) with xt the feasible scaling of x."""
    row_ptr = np.asarray(row_ptr)
    n = len(row_ptr) - 1
    m = len(p)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    c = np.bincount(col, weights=x, minlength=m)
    xt = x / np.maximum(1.0, c)[col]
    t = np.bincount(rows, weights=u * xt, minlength=n)
    alpha = np.full(n, -np.inf)
    np.maximum.at(alpha, rows, u / p[col])
    g = p.sum() + np.sum(w * (np.log(w) + np.log(alpha) - 1.0))
    return g - np.sum(w * np.log(t))


def dense_to_csr(U):
    U = np.asarray(U, float)
    rows, cols = np.nonzero(U)
    n = U.shape[0]
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return row_ptr, cols.astype(np.int32), U[rows, cols]
