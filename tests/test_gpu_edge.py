"""Degenerate and boundary cases of the GPU path, through the C ABI, against
equilibria known in closed form (Sec. 3: prices are unique, and for these
markets the equilibrium conditions pin them down by hand):

* one buyer: it must buy every good and spend only on goods of maximal
  u_j / p_j, so p_j = w u_j / sum_k u_k;
* one good: it costs sum_i w_i and buyer i gets w_i / sum(w);
* diagonal U (each buyer values only its own good): p_j = w_j;
* rank-one dense U = a v^T: every buyer has the same bang per buck, so
  p = v sum(w) / sum(v) (rows of 500 entries: the wide register shapes);
and the size limits of market creation.  The same closed forms are checked
for the batched solver.  The bar: relative price error <= 1e-5 at relative
KKT <= 1e-6, the solver's accuracy target (float32 iterates put a floor of a
few 1e-8 under the KKT error of these markets, so tighter tolerances are
not reachable on the device).
"""
import numpy as np
import pytest
import torch

from paper_2506_06258_amd import pdhcg, synth

pytestmark = pytest.mark.gpu


def _dense(U, w):
    U = np.asarray(U, dtype=np.float64)
    rows, cols = np.nonzero(U)
    row_ptr = np.zeros(U.shape[0] + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=U.shape[0]), out=row_ptr[1:])
    return synth.Market(U.shape[0], U.shape[1], row_ptr.astype(np.int32), cols.astype(np.int32),
                        U[rows, cols].astype(np.float32), np.asarray(w, np.float32), "dense")


def _cases():
    rng = np.random.default_rng(3)
    u1 = rng.uniform(0.05, 1.0, 37)
    yield "one buyer", _dense(u1[None, :], [1.7]), 1.7 * u1.astype(np.float32) / u1.astype(np.float32).sum()
    w2 = rng.uniform(0.5, 1.5, 50)
    yield "one good", _dense(rng.uniform(0.1, 1.0, (50, 1)), w2), np.array([w2.astype(np.float32).sum()])
    yield "one buyer, one good", _dense([[0.3]], [2.5]), np.array([2.5])
    w3 = rng.uniform(0.5, 1.5, 40)
    yield "diagonal", _dense(np.diag(rng.uniform(0.1, 1.0, 40)), w3), w3.astype(np.float32)
    a, v = rng.uniform(0.2, 1.0, 2000), rng.uniform(0.1, 1.0, 500)
    w4 = rng.uniform(0.5, 1.5, 2000)
    v32 = v.astype(np.float32).astype(np.float64)
    # u = a v^T rounded to float32 is rank one only up to rounding; the
    # normalised rows u / max_j u are v / max v to float32 rounding
    yield "rank one", _dense(np.outer(a, v), w4), v32 * w4.astype(np.float32).sum() / v32.sum()


CASES = list(_cases())


def _rel(a, b):
    return float(np.max(np.abs(np.asarray(a, np.float64) - b)) / np.max(np.abs(b)))


@pytest.mark.parametrize("name,mk,p_star", CASES, ids=[c[0] for c in CASES])
def test_closed_form_equilibria(cuda, name, mk, p_star):
    M = pdhcg.Market.from_synth(mk, device=cuda)
    sol = M.solve(tol=1e-6, max_iter=100000)
    assert sol.info.status == pdhcg.PDHCG_OK, (name, pdhcg.pdhcg_last_error())
    p = sol.p.double().cpu().numpy()
    assert _rel(p, p_star) <= 1e-5, (name, _rel(p, p_star))
    # every good is sold (column sums of x are one)
    x = sol.x.double().cpu().numpy()
    c = np.bincount(mk.col, weights=x, minlength=mk.m)
    assert np.max(np.abs(c - 1.0)) <= 1e-5, name
    M.close()


def test_closed_forms_in_one_batch(cuda):
    bt = synth.batch_from_markets([mk for _, mk, _ in CASES])
    B = pdhcg.Batch(bt, device=cuda)
    st, p, _, infos = B.solve(tol=1e-6, max_iter=100000)
    assert st == pdhcg.PDHCG_OK, [i.status for i in infos]
    p = p.double().cpu().numpy()
    for b, (name, _, p_star) in enumerate(CASES):
        pb = p[B.good_off[b]:B.good_off[b + 1]]
        assert _rel(pb, p_star) <= 1e-5, (name, _rel(pb, p_star))
    B.close()


def test_creation_limits(cuda):
    rp = torch.tensor([0, 1], dtype=torch.int32, device=cuda)
    col = torch.zeros(1, dtype=torch.int32, device=cuda)
    u = torch.ones(1, device=cuda)
    w = torch.ones(1, device=cuda)
    # more stored entries than 32-bit buffer offsets address: rejected before
    # any array is read
    with pytest.raises(pdhcg.PDHCGError) as e:
        pdhcg.pdhcg_market_create(1, 1, (1 << 29) + 1, rp, col, u, w)
    assert e.value.status == pdhcg.PDHCG_ERR_UNSUPPORTED
    for n, m, nnz in ((0, 1, 1), (1, 0, 1), (1, 1, 0), (1, 1, -5)):
        with pytest.raises(pdhcg.PDHCGError) as e:
            pdhcg.pdhcg_market_create(n, m, nnz, rp, col, u, w)
        assert e.value.status == pdhcg.PDHCG_ERR_ARG, (n, m, nnz)
    # the smallest market works
    M = pdhcg.Market(rp, col, u, w, m=1, device=cuda)
    s = M.solve(tol=1e-6)
    assert s.info.status == pdhcg.PDHCG_OK and abs(float(s.p[0]) - 1.0) <= 1e-6
    M.close()
