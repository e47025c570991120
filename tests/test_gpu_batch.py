"""Batched persistent solve (many markets in one launch) against the FP64
oracle, market by market, through the C ABI.

Each market is solved independently on the device, so its prices must match
the oracle's unique equilibrium prices (Sec. 3 Fact 1) to relative error
1e-5.  The markets of a batch are not all well conditioned (some have far
more goods than buyers, where KKT 1e-6 still leaves price errors of a few
1e-5 in the oracle itself), so the batch is solved to relative KKT 1e-7,
which the oracle shows is enough for 1e-5 on every market here.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_06258_amd import pdhcg, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small_batch():
    # sizes span every row shape of the batched kernel; the last market has
    # rows longer than 512 entries (whole-wave path)
    bt = synth.batch_markets(24, 11, n_range=(16, 1200), m_range=(4, 1100),
                             q_range=(0.05, 0.6))
    markets = [bt.market(b) for b in range(bt.count)]
    markets.append(synth.bernoulli_market(40, 1100, 0.55, 5, w_mode="uniform",
                                          dtype=np.float32))
    return synth.batch_from_markets(markets)


def test_batch_matches_oracle_per_market(cuda, small_batch):
    B = pdhcg.Batch(small_batch, device=cuda)
    st, p, x, infos = B.solve(tol=1e-7, max_iter=200000)
    assert st == pdhcg.PDHCG_OK, [i.status for i in infos]
    p = p.double().cpu().numpy()
    x = x.double().cpu().numpy()
    for b in range(small_batch.count):
        mk = small_batch.market(b)
        ref = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, mk.u.astype(np.float64),
                           mk.w.astype(np.float64), tol=1e-11, max_iter=400000)
        pb = p[B.good_off[b]:B.good_off[b + 1]]
        xb = x[B.edge_off[b]:B.edge_off[b + 1]]
        assert infos[b].status == pdhcg.PDHCG_OK and infos[b].rel_kkt <= 1e-7, b
        err = np.max(np.abs(pb - ref.p)) / np.max(ref.p)
        assert err <= 1e-5, (b, mk.n, mk.m, err)
        uh, _ = oracle.normalize_rows(mk.row_ptr, mk.u.astype(np.float64))
        r, _ = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, xb, pb)
        assert r <= 1e-6, (b, r)
    B.close()


def test_batch_agrees_with_single_market_solver(cuda, small_batch):
    """The same market through pdhcg_solve and through the batch reach the
    same prices."""
    B = pdhcg.Batch(small_batch, device=cuda)
    st, p, _, _ = B.solve(tol=1e-7, max_iter=200000)
    p = p.cpu().numpy()
    for b in (0, 7, 24):
        mk = small_batch.market(b)
        M = pdhcg.Market.from_synth(mk, device=cuda)
        s = M.solve(tol=1e-7, max_iter=200000)
        q = s.p.cpu().numpy()
        pb = p[B.good_off[b]:B.good_off[b + 1]]
        assert np.max(np.abs(pb - q)) / np.max(q) <= 2e-5
        M.close()
    B.close()


def test_batch_max_iter_and_rejects_oversized(cuda):
    bt = synth.batch_markets(6, 2, n_range=(20, 60), m_range=(5, 30))
    B = pdhcg.Batch(bt, device=cuda)
    st, _, _, infos = B.solve(tol=1e-14, max_iter=10)
    assert st == pdhcg.PDHCG_MAX_ITER
    assert all(i.iters == 10 and i.status == pdhcg.PDHCG_MAX_ITER for i in infos)
    B.close()
    big = synth.batch_markets(1, 3, n_range=(50, 50), m_range=(3000, 3000), q_range=(0.01, 0.01))
    with pytest.raises(pdhcg.PDHCGError) as e:
        pdhcg.Batch(big, device=cuda)
    assert e.value.status == pdhcg.PDHCG_ERR_UNSUPPORTED
