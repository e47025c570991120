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


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_graph_replays_match_eager_launch(cuda, monkeypatch, small_batch):
    """The solve runs as a replayed HIP graph; each replay, with eager device
    work and synchronisations in between, reaches the prices of a directly
    launched solve (column sums are float64 LDS atomics in no fixed order,
    so runs agree to the solve tolerance, not bit for bit)."""
    B = pdhcg.Batch(small_batch, device=cuda)
    monkeypatch.setenv("PDHCG_BATCH_EAGER", "1")
    st, p_e, _, _ = B.solve(tol=1e-7, max_iter=200000)
    assert st == pdhcg.PDHCG_OK
    p_e = p_e.double().cpu().numpy()
    monkeypatch.delenv("PDHCG_BATCH_EAGER")
    for rep in range(3):
        junk = torch.randn(1 << 20, device=cuda)
        (junk * 2.0).sum().item()
        torch.cuda.synchronize()
        st, p_g, _, infos = B.solve(tol=1e-7, max_iter=200000)
        assert st == pdhcg.PDHCG_OK, rep
        assert all(i.rel_kkt <= 1e-7 for i in infos)
        for b in range(small_batch.count):
            sl = slice(B.good_off[b], B.good_off[b + 1])
            assert _rel(p_g.double().cpu().numpy()[sl], p_e[sl]) <= 2e-5, (rep, b)
        # per-market times are reported and bounded by the launch
        assert all(0.0 < i.seconds <= i.row_pass_seconds * 1.01 + 1e-3 for i in infos)
    B.close()


def test_autotune_keeps_results(cuda, small_batch):
    B = pdhcg.Batch(small_batch, device=cuda)
    sch = B.autotune(trial_iters=32)
    assert sch.trials >= 2 and sch.wg_per_cu >= 1 and sch.shape_policy in (0, 1)
    assert sch.best_trial_seconds > 0.0
    st, p, _, infos = B.solve(tol=1e-7, max_iter=200000)
    assert st == pdhcg.PDHCG_OK
    p = p.double().cpu().numpy()
    for b in (0, 5, 11, 24):
        mk = small_batch.market(b)
        ref = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, mk.u.astype(np.float64),
                           mk.w.astype(np.float64), tol=1e-11, max_iter=400000)
        assert _rel(p[B.good_off[b]:B.good_off[b + 1]], ref.p) <= 1e-5, b
    with pytest.raises(pdhcg.PDHCGError) as e:
        B.autotune(trial_iters=0)
    assert e.value.status == pdhcg.PDHCG_ERR_ARG
    B.close()


def test_rows_beyond_register_capacity(cuda):
    """Rows of 513-1024 entries take the 64x16 register shape, longer rows
    the whole-wave path: both against the single-market solver and the
    oracle's KKT of the batch output."""
    markets = [synth.bernoulli_market(40, 1100, 0.55, 5, w_mode="uniform", dtype=np.float32),
               synth.bernoulli_market(24, 2000, 0.6, 9, w_mode="uniform", dtype=np.float32),
               synth.bernoulli_market(300, 200, 0.2, 4, w_mode="uniform", dtype=np.float32)]
    dmax = [int(np.diff(mk.row_ptr).max()) for mk in markets]
    assert 512 < dmax[0] <= 1024 and dmax[1] > 1024
    bt = synth.batch_from_markets(markets)
    B = pdhcg.Batch(bt, device=cuda)
    st, p, x, infos = B.solve(tol=1e-7, max_iter=400000)
    assert st == pdhcg.PDHCG_OK, [i.status for i in infos]
    p, x = p.double().cpu().numpy(), x.double().cpu().numpy()
    for b, mk in enumerate(markets):
        pb = p[B.good_off[b]:B.good_off[b + 1]]
        xb = x[B.edge_off[b]:B.edge_off[b + 1]]
        uh, _ = oracle.normalize_rows(mk.row_ptr, mk.u.astype(np.float64))
        r, _ = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, xb, pb)
        assert r <= 1e-6, (b, r)
        M = pdhcg.Market.from_synth(mk, device=cuda)
        q = M.solve(tol=1e-7, max_iter=400000).p.double().cpu().numpy()
        M.close()
        assert _rel(pb, q) <= 2e-5, b
    B.close()


def _lopsided_market():
    """Row 0 holds 1000 of 1003 entries: split over four workgroups by
    entries, two members own no rows."""
    rng = np.random.default_rng(21)
    m = 1000
    cols = [np.arange(m, dtype=np.int32), np.array([3], np.int32), np.array([500], np.int32),
            np.array([999], np.int32)]
    row_ptr = np.zeros(5, np.int32)
    row_ptr[1:] = np.cumsum([len(c) for c in cols])
    col = np.concatenate(cols)
    u = rng.uniform(0.01, 1.0, len(col)).astype(np.float32)
    w = rng.uniform(0.5, 1.5, 4).astype(np.float32)
    return synth.Market(4, m, row_ptr, col, u, w, "lopsided")


@pytest.mark.parametrize("mode", ["2", "3", "auto"])
def test_gangs_match_single_workgroup_markets(cuda, monkeypatch, small_batch, mode):
    """Markets split over gangs of workgroups (one meeting per iteration,
    column partials summed in member order) reach the prices of the same
    markets solved by one workgroup each, and the oracle's KKT of their
    allocations; a market whose rows cannot be split evenly (members with
    no rows) too."""
    markets = [small_batch.market(b) for b in range(small_batch.count)] + [_lopsided_market()]
    bt = synth.batch_from_markets(markets)
    monkeypatch.setenv("PDHCG_BATCH_GANG", "0")
    B0 = pdhcg.Batch(bt, device=cuda)
    if mode == "auto":
        monkeypatch.delenv("PDHCG_BATCH_GANG")
    else:
        monkeypatch.setenv("PDHCG_BATCH_GANG", mode)
    B1 = pdhcg.Batch(bt, device=cuda)
    monkeypatch.delenv("PDHCG_BATCH_GANG", raising=False)
    st0, p0, _, i0 = B0.solve(tol=1e-7, max_iter=200000)
    st1, p1, x1, i1 = B1.solve(tol=1e-7, max_iter=200000)
    assert st0 == pdhcg.PDHCG_OK and st1 == pdhcg.PDHCG_OK, [i.status for i in i1]
    p0, p1, x1 = (t.double().cpu().numpy() for t in (p0, p1, x1))
    for b, mk in enumerate(markets):
        sl = slice(B1.good_off[b], B1.good_off[b + 1])
        assert i1[b].rel_kkt <= 1e-7 and i1[b].iters > 0, b
        assert _rel(p1[sl], p0[sl]) <= 2e-5, (b, mk.n, mk.m)
        xb = x1[B1.edge_off[b]:B1.edge_off[b + 1]]
        uh, _ = oracle.normalize_rows(mk.row_ptr, mk.u.astype(np.float64))
        r, _ = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, xb, p1[sl])
        assert r <= 1e-6, (b, r)
    B0.close()
    B1.close()


def test_gangs_stop_together_at_the_iteration_cap(cuda, monkeypatch, small_batch):
    """Every member of a gang takes the same decisions: with a cap of 10 and
    of 100 iterations each market reports exactly that many."""
    monkeypatch.setenv("PDHCG_BATCH_GANG", "4")
    B = pdhcg.Batch(small_batch, device=cuda)
    monkeypatch.delenv("PDHCG_BATCH_GANG")
    for cap in (10, 100):
        st, _, _, infos = B.solve(tol=1e-14, max_iter=cap)
        assert st == pdhcg.PDHCG_MAX_ITER
        assert all(i.iters == cap and i.status == pdhcg.PDHCG_MAX_ITER for i in infos)
    B.close()
