"""Gradients of equilibrium prices on the GPU (pdhcg_backward, FisherPrices)
against the FP64 oracle, through the C ABI.

Reference: the oracle's implicit derivative of the equilibrium prices on the
active support (oracle.implicit_grad, pinned by closed forms and finite
differences in test_oracle_grad.py).  The GPU unrolls 1024 fixed-step
iterations from its own solution; the unrolled derivative converges to the
implicit one geometrically (the oracle pins that too), so the bar is the
gradient accuracy target, 1e-4 relative to the largest gradient entry.  The oracle's
own unrolled reverse mode from its own solution is a second reference with
the same bar.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_06258_amd import pdhcg

pytestmark = pytest.mark.gpu


def _market(seed, n, m, q):
    rng = np.random.default_rng(seed)
    U = rng.uniform(0.05, 1.0, (n, m)) * (rng.uniform(size=(n, m)) < q)
    for i in range(n):
        if not U[i].any():
            U[i, rng.integers(m)] = 0.5
    for j in range(m):
        if not U[:, j].any():
            U[rng.integers(n), j] = 0.5
    rows, cols = np.nonzero(U)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    u = U[rows, cols].astype(np.float32)  # both sides solve the float32 instance
    w = rng.uniform(0.5, 1.5, n).astype(np.float32)
    return row_ptr, cols.astype(np.int32), u, w, rng


def _rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30)


@pytest.mark.parametrize("seed,n,m", [(3, 30, 10), (5, 60, 20)])
def test_backward_matches_oracle(cuda, seed, n, m):
    rp, col, u, w, rng = _market(seed, n, m, 0.5)
    ref = oracle.solve(n, m, rp, col, u.astype(np.float64), w.astype(np.float64), tol=1e-13,
                       max_iter=2000000)
    assert ref.status == oracle.OK
    g = rng.normal(size=m)
    st, du_i, dw_i, _ = oracle.implicit_grad(n, m, rp, col, u, w, ref.x, ref.p, g)
    assert st == oracle.OK
    # the step on the support of the start point (pdhcg_backward's rule)
    act = np.bincount(col[ref.x > 0], minlength=m)
    eta = 0.9 / np.sqrt(max(act.max(), 1))
    st, du_u, dw_u, _ = oracle.unrolled_grad(n, m, rp, col, u, w, ref.x, ref.p, eta / ref.omega,
                                             eta * ref.omega, 1024, g)
    assert st == oracle.OK

    M = pdhcg.Market(rp, col, u, w, m=m, device=cuda)
    sol = M.solve(tol=1e-7, max_iter=200000)
    assert sol.info.status == pdhcg.PDHCG_OK
    # The limit of the unrolled reverse mode does not depend on the primal
    # weight, but how fast it is reached does, by orders of magnitude (on
    # this market the oracle's 1024-step error is 2e-7 at omega 0.45 and
    # 5e-3 at omega 0.17); the GPU solve's final omega depends on its own
    # float32 trajectory, so both sides unroll with the oracle's.
    du, dw = M.backward(sol.x, sol.p, ref.omega, torch.tensor(g, dtype=torch.float32),
                        unroll=1024, ckpt_every=32)
    du = du.double().cpu().numpy()
    dw = dw.double().cpu().numpy()
    assert np.all(np.isfinite(du)) and np.all(np.isfinite(dw))
    assert _rel(du, du_i) <= 1e-4, _rel(du, du_i)
    assert _rel(dw, dw_i) <= 1e-4, _rel(dw, dw_i)
    assert _rel(du, du_u) <= 1e-4 and _rel(dw, dw_u) <= 1e-4
    M.close()


def test_checkpoint_spacing_does_not_change_the_gradient(cuda):
    rp, col, u, w, rng = _market(8, 40, 12, 0.5)
    M = pdhcg.Market(rp, col, u, w, m=12, device=cuda)
    sol = M.solve(tol=1e-7, max_iter=200000)
    g = torch.tensor(rng.normal(size=12), dtype=torch.float32)
    out = [M.backward(sol.x, sol.p, sol.info.omega, g, unroll=300, ckpt_every=c) for c in (1, 7, 300)]
    # recomputed segments repeat the forward steps; column sums are added by
    # float64 LDS atomics in no fixed order, so equal to rounding only
    for du, dw in out[1:]:
        assert torch.allclose(du, out[0][0], rtol=1e-5, atol=1e-6 * float(out[0][0].abs().max()))
        assert torch.allclose(dw, out[0][1], rtol=1e-5, atol=1e-6 * float(out[0][1].abs().max()))
    M.close()


def test_fisher_prices_autograd(cuda):
    n, m = 50, 15
    rp, col, u, w, rng = _market(13, n, m, 0.5)
    ref = oracle.solve(n, m, rp, col, u.astype(np.float64), w.astype(np.float64), tol=1e-13,
                       max_iter=2000000)
    target = ref.p * (1.0 + 0.05 * rng.normal(size=m))
    # d/dp sum (p - p*)^2 at the oracle equilibrium
    st, du_i, dw_i, _ = oracle.implicit_grad(n, m, rp, col, u, w, ref.x, ref.p,
                                             2.0 * (ref.p - target))
    assert st == oracle.OK
    ut = torch.tensor(u, device=cuda, requires_grad=True)
    wt = torch.tensor(w, device=cuda, requires_grad=True)
    prm = pdhcg.pdhcg_default_params(tol=1e-7, max_iter=200000)
    p = pdhcg.FisherPrices.apply(ut, wt, torch.tensor(rp, dtype=torch.int32, device=cuda),
                                 torch.tensor(col, device=cuda), m, prm, 1024, 32)
    loss = ((p.double() - torch.tensor(target, device=cuda)) ** 2).sum()
    loss.backward()
    assert _rel(ut.grad.double().cpu().numpy(), du_i) <= 1e-4
    assert _rel(wt.grad.double().cpu().numpy(), dw_i) <= 1e-4


def test_backward_central_differences_of_gpu_solves(cuda):
    # a coarse check that needs no oracle: central differences of float32
    # GPU solves (noise ~1e-6 relative in p) on a few budgets and utilities
    n, m = 30, 10
    rp, col, u, w, rng = _market(3, n, m, 0.5)
    g = rng.normal(size=m)
    M = pdhcg.Market(rp, col, u, w, m=m, device=cuda)
    sol = M.solve(tol=1e-8, max_iter=400000)
    du, dw = M.backward(sol.x, sol.p, sol.info.omega, torch.tensor(g, dtype=torch.float32))
    du, dw = du.double().cpu().numpy(), dw.double().cpu().numpy()
    M.close()

    def loss(uu, ww):
        Mx = pdhcg.Market(rp, col, uu, ww, m=m, device=cuda)
        s = Mx.solve(tol=1e-8, max_iter=400000)
        Mx.close()
        return float(g @ s.p.double().cpu().numpy())

    h = 2e-3
    for i in (0, 7, 19):
        e = np.zeros(n, np.float32)
        e[i] = h
        fd = (loss(u, w + e) - loss(u, w - e)) / (2 * h)
        assert abs(fd - dw[i]) <= 2e-2 * (1 + abs(fd)), (i, fd, dw[i])
    big = np.argsort(-np.abs(du))[:3]
    for q in big:
        e = np.zeros(len(u), np.float32)
        e[q] = h
        fd = (loss(u + e, w) - loss(u - e, w)) / (2 * h)
        assert abs(fd - du[q]) <= 2e-2 * (1 + abs(fd)), (q, fd, du[q])


def test_backward_rejects_bad_arguments(cuda):
    rp, col, u, w, _ = _market(3, 20, 6, 0.5)
    M = pdhcg.Market(rp, col, u, w, m=6, device=cuda)
    sol = M.solve(tol=1e-5)
    g = torch.ones(6)
    for kw in (dict(omega=0.0), dict(omega=float("nan"))):
        with pytest.raises(pdhcg.PDHCGError) as e:
            M.backward(sol.x, sol.p, kw["omega"], g)
        assert e.value.status == pdhcg.PDHCG_ERR_ARG
    with pytest.raises(pdhcg.PDHCGError) as e:
        M.backward(sol.x, sol.p, 1.0, g, unroll=0)
    assert e.value.status == pdhcg.PDHCG_ERR_ARG
    M.close()


def test_batch_backward_matches_oracle(cuda):
    """pdhcg_batch_backward: every market of a batch against the oracle's
    implicit derivative at its equilibrium (same bar as above)."""
    from paper_2506_06258_amd import synth
    specs = [(3, 30, 10), (5, 60, 20), (8, 40, 12), (13, 50, 15)]
    markets, refs, gs = [], [], []
    for seed, n, m in specs:
        rp, col, u, w, rng = _market(seed, n, m, 0.5)
        mk = synth.Market(n, m, rp.astype(np.int32), col, u, w, f"grad-{seed}")
        ref = oracle.solve(n, m, rp, col, u.astype(np.float64), w.astype(np.float64), tol=1e-13,
                           max_iter=2000000)
        assert ref.status == oracle.OK
        g = rng.normal(size=m)
        st, du_i, dw_i, _ = oracle.implicit_grad(n, m, rp, col, u, w, ref.x, ref.p, g)
        assert st == oracle.OK
        markets.append(mk)
        refs.append((du_i, dw_i))
        gs.append(g)
    bt = synth.batch_from_markets(markets)
    B = pdhcg.Batch(bt, device=cuda)
    st, p, x, infos = B.solve(tol=1e-7, max_iter=200000)
    assert st == pdhcg.PDHCG_OK
    du, dw = B.backward(x, p, [i.omega for i in infos], torch.tensor(np.concatenate(gs)),
                        unroll=1024, ckpt_every=32)
    du, dw = du.double().cpu().numpy(), dw.double().cpu().numpy()
    row_off = np.concatenate([[0], np.cumsum([mk.n for mk in markets])])
    for b, (du_i, dw_i) in enumerate(refs):
        dub = du[B.edge_off[b]:B.edge_off[b + 1]]
        dwb = dw[row_off[b]:row_off[b + 1]]
        assert _rel(dub, du_i) <= 1e-4, (b, _rel(dub, du_i))
        assert _rel(dwb, dw_i) <= 1e-4, (b, _rel(dwb, dw_i))
    with pytest.raises(pdhcg.PDHCGError) as e:
        B.backward(x, p, [0.0] * len(markets), torch.tensor(np.concatenate(gs)))
    assert e.value.status == pdhcg.PDHCG_ERR_ARG
    B.close()


@pytest.mark.parametrize("gang", ["0", "3", "auto"])
def test_batch_backward_matches_single_market(cuda, monkeypatch, gang):
    """The persistent batched reverse mode computes, market by market, what
    the single-market reverse mode computes (same unrolled iteration, same
    primal weights): markets chosen so that every batch row shape appears,
    including rows of more than 1024 entries; each market on one workgroup,
    split over gangs of three, and as the automatic plan splits them (every
    market of so small a batch goes to a gang)."""
    from paper_2506_06258_amd import synth
    specs = [(300, 40, 0.3), (300, 120, 0.3), (400, 300, 0.3), (500, 700, 0.3),
             (300, 1500, 0.4), (60, 2000, 0.6)]
    markets = [synth.bernoulli_market(n, m, q, 60 + k, w_mode="uniform").as_float32()
               for k, (n, m, q) in enumerate(specs)]
    bt = synth.batch_from_markets(markets)
    if gang != "auto":
        monkeypatch.setenv("PDHCG_BATCH_GANG", gang)
    B = pdhcg.Batch(bt, device=cuda)
    monkeypatch.delenv("PDHCG_BATCH_GANG", raising=False)
    st, p, x, infos = B.solve(tol=1e-5, max_iter=200000)
    assert st == pdhcg.PDHCG_OK
    rng = np.random.default_rng(5)
    g = torch.tensor(rng.normal(size=int(B.good_off[-1])), dtype=torch.float32)
    omegas = [i.omega for i in infos]
    K, L = 48, 8
    du, dw = B.backward(x, p, omegas, g, unroll=K, ckpt_every=L)
    du, dw = du.double().cpu().numpy(), dw.double().cpu().numpy()
    row_off = np.concatenate([[0], np.cumsum([mk.n for mk in markets])])
    for b, mk in enumerate(markets):
        eo0, eo1 = int(B.edge_off[b]), int(B.edge_off[b + 1])
        go0, go1 = int(B.good_off[b]), int(B.good_off[b + 1])
        M = pdhcg.Market.from_synth(mk, device=cuda)
        d1, w1 = M.backward(x[eo0:eo1], p[go0:go1], omegas[b], g[go0:go1], unroll=K,
                            ckpt_every=L)
        M.close()
        d1, w1 = d1.double().cpu().numpy(), w1.double().cpu().numpy()
        assert np.all(np.isfinite(du[eo0:eo1])), b
        # float64 LDS sums in no fixed order on both sides: equal to rounding
        assert _rel(du[eo0:eo1], d1) <= 1e-5, (b, _rel(du[eo0:eo1], d1))
        assert _rel(dw[row_off[b]:row_off[b + 1]], w1) <= 1e-5, b
    B.close()


def test_batch_backward_on_c3_markets_matches_implicit_derivative(cuda):
    """The batched and differentiated workload's loss, sum_j (p_j - q_j)^2 with
    q a seeded 1% perturbation of the oracle's prices, on markets of the
    4096-market batch itself (generated one by one with the batch's per-market
    seeds; eight of the first 400 spread over sizes up to 40,000 entries, so
    that the oracle's implicit derivative is quick): the batched reverse mode
    through 4096 unrolled steps (1024 and 2048 reported)
    against the FP64 implicit derivative at the equilibrium, 1e-4 of the
    largest entry."""
    from paper_2506_06258_amd import synth
    picks = []
    for b in range(400):
        rng = np.random.default_rng([1001, b])
        n = int(round(np.exp(rng.uniform(np.log(64), np.log(8192)))))
        m = int(round(np.exp(rng.uniform(np.log(16), np.log(2048)))))
        q = float(rng.uniform(0.05, 0.30))
        picks.append((int(round(n * m * q)), b))
    # eight markets spread over sizes up to 40,000 entries
    small = sorted(t for t in picks if t[0] <= 40000)
    picks = [small[int(round(k * (len(small) - 1) / 7))][1] for k in range(8)]
    markets, refs, gs = [], [], []
    for b in picks:
        rng = np.random.default_rng([1001, b])
        n = int(round(np.exp(rng.uniform(np.log(64), np.log(8192)))))
        m = int(round(np.exp(rng.uniform(np.log(16), np.log(2048)))))
        q = float(rng.uniform(0.05, 0.30))
        rp, col, u, w = synth._sample_market(rng, n, m, q)
        mk = synth.Market(n, m, rp.astype(np.int32), col, u, w, f"c3[{b}]")
        ref = oracle.solve(n, m, mk.row_ptr, col, u.astype(np.float64), w.astype(np.float64),
                           tol=1e-13, max_iter=4000000)
        assert ref.status == oracle.OK, b
        qp = ref.p * (1.0 + 0.01 * np.random.default_rng(b).normal(size=m))
        g = 2.0 * (ref.p - qp)
        st, du_i, dw_i, _ = oracle.implicit_grad(n, m, mk.row_ptr, col, u, w, ref.x, ref.p, g)
        assert st == oracle.OK, b
        markets.append(mk)
        refs.append((du_i, dw_i))
        gs.append(g)
    bt = synth.batch_from_markets(markets)
    B = pdhcg.Batch(bt, device=cuda)
    st, p, x, infos = B.solve(tol=1e-7, max_iter=400000)
    assert st == pdhcg.PDHCG_OK
    row_off = np.concatenate([[0], np.cumsum([mk.n for mk in markets])])
    for K in (1024, 2048, 4096):
        du, dw = B.backward(x, p, [i.omega for i in infos], torch.tensor(np.concatenate(gs)),
                            unroll=K, ckpt_every=32)
        du, dw = du.double().cpu().numpy(), dw.double().cpu().numpy()
        errs = []
        for k, (du_i, dw_i) in enumerate(refs):
            eu = _rel(du[B.edge_off[k]:B.edge_off[k + 1]], du_i)
            ew = _rel(dw[row_off[k]:row_off[k + 1]], dw_i)
            errs.append((picks[k], markets[k].n, markets[k].m, markets[k].nnz, float(eu), float(ew)))
        print(f"c3 markets, unroll {K} (b, n, m, nnz, du err, dw err):", errs)
    for b, n, m, nnz, eu, ew in errs:
        assert eu <= 1e-4 and ew <= 1e-4, (b, n, m, eu, ew)
    B.close()
