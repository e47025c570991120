"""Skewed markets on the GPU against the FP64 oracle, through the C ABI:
rows longer than the register-resident shapes hold (more than 512 entries,
one wave per row) mixed with short rows, Zipf buyer degrees and
popularity-skewed goods (the shape of the skewed workload at a size the
oracle solves in seconds).  Same bars as tests/test_gpu_parity.py."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_06258_amd import pdhcg, synth
from test_gpu_parity import check_row_prox, prox_state, rel_err

pytestmark = pytest.mark.gpu


# team kernel shape code of a row length (rows held by teams of waves)
TEAM_CODE = {513: 1, 1500: 2, 4000: 3, 6000: 4, 12000: 5, 17000: 0}



@pytest.mark.parametrize("kernel", ["team", "wave"])
@pytest.mark.parametrize("d", [513, 1500, 4000, 6000, 12000, 17000])
def test_row_prox_long_rows(cuda, monkeypatch, d, kernel):
    """Rows above 512 entries: in registers of teams of waves (every team
    shape; rows above 16384 entries stay on the one-wave-per-row kernel) and
    on the one-wave-per-row kernel (PDHCG_TEAM=0), entry by entry against
    the exact prox (PDHCG_TEAM=2 takes the teams on every layout).  Above
    10,112 goods the market takes the relabelled layout (goods beyond LDS)."""
    n, m = (300, d + 200) if d <= 4000 else (40, d + 200)
    mk = synth.fixed_degree_market(n, m, d, 300 + d, "uniform").as_float32()
    monkeypatch.setenv("PDHCG_TEAM", "0" if kernel == "wave" else "2")
    M = pdhcg.Market.from_synth(mk, device=cuda)
    assert M.bins() == [(0, TEAM_CODE[d] if kernel == "team" else 0, n)]
    M.close()
    rng = np.random.default_rng(d)
    for kind in ("init", "random", "sparse"):
        x_in, p = prox_state(mk, rng, kind)
        check_row_prox(mk, cuda, x_in, p, 0.3 / (mk.w.sum() / mk.m))


@pytest.mark.parametrize("hot", [None, 64])
def test_team_and_wave_kernels_reach_the_same_prices(cuda, monkeypatch, zipf_small, hot):
    """Solves of a market with rows of up to 1500 entries, its long rows on
    the team kernel or on the one-wave-per-row kernel, with all goods in LDS
    and with 64 (the others' column sums through the panel buffers or the
    column gathers), against the oracle and each other."""
    mk, ora = zipf_small
    prices = {}
    for kernel in ("team", "wave"):
        if hot is not None:
            monkeypatch.setenv("PDHCG_HOT", str(hot))
        monkeypatch.setenv("PDHCG_TEAM", "0" if kernel == "wave" else "2")
        M = pdhcg.Market.from_synth(mk, device=cuda)
        monkeypatch.delenv("PDHCG_TEAM", raising=False)
        monkeypatch.delenv("PDHCG_HOT", raising=False)
        long_bins = [e for g, e, _ in M.bins() if g == 0]
        assert long_bins and all((e == 0) == (kernel == "wave") for e in long_bins), M.bins()
        sol = M.solve(tol=1e-6, max_iter=400000)
        assert sol.info.status == pdhcg.PDHCG_OK, pdhcg.pdhcg_last_error()
        p, x = sol.p.cpu().numpy().astype(np.float64), sol.x.cpu().numpy().astype(np.float64)
        uh, _ = oracle.normalize_rows(mk.row_ptr, mk.u.astype(np.float64))
        r, _ = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, x, p)
        assert r <= 2e-6, (kernel, r)
        assert rel_err(p, ora.p) <= 1e-5, kernel
        prices[kernel] = p
        M.close()
    assert rel_err(prices["team"], prices["wave"]) <= 2e-5


@pytest.fixture(scope="module")
def zipf_small():
    mk = synth.zipf_market(6000, 800, 11, dmax=1500).as_float32()
    ora = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, mk.u.astype(np.float64),
                       mk.w.astype(np.float64), tol=1e-11, max_iter=400000)
    assert ora.status == oracle.OK
    return mk, ora


def test_zipf_market_bins(cuda, zipf_small):
    mk, _ = zipf_small
    M = pdhcg.Market.from_synth(mk, device=cuda)
    bins = M.bins()
    assert any(g == 0 for g, _, _ in bins) and any(g > 0 for g, _, _ in bins)
    assert sum(r for _, _, r in bins) == mk.n
    M.close()


def test_zipf_row_prox(cuda, zipf_small):
    mk, _ = zipf_small
    rng = np.random.default_rng(5)
    x_in, p = prox_state(mk, rng, "random")
    check_row_prox(mk, cuda, x_in, p, 0.05)


def test_zipf_solve_parity(cuda, zipf_small):
    mk, ora = zipf_small
    M = pdhcg.Market.from_synth(mk, device=cuda)
    sol = M.solve(tol=1e-6, max_iter=400000)
    assert sol.info.status == pdhcg.PDHCG_OK, pdhcg.pdhcg_last_error()
    p, x = sol.p.cpu().numpy().astype(np.float64), sol.x.cpu().numpy().astype(np.float64)
    uh, _ = oracle.normalize_rows(mk.row_ptr, mk.u.astype(np.float64))
    r, _ = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, x, p)
    assert r <= 2e-6
    assert rel_err(p, ora.p) <= 1e-5
    # the KKT entry point on the oracle's solution, perturbed
    rng = np.random.default_rng(1)
    pp = (ora.p * (1 + 1e-3 * rng.standard_normal(mk.m))).astype(np.float32)
    xx = np.maximum(ora.x * (1 + 1e-3 * rng.standard_normal(mk.nnz)), 0).astype(np.float32)
    info = M.kkt(torch.as_tensor(pp, device=cuda), torch.as_tensor(xx, device=cuda))
    _, parts = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, xx.astype(np.float64),
                          pp.astype(np.float64))
    got = np.array([info.rel_primal, info.rel_dual, info.rel_gap])
    assert np.all(np.abs(got - parts) <= 1e-7 + 1e-6 * parts), (got, parts)
    M.close()


def test_backward_with_long_rows(cuda):
    # 30 buyers valuing 520-600 of 700 goods: every row takes the long path
    rng = np.random.default_rng(17)
    n, m = 30, 700
    rows, cols = [], []
    for i in range(n):
        d = int(rng.integers(520, 601))
        c = np.sort(rng.choice(m, size=d, replace=False))
        rows.append(np.full(d, i))
        cols.append(c)
    rows, col = np.concatenate(rows), np.concatenate(cols).astype(np.int32)
    assert np.all(np.bincount(col, minlength=m) > 0)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    u = rng.uniform(0.05, 1.0, col.size).astype(np.float32)
    w = rng.uniform(0.5, 1.5, n).astype(np.float32)
    ref = oracle.solve(n, m, row_ptr, col, u.astype(np.float64), w.astype(np.float64),
                       tol=1e-13, max_iter=4000000)
    assert ref.status == oracle.OK
    g = rng.normal(size=m)
    st, du_i, dw_i, _ = oracle.implicit_grad(n, m, row_ptr, col, u, w, ref.x, ref.p, g)
    assert st == oracle.OK
    M = pdhcg.Market(row_ptr, col, u, w, m=m, device=cuda)
    assert M.bins() == [(0, 0, n)]  # the one-wave-per-row kernel (all goods in LDS)
    sol = M.solve(tol=1e-7, max_iter=400000)
    assert sol.info.status == pdhcg.PDHCG_OK
    # the fixed-step map contracts slowly on this market (few buyers, long
    # rows): the oracle's own unrolled derivative is 6e-3 off at K = 2048 and
    # 1e-8 at K = 8192
    du, dw = M.backward(sol.x, sol.p, sol.info.omega, torch.tensor(g, dtype=torch.float32),
                        unroll=8192, ckpt_every=128)
    du, dw = du.double().cpu().numpy(), dw.double().cpu().numpy()
    assert rel_err(du, du_i) <= 1e-4, rel_err(du, du_i)
    assert rel_err(dw, dw_i) <= 1e-4, rel_err(dw, dw_i)
    M.close()


def test_ksection_rejected_on_long_rows(cuda):
    """The k-section search is built for the register-resident shapes: on a
    market with rows above 512 entries the solve and the row prox say so
    instead of silently using another search."""
    mk = synth.fixed_degree_market(40, 700, 520, 9, "uniform").as_float32()
    M = pdhcg.Market.from_synth(mk, device=cuda)
    x_in = torch.full((mk.nnz,), 0.01, device=cuda)
    p = torch.ones(mk.m, device=cuda)
    for search in (pdhcg.PDHCG_SEARCH_KSECTION, pdhcg.PDHCG_SEARCH_KSECTION_WAVE):
        prm = pdhcg.pdhcg_default_params(search=search, sections=32)
        with pytest.raises(pdhcg.PDHCGError) as e:
            M.solve(prm)
        assert e.value.status == pdhcg.PDHCG_ERR_UNSUPPORTED
        with pytest.raises(pdhcg.PDHCGError) as e:
            M.row_prox(x_in, p, 0.1, prm)
        assert e.value.status == pdhcg.PDHCG_ERR_UNSUPPORTED
    M.close()
