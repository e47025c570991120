"""Markets whose goods do not all fit in LDS, on the GPU against the FP64
oracle through the C ABI.

Goods are relabelled by degree at creation and only the most bought keep
their prices and column partials in LDS; the others are gathered from
global memory and summed with float64 device atomics.  Creation picks this
layout when 16 bytes per good exceed the LDS; PDHCG_HOT=k forces it with k
goods in LDS, so that markets the oracle solves in seconds take the same
kernels.  Every entry point still takes and returns goods in the caller's
order, so the bars are the ones of the all-LDS layout (test_gpu_parity.py,
test_gpu_grad.py)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_06258_amd import pdhcg, synth
from test_gpu_parity import check_row_prox, prox_state, rel_err
from test_gpu_grad import _market, _rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zipf_small():
    mk = synth.zipf_market(6000, 800, 11, dmax=1500).as_float32()
    ora = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, mk.u.astype(np.float64),
                       mk.w.astype(np.float64), tol=1e-11, max_iter=400000)
    assert ora.status == oracle.OK
    return mk, ora


@pytest.mark.parametrize("hot", [1, 64, 500])
def test_forced_layout(cuda, monkeypatch, zipf_small, hot):
    mk, _ = zipf_small
    monkeypatch.setenv("PDHCG_HOT", str(hot))
    M = pdhcg.Market.from_synth(mk, device=cuda)
    assert M.lds_goods() == hot
    M.close()
    monkeypatch.delenv("PDHCG_HOT")
    M = pdhcg.Market.from_synth(mk, device=cuda)
    assert M.lds_goods() == mk.m
    M.close()


@pytest.mark.parametrize("hot", [1, 64, 500])
@pytest.mark.parametrize("kind", ["init", "random"])
def test_row_prox(cuda, monkeypatch, zipf_small, hot, kind):
    mk, _ = zipf_small
    monkeypatch.setenv("PDHCG_HOT", str(hot))
    rng = np.random.default_rng(hot * 7 + len(kind))
    x_in, p = prox_state(mk, rng, kind)
    check_row_prox(mk, cuda, x_in, p, 0.05)


@pytest.mark.parametrize("d", [3, 17, 100])
def test_row_prox_fixed_degree(cuda, monkeypatch, d):
    # every register shape of the row kernel, with most goods outside LDS
    mk = synth.fixed_degree_market(2000, 700, d, 40 + d, "uniform").as_float32()
    monkeypatch.setenv("PDHCG_HOT", "96")
    rng = np.random.default_rng(d)
    x_in, p = prox_state(mk, rng, "random")
    check_row_prox(mk, cuda, x_in, p, 0.3 / (mk.w.sum() / mk.m))


@pytest.mark.parametrize("hot", [1, 64])
def test_solve_and_kkt(cuda, monkeypatch, zipf_small, hot):
    mk, ora = zipf_small
    monkeypatch.setenv("PDHCG_HOT", str(hot))
    M = pdhcg.Market.from_synth(mk, device=cuda)
    assert M.lds_goods() == hot
    sol = M.solve(tol=1e-6, max_iter=400000)
    assert sol.info.status == pdhcg.PDHCG_OK, pdhcg.pdhcg_last_error()
    p, x = sol.p.cpu().numpy().astype(np.float64), sol.x.cpu().numpy().astype(np.float64)
    uh, _ = oracle.normalize_rows(mk.row_ptr, mk.u.astype(np.float64))
    r, _ = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, x, p)
    assert r <= 2e-6
    assert rel_err(p, ora.p) <= 1e-5
    assert sol.info.rel_kkt <= 1e-6
    rng = np.random.default_rng(1)
    pp = (ora.p * (1 + 1e-3 * rng.standard_normal(mk.m))).astype(np.float32)
    xx = np.maximum(ora.x * (1 + 1e-3 * rng.standard_normal(mk.nnz)), 0).astype(np.float32)
    info = M.kkt(torch.as_tensor(pp, device=cuda), torch.as_tensor(xx, device=cuda))
    _, parts = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, mk.w, xx.astype(np.float64),
                          pp.astype(np.float64))
    got = np.array([info.rel_primal, info.rel_dual, info.rel_gap])
    assert np.all(np.abs(got - parts) <= 1e-7 + 1e-6 * parts), (got, parts)
    # warm start from the caller-ordered solution stays at the solution
    prm = pdhcg.pdhcg_default_params(tol=1e-6, max_iter=400000)
    sol2 = M.solve(prm, p0=sol.p, x0=sol.x)
    assert sol2.info.status == pdhcg.PDHCG_OK
    assert sol2.info.iters <= 2 * prm.eval_every, sol2.info.iters
    assert rel_err(sol2.p.cpu().numpy().astype(np.float64), ora.p) <= 1e-5
    M.close()


def test_backward(cuda, monkeypatch):
    n, m = 60, 20
    rp, col, u, w, rng = _market(5, n, m, 0.5)
    ref = oracle.solve(n, m, rp, col, u.astype(np.float64), w.astype(np.float64), tol=1e-13,
                       max_iter=2000000)
    assert ref.status == oracle.OK
    g = rng.normal(size=m)
    st, du_i, dw_i, _ = oracle.implicit_grad(n, m, rp, col, u, w, ref.x, ref.p, g)
    assert st == oracle.OK
    monkeypatch.setenv("PDHCG_HOT", "5")
    M = pdhcg.Market(rp, col, u, w, m=m, device=cuda)
    assert M.lds_goods() == 5
    sol = M.solve(tol=1e-7, max_iter=200000)
    assert sol.info.status == pdhcg.PDHCG_OK
    # the oracle's primal weight for the unrolled steps: the limit does not
    # depend on it, how fast it is reached does (see test_gpu_grad.py)
    du, dw = M.backward(sol.x, sol.p, ref.omega, torch.tensor(g, dtype=torch.float32),
                        unroll=1024, ckpt_every=32)
    du, dw = du.double().cpu().numpy(), dw.double().cpu().numpy()
    assert _rel(du, du_i) <= 1e-4, _rel(du, du_i)
    assert _rel(dw, dw_i) <= 1e-4, _rel(dw, dw_i)
    M.close()
