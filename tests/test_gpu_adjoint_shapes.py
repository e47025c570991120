"""The reverse mode (pdhcg_backward) against the oracle's FP64 reverse mode
through the same unrolled iteration (oracle.unrolled_grad: the same K
fixed steps, tau = eta/omega, sigma = eta*omega with eta = 0.9/||K_x||, K_x
the column-sum operator on the support of the start point, from the same
start point), on every row-kernel shape the solver picks: the
short shapes with 2-byte good ids, 16 lanes x 7 entries (the 1e8-edge
market's rows of 100), 64 x 8 (rows of up to 512), rows of more than 512
entries (one wave per row), goods beyond LDS (relabelled market), and a
market with several bins.  Both sides differentiate the same function, so
the bar is the gradient target itself: 1e-4 of the largest entry."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_06258_amd import pdhcg, synth

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


def _check(mk, cuda, K=64, expect=None, hot=None, monkeypatch=None):
    if hot is not None:
        monkeypatch.setenv("PDHCG_HOT", str(hot))
    M = pdhcg.Market.from_synth(mk, device=cuda)
    if hot is not None:
        monkeypatch.delenv("PDHCG_HOT")
        assert M.lds_goods() == hot
    bins = M.bins()
    if expect is not None:
        assert any((g, e) == expect for g, e, _ in bins), bins
    # a tight start point: the unrolled map is piecewise smooth (entries
    # cross zero), and from a loose start the trajectory moves enough for
    # float32 and float64 iterates to take different pieces
    sol = M.solve(tol=1e-7, max_iter=400000)
    assert sol.info.status == pdhcg.PDHCG_OK
    rng = np.random.default_rng(mk.nnz % 1000)
    g = rng.normal(size=mk.m)
    omega = float(sol.info.omega)
    du, dw = M.backward(sol.x, sol.p, omega, torch.tensor(g, dtype=torch.float32), unroll=K,
                        ckpt_every=16)
    du, dw = du.double().cpu().numpy(), dw.double().cpu().numpy()
    M.close()
    x0 = sol.x.double().cpu().numpy()
    # pdhcg_backward's step: 0.9 / sqrt(largest number of buyers with x > 0)
    act = np.bincount(mk.col[x0 > 0], minlength=mk.m)
    eta = 0.9 / np.sqrt(max(act.max(), 1))
    p0 = sol.p.double().cpu().numpy()
    st, du_o, dw_o, _ = oracle.unrolled_grad(mk.n, mk.m, mk.row_ptr, mk.col, mk.u, mk.w, x0, p0,
                                             eta / omega, eta * omega, K, g)
    assert st == oracle.OK
    assert np.all(np.isfinite(du)) and np.all(np.isfinite(dw))
    assert _rel(du, du_o) <= 1e-4, _rel(du, du_o)
    assert _rel(dw, dw_o) <= 1e-4, _rel(dw, dw_o)
    # p is invariant to scaling a buyer's utilities (Sec. 5 preprocessing),
    # and so is the unrolled map through the normalisation: Euler's
    # identity sum_j u_ij dL/du_ij = 0 for every buyer
    rows = np.repeat(np.arange(mk.n), np.diff(mk.row_ptr))
    eu = np.bincount(rows, weights=mk.u.astype(np.float64) * du, minlength=mk.n)
    scale = np.bincount(rows, weights=np.abs(mk.u.astype(np.float64) * du), minlength=mk.n)
    assert np.all(np.abs(eu) <= 1e-4 * scale + 1e-12), float(np.max(np.abs(eu) / (scale + 1e-30)))


@pytest.mark.parametrize("d,expect", [(3, None), (17, None), (100, (16, 7)), (300, None),
                                      (500, (64, 8))])
def test_adjoint_register_shapes(cuda, d, expect):
    n = max(300, 4 * d)
    mk = synth.fixed_degree_market(n, max(2 * d, 120), d, 500 + d).as_float32()
    _check(mk, cuda, expect=expect)


@pytest.mark.parametrize("kernel", ["team", "wave"])
def test_adjoint_long_rows(cuda, monkeypatch, kernel):
    """Rows of 700 entries: the forward steps of the reverse mode on the team
    kernel (shape code 1, forced) or on the one-wave-per-row kernel; the adjoint
    pass is the one-wave-per-row adjoint kernel in both."""
    mk = synth.fixed_degree_market(120, 1500, 700, 41).as_float32()
    monkeypatch.setenv("PDHCG_TEAM", "0" if kernel == "wave" else "2")
    _check(mk, cuda, expect=(0, 1 if kernel == "team" else 0))


def test_adjoint_goods_beyond_lds(cuda, monkeypatch):
    mk = synth.fixed_degree_market(600, 400, 40, 42).as_float32()
    _check(mk, cuda, hot=64, monkeypatch=monkeypatch)


def test_adjoint_mixed_bins(cuda):
    mk = synth.bernoulli_market(2000, 600, 0.05, 43, w_mode="uniform").as_float32()
    _check(mk, cuda)
