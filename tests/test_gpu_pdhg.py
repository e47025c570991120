"""Restarted PDHG (Alg. 1, pdhcg_pdhg_solve) on the GPU against the FP64
oracle's restarted PDHG (oracle.pdhg_solve), through the C ABI.

* fixed-step, restart-free trajectories: prices, allocations, utilities t
  and their duals y after 40 iterations within 2e-4 of their scale (float32
  allocations; the bar of the PDHCG trajectory test);
* adaptive steps with restarts (Sec. 5), step by step through the first
  restart: kept-step and restart counts exactly, omega to 1e-3, eta to 0.15;
* the solve on the 1000 x 500 market: the unique equilibrium prices (Sec. 3
  Fact 1) of the PDHCG oracle to 1e-5 at relative KKT 1e-6, the oracle's
  FP64 KKT error of the returned (x, t, p, y) (Sec. 5 Criteria);
* shapes outside the built kernels are rejected."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_06258_amd import pdhcg, synth

pytestmark = pytest.mark.gpu


def _norm_rows(mk):
    uh, rmax = oracle.normalize_rows(mk.row_ptr, mk.u.astype(np.float64))
    return uh, rmax


def test_pdhg_fixed_step_trajectory(cuda):
    mk = synth.fisher_small(2).as_float32()
    deg = np.bincount(mk.col, minlength=mk.m)
    rdeg = np.diff(mk.row_ptr)
    kb = np.sqrt(deg.max()) + 1.0 + np.sqrt(float(deg.max()) * rdeg.max())
    common = dict(tol=0.0, max_iter=40, eval_every=16, step_mode=0, restart=0,
                  eta0=0.9 / kb, omega0=0.05 * float(mk.w.astype(np.float64).sum()) / mk.m,
                  output=1)
    M = pdhcg.Market.from_synth(mk, device=cuda)
    g, yg = M.pdhg_solve(**common)
    ora = oracle.pdhg_solve(mk.n, mk.m, mk.row_ptr, mk.col, mk.u.astype(np.float64),
                            mk.w.astype(np.float64), **common)
    M.close()
    assert g.info.iters == 40 and ora.iters == 40
    _, rmax = _norm_rows(mk)
    pg, xg = g.p.cpu().numpy(), g.x.cpu().numpy()
    tg = g.t.cpu().numpy() / rmax
    yg = yg.cpu().numpy() * rmax
    for a, b in ((pg, ora.p), (xg, ora.x), (tg, ora.t), (yg, ora.y)):
        assert np.max(np.abs(a - b)) <= 2e-4 * np.max(np.abs(b))


def test_pdhg_adaptive_trajectory(cuda):
    """Step by step for every k up to 66 (rejected steps, the first check
    and restart at 64 and its primal-weight update), with the bars of the
    PDHCG test: kept-step and restart counts exactly, omega to 1e-3, eta to
    0.15, prices to 1e-3 of their scale.  Measured: eta agrees to 3e-6
    through the first restart; the trajectories separate after about 75
    iterations."""
    mk = synth.fisher_small(0).as_float32()
    M = pdhcg.Market.from_synth(mk, device=cuda)
    seen_restart = seen_reject = False
    for k in range(1, 67):
        common = dict(tol=0.0, max_iter=k, output=1)
        g, _ = M.pdhg_solve(**common)
        ora = oracle.pdhg_solve(mk.n, mk.m, mk.row_ptr, mk.col, mk.u.astype(np.float64),
                                mk.w.astype(np.float64), **common)
        ge, oe, go, oo = float(g.info.eta), float(ora.eta), float(g.info.omega), float(ora.omega)
        ga, oa, gr, orr = int(g.info.accepted), int(ora.accepted), int(g.info.restarts), int(ora.restarts)
        pg = g.p.cpu().numpy().astype(np.float64)
        perr = float(np.max(np.abs(pg - ora.p)) / np.max(np.abs(ora.p)))
        case = (k, ga, oa, gr, orr, ge, oe, go, oo, perr)
        assert int(g.info.iters) == k and ora.iters == k, case
        assert ga == oa and gr == orr, case
        assert abs(ge - oe) <= 0.15 * oe and abs(go - oo) <= 1e-3 * oo, case
        assert perr <= 1e-3, case
        seen_restart |= orr > 0
        seen_reject |= oa < k
    assert seen_restart and seen_reject
    M.close()


def test_pdhg_solve_small_market(cuda):
    mk = synth.fisher_small(0).as_float32()
    u64, w64 = mk.u.astype(np.float64), mk.w.astype(np.float64)
    ref = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u64, w64, tol=1e-11, max_iter=400000)
    assert ref.status == oracle.OK
    M = pdhcg.Market.from_synth(mk, device=cuda)
    sol, y = M.pdhg_solve(tol=1e-6, max_iter=400000)
    assert sol.info.status == pdhcg.PDHCG_OK, pdhcg.lib().pdhcg_last_error()
    assert sol.info.rel_kkt <= 1e-6
    p, x = sol.p.cpu().numpy().astype(np.float64), sol.x.cpu().numpy().astype(np.float64)
    uh, rmax = _norm_rows(mk)
    t = sol.t.cpu().numpy().astype(np.float64) / rmax
    yy = y.cpu().numpy().astype(np.float64) * rmax
    r, parts = oracle.kkt_ty(mk.n, mk.m, mk.row_ptr, mk.col, uh, w64, x, t, p, yy)
    assert r <= 2e-6, parts
    err = np.max(np.abs(p - ref.p)) / np.max(np.abs(ref.p))
    assert err <= 1e-5, err
    assert abs(p.sum() - w64.sum()) / w64.sum() <= 1e-5
    # PDHG needs more iterations than PDHCG on the same market (Sec. 5 tables)
    s2 = M.solve(tol=1e-6, max_iter=400000)
    assert sol.info.iters > s2.info.iters
    M.close()


def test_pdhg_rejects_unbuilt_shapes(cuda):
    # a row of more than 512 entries
    mk = synth.bernoulli_market(40, 1100, 0.6, 3, w_mode="uniform").as_float32()
    M = pdhcg.Market.from_synth(mk, device=cuda)
    with pytest.raises(pdhcg.PDHCGError) as e:
        M.pdhg_solve(tol=1e-4)
    assert e.value.status == pdhcg.PDHCG_ERR_UNSUPPORTED
    M.close()
    # goods beyond LDS
    mk = synth.bernoulli_market(3000, 12000, 0.001, 4, w_mode="uniform").as_float32()
    M = pdhcg.Market.from_synth(mk, device=cuda)
    with pytest.raises(pdhcg.PDHCGError) as e:
        M.pdhg_solve(tol=1e-4)
    assert e.value.status == pdhcg.PDHCG_ERR_UNSUPPORTED
    M.close()
