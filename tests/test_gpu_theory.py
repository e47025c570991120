"""Alg. 2 in the setting of its analysis (Sec. 3: fixed sigma = tau =
1/(2||K||), fixed restart length K, restarts to the average) on the GPU
(pdhcg_solve_fixed_restart) against the oracle's (oracle.fixed_restart):
the distance of every restart point to p* and its relative KKT error agree,
and the distance contracts from restart to restart (Theorem 1)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2506_06258_amd import pdhcg, synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("K,R", [(64, 12), (256, 8)])
def test_fixed_restart_distances_match_oracle(cuda, K, R):
    mk = synth.fisher_small(0).as_float32()
    u64, w64 = mk.u.astype(np.float64), mk.w.astype(np.float64)
    ref = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u64, w64, tol=1e-11, max_iter=400000)
    assert ref.status == oracle.OK
    st, p_o, _, d_o, k_o = oracle.fixed_restart(mk.n, mk.m, mk.row_ptr, mk.col, u64, w64, K, R,
                                                p_ref=ref.p)
    assert st == oracle.OK
    M = pdhcg.Market.from_synth(mk, device=cuda)
    sol, d_g, k_g = M.solve_fixed_restart(K, R, p_ref=torch.tensor(ref.p, dtype=torch.float32))
    M.close()
    assert sol.info.iters == K * R
    # float32 allocations over K * R fixed steps: distances to 1e-4 of the
    # starting distance, KKT errors to 1e-3 relative
    assert np.max(np.abs(d_g - d_o)) <= 1e-4 * d_o[0], (d_g, d_o)
    assert np.max(np.abs(k_g - k_o) / k_o) <= 1e-3, (k_g, k_o)
    pg = sol.p.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(pg - p_o)) <= 1e-4 * np.max(p_o)
    # linear convergence of the restart points (Theorem 1): after the first
    # restart the distance shrinks every time, and overall by a factor
    assert np.all(np.diff(d_g[1:]) < 0), d_g
    assert d_g[-1] <= 0.5 * d_g[1]


def test_fixed_restart_rejects_bad_arguments(cuda):
    mk = synth.bernoulli_market(50, 20, 0.3, 8, w_mode="uniform").as_float32()
    M = pdhcg.Market.from_synth(mk, device=cuda)
    for K, R in ((0, 3), (4, -1)):
        with pytest.raises(pdhcg.PDHCGError) as e:
            M.solve_fixed_restart(K, R)
        assert e.value.status == pdhcg.PDHCG_ERR_ARG
    M.close()
