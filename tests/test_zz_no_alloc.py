"""pdhcg_backward_noalloc (the reverse mode with the library's fixed device
workspace instead of per-call allocations) against pdhcg_backward, through
the C ABI: two calls in a row on one GPU, the second on a smaller market,
each compared with the allocating entry point on the same inputs; and the
size limit reported before any device work."""
import numpy as np
import pytest
import torch

from paper_2506_06258_amd import pdhcg, synth

pytestmark = pytest.mark.gpu


def _solved(n, m, q, seed, cuda):
    mk = synth.bernoulli_market(n, m, q, seed, w_mode="uniform").as_float32()
    M = pdhcg.Market.from_synth(mk, device=cuda)
    sol = M.solve(tol=1e-7, max_iter=200000)
    assert sol.info.status == pdhcg.PDHCG_OK
    g = torch.tensor(np.random.default_rng(seed).normal(size=m), dtype=torch.float32)
    return mk, M, sol, g


def _both(M, sol, g, unroll, ckpt):
    ref = M.backward(sol.x, sol.p, sol.info.omega, g, unroll=unroll, ckpt_every=ckpt)
    # outputs pre-filled with garbage: the no-allocation call must write every entry
    du = torch.full_like(ref[0], float("nan"))
    dw = torch.full_like(ref[1], float("nan"))
    got = M.backward(sol.x, sol.p, sol.info.omega, g, unroll=unroll, ckpt_every=ckpt,
                     out=(du, dw), noalloc=True)
    torch.cuda.synchronize()
    return ref, got


def _close(a, b):
    # column sums are float64 LDS atomics in no fixed order: equal to rounding
    scale = float(a.abs().max())
    assert torch.isfinite(b).all()
    assert torch.allclose(b, a, rtol=1e-5, atol=1e-6 * scale), float((a - b).abs().max()) / scale


def test_noalloc_backward_matches_backward_twice(cuda):
    # first call: a 400 x 150 market (about 6000 edges), 96 steps, checkpoints every 16
    mk1, M1, s1, g1 = _solved(400, 150, 0.1, 21, cuda)
    (du_r, dw_r), (du_n, dw_n) = _both(M1, s1, g1, 96, 16)
    _close(du_r, du_n)
    _close(dw_r, dw_n)
    # second call right after, on a smaller market (the workspace keeps the
    # first call's contents): 120 x 40, 64 steps, checkpoints every 8
    mk2, M2, s2, g2 = _solved(120, 40, 0.2, 22, cuda)
    (du_r2, dw_r2), (du_n2, dw_n2) = _both(M2, s2, g2, 64, 8)
    _close(du_r2, du_n2)
    _close(dw_r2, dw_n2)
    M1.close()
    M2.close()


def test_noalloc_backward_rejects_oversized_workspace(cuda):
    # 1e6 edges with 64 steps and checkpoints every 16 need about 100 MB > 64 MiB
    mk = synth.fisher_1e8(3, 10000, 1000, 100)
    M = pdhcg.Market.from_synth(mk, device=cuda)
    x = torch.full((mk.nnz,), 1.0 / 1000.0, device=cuda)
    p = torch.ones(mk.m, device=cuda)
    g = torch.ones(mk.m)
    with pytest.raises(pdhcg.PDHCGError) as e:
        M.backward(x, p, 1.0, g, unroll=64, ckpt_every=16, noalloc=True)
    assert e.value.status == pdhcg.PDHCG_ERR_UNSUPPORTED
    assert "67108864" in str(e.value)
    M.close()
