"""Benchmark: time to relative KKT <= 1e-4 on the 1e8-edge linear Fisher
market (n = 1e6 buyers, m = 1e4 goods, 100 goods per buyer) on one GPU.

A step is one complete solve (restarted PDHCG, Alg. 2 with the Sec. 5
enhancements) from the default cold start to the tolerance, with the market
already resident in HBM.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E
PROFILE_COUNTERS = os.path.join(ROOT, "profiles", "row_pass_fisher1e8_counters.json")
KERNEL_SRCS = [os.path.join(ROOT, "paper_2506_06258_amd", "csrc", f)
               for f in ("pdhcg_kernels.hip", "pdhcg_device.h", "pdhcg_internal.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """Hash of the sources the row kernel is compiled from."""
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(n_launch_bytes_key="row_pass"):
    """HBM bytes per row-pass launch from the committed counter summary, or
    None when it is missing or was taken on a different kernel source."""
    try:
        prof = json.load(open(PROFILE_COUNTERS))
    except (OSError, ValueError):
        return None
    if prof.get("kernel_source_sha256_16") != kernel_hash():
        return None
    return prof.get("bytes_per_launch")


def batched_leg(args, pdhcg, synth, torch):
    """Markets/s of one persistent launch over many independent markets
    against solving a spread sample of the same markets one call at a time,
    both to the same relative KKT tolerance."""
    t0 = time.time()
    bt = synth.batch_markets(args.batch_markets, args.seed + 1000)
    nnz = int(len(bt.col))
    log(f"batch of {bt.count} markets generated in {time.time() - t0:.1f}s, nnz={nnz}")
    B = pdhcg.Batch(bt, device=torch.device("cuda:0"))
    prm = pdhcg.pdhcg_default_params(tol=args.tol, max_iter=200000)
    t0 = time.time()
    sch = B.autotune(prm, trial_iters=64)  # schedule choice, outside the timed region
    log(f"batch schedule {sch.as_dict()} tuned in {time.time() - t0:.2f}s")
    st, _, _, infos = B.solve(prm)  # warmup
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st, p, _, infos = B.solve(prm)
    torch.cuda.synchronize()
    dt_b = time.perf_counter() - t1
    iters_b = np.array([i.iters for i in infos])
    kkt_b = max(i.rel_kkt for i in infos)
    ok_b = sum(1 for i in infos if i.status == pdhcg.PDHCG_OK)
    log(f"batched: {dt_b:.3f}s for {bt.count} markets, {ok_b} converged, max kkt {kkt_b:.2e}")
    B.close()

    k = max(1, min(args.loop_markets, bt.count))
    pick = np.linspace(0, bt.count - 1, k).round().astype(int)
    Ms = [pdhcg.Market.from_synth(bt.market(int(b)), device=torch.device("cuda:0")) for b in pick]
    for M in Ms[:2]:
        M.solve(prm)  # warmup
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kkt_l, iters_l, ok_l = 0.0, [], 0
    for M in Ms:
        s = M.solve(prm)
        kkt_l = max(kkt_l, s.info.rel_kkt)
        iters_l.append(s.info.iters)
        ok_l += int(s.info.status == pdhcg.PDHCG_OK)
    torch.cuda.synchronize()
    dt_l = time.perf_counter() - t1
    for M in Ms:
        M.close()
    log(f"looped: {dt_l:.3f}s for {k} markets, {ok_l} converged, max kkt {kkt_l:.2e}")
    mps_b = bt.count / dt_b
    mps_l = k / dt_l
    return {
        "workload": (f"{bt.count} independent linear Fisher markets, n~logU[64,8192], "
                     f"m~logU[16,2048], density~U(5%,30%), u~U(0.01,1), w~U(0.5,1.5), "
                     f"seed {args.seed + 1000}, total nnz {nnz}; rel. KKT <= {args.tol:g}"),
        "batched_markets_per_s": mps_b,
        "batched_seconds": dt_b,
        "batched_converged": ok_b,
        "batched_max_rel_kkt": kkt_b,
        "batched_iters_median": float(np.median(iters_b)),
        "batched_iters_max": int(iters_b.max()),
        "batched_schedule": sch.as_dict(),
        "batched_longest_market_s": float(max(i.seconds for i in infos)),
        "looped_markets_per_s": mps_l,
        "looped_sample": f"{k} markets evenly spaced through the batch, one pdhcg_solve call each",
        "looped_seconds": dt_l,
        "looped_converged": ok_l,
        "looped_max_rel_kkt": kkt_l,
        "speedup": mps_b / mps_l,
    }


def backward_leg(args, M, mk, s, pdhcg, torch):
    """Reverse mode (pdhcg_backward) through `backward_unroll` fixed-step
    iterations from the solution, checkpoints every 16: one forward sweep,
    one recomputed forward pass and one adjoint pass per step."""
    K = args.backward_unroll
    g = torch.randn(mk.m, device=M.device, generator=torch.Generator(device=M.device).manual_seed(7))
    M.backward(s.x, s.p, s.info.omega, g, unroll=4, ckpt_every=2)  # warmup
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    M.backward(s.x, s.p, s.info.omega, g, unroll=K, ckpt_every=16)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    # per step: two forward passes without the average (u 4, id 2, x read 4,
    # x write 4 B/edge) and one adjoint pass (u 4, id 2, x 4, R in 4, R out 4,
    # dL/du read and write 8 B/edge)
    per_edge = 2 * 14 + 26
    log(f"backward: {K} unrolled steps in {dt:.3f}s")
    return {"workload": f"pdhcg_backward on the same market, {K} unrolled fixed steps, "
                        "checkpoints every 16, from the timed solve's point",
            "seconds": dt, "ms_per_step": 1e3 * dt / K,
            "alg_bytes_per_step": per_edge * mk.nnz,
            "achieved_GBs": per_edge * mk.nnz * K / dt / 1e9}


def exchange_leg(pdhcg, synth, torch):
    """Arrow-Debreu fixed point (Sec. 4) on n = m = 1e5 (5e6 utility edges),
    warm-started inner solves to rel. KKT 1e-7, outer tolerance 1e-6."""
    mk = synth.arrow_debreu_1e5()
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    inner = pdhcg.pdhcg_default_params(tol=1e-7, max_iter=200000)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = M.arrow_debreu(mk.e_row_ptr, mk.e_col, mk.e_val, np.ones(mk.n, np.float32), inner,
                         outer_tol=1e-6, outer_max=400)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    M.close()
    log(f"exchange: {dt:.3f}s, {res['outer']} outer / {res['inner']} inner iterations")
    return {"workload": "Arrow-Debreu fixed point, n = m = 1e5, 50 utility edges and 5 endowed goods "
                        "per agent; inner rel. KKT 1e-7, outer rel. price change 1e-6",
            "seconds": dt, "status": int(res["status"]), "outer_iterations": int(res["outer"]),
            "inner_iterations": int(res["inner"]),
            "ms_per_inner_iteration": 1e3 * dt / max(int(res["inner"]), 1)}


def skewed_leg(args, pdhcg, synth, torch):
    """The skewed market (n = 4e6, m = 2e5, Zipf(1.5) degrees, 1/rank
    popularity) to rel. KKT 1e-4."""
    t0 = time.time()
    mk = synth.fisher_skewed(workers=12)
    log(f"skewed market generated in {time.time() - t0:.1f}s, nnz={mk.nnz}")
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    prm = pdhcg.pdhcg_default_params(tol=args.tol, max_iter=20000, timing=1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    s = M.solve(prm)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    info = s.info
    M.close()
    log(f"skewed: {dt:.3f}s, {info.iters} iterations, kkt {info.rel_kkt:.2e}")
    return {"workload": f"skewed linear Fisher market, n={mk.n}, m={mk.m}, nnz={mk.nnz}; "
                        f"rel. KKT <= {args.tol:g}",
            "seconds": dt, "iterations": int(info.iters), "final_rel_kkt": float(info.rel_kkt),
            "row_pass_ms": 1e3 * info.row_pass_seconds / max(info.row_pass_launches, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--buyers", type=int, default=1_000_000)
    ap.add_argument("--goods", type=int, default=10_000)
    ap.add_argument("--degree", type=int, default=100)
    ap.add_argument("--cpu-iters", type=int, default=3,
                    help="oracle iterations timed for the CPU baseline (0: skip)")
    ap.add_argument("--batch-markets", type=int, default=4096,
                    help="markets of the batched leg (0: skip)")
    ap.add_argument("--backward-unroll", type=int, default=64,
                    help="unrolled steps of the reverse-mode leg on the same market (0: skip)")
    ap.add_argument("--exchange", type=int, default=1,
                    help="run the Arrow-Debreu leg (1e5 agents and goods; 0: skip)")
    ap.add_argument("--skewed", type=int, default=0,
                    help="run the skewed-market leg (4e6 x 2e5, 4.5e8 edges; about a minute)")
    ap.add_argument("--loop-markets", type=int, default=32,
                    help="markets of the batch solved one call at a time for the looped rate")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_2506_06258_amd import pdhcg, synth

    t0 = time.time()
    mk = synth.fisher_1e8(args.seed, args.buyers, args.goods, args.degree)
    log(f"generated {mk.name}: nnz={mk.nnz} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.time()
    M = pdhcg.Market.from_synth(mk, device=dev)
    torch.cuda.synchronize()
    log(f"market created in {time.time() - t0:.1f}s; bins={M.bins()}")

    prm = pdhcg.pdhcg_default_params(tol=args.tol, max_iter=20000, timing=1)
    for w in range(args.warmup):
        s = M.solve(prm)
        log(f"warmup {w}: iters={s.info.iters} kkt={s.info.rel_kkt:.2e} "
            f"t={s.info.seconds:.3f}s")
    times, infos = [], []
    torch.cuda.synchronize()
    for k in range(args.steps):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s = M.solve(prm)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        times.append(dt)
        infos.append(s.info)
        log(f"step {k}: {dt:.4f}s iters={s.info.iters} kkt={s.info.rel_kkt:.2e} "
            f"restarts={s.info.restarts} rounds_mean={s.info.search_rounds_mean:.2f}")
        if s.info.status != pdhcg.PDHCG_OK:
            log(f"solve ended with status {s.info.status}")
    p = s.p.double().cpu().numpy()
    psum_err = abs(p.sum() - float(mk.w.astype(np.float64).sum())) / float(mk.w.sum())

    mean_t = float(np.mean(times))
    iters = int(np.mean([i.iters for i in infos]))
    launches = sum(i.row_pass_launches for i in infos)
    row_sec = sum(i.row_pass_seconds for i in infos)
    avg_launch = row_sec / max(launches, 1)
    # per edge: u, x read, x written, average read and written (4 B each) and
    # the good id (2 B when every good sits in LDS, else 4 B); per buyer the
    # row pointer and budget; per good its price
    id_bytes = 2 if M.lds_goods() == mk.m else 4
    alg_bytes = (20 + id_bytes) * mk.nnz + 8 * mk.n + 4 * mk.m
    achieved = alg_bytes / avg_launch / 1e9
    traffic = traffic_from_profile()

    cpu = None
    if args.cpu_iters > 0:
        import oracle
        oracle.build(force=False)
        u64, w64 = mk.u.astype(np.float64), mk.w.astype(np.float64)
        t1 = time.perf_counter()
        r = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u64, w64, tol=0.0,
                         max_iter=args.cpu_iters, eval_every=10**9)
        cpu_dt = time.perf_counter() - t1
        per_it = cpu_dt / max(r.iters, 1)
        cpu = {"value": per_it * iters, "unit": "s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": (f"{r.iters} FP64 oracle iterations on the same 1e8-edge market "
                          f"({per_it:.2f} s/iteration, setup included), scaled by the "
                          f"{iters} iterations the GPU solve needed to reach rel. KKT "
                          f"{args.tol:g}")}
        log(f"cpu oracle: {per_it:.3f}s/iter on {oracle.num_threads()} threads")

    backward = None
    if args.backward_unroll > 0:
        backward = backward_leg(args, M, mk, s, pdhcg, torch)

    batched = None
    if args.batch_markets > 0:
        batched = batched_leg(args, pdhcg, synth, torch)
    exchange = exchange_leg(pdhcg, synth, torch) if args.exchange else None
    skewed = skewed_leg(args, pdhcg, synth, torch) if args.skewed else None

    out = {
        "metric": "time-to-1e-4 KKT & HBM GB/s (1e8-nnz Fisher); batched vs looped markets/s",
        "value": mean_t,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * mean_t,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": (f"linear Fisher market, n={mk.n} buyers, m={mk.m} goods, "
                                f"{args.degree} uniformly random goods per buyer "
                                f"(nnz={mk.nnz}), u~LogNormal(0,1), w~U(0.5,1.5), "
                                f"seed {args.seed}; restarted PDHCG to rel. KKT <= "
                                f"{args.tol:g}"),
                   "n": mk.n, "m": mk.m, "nnz": mk.nnz, "tol": args.tol},
        "iterations": iters,
        "ms_per_iter": 1e3 * mean_t / max(iters, 1),
        "final_rel_kkt": float(infos[-1].rel_kkt),
        "price_sum_rel_err": psum_err,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": traffic,
                     "kernel": "k_row_pass (row prox + average fold + column partials)",
                     "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": 1e3 * avg_launch, "launches_timed": launches},
        "cpu_baseline": cpu,
        "batched": batched,
        "backward": backward,
        "exchange": exchange,
        "skewed": skewed,
    }
    print(json.dumps(out), flush=True)
    M.close()


if __name__ == "__main__":
    main()
