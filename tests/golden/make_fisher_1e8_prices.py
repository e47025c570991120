"""Write the reference equilibrium prices of the 1e8-edge linear Fisher market.

The market is ``synth.fisher_1e8(seed)``: n = 1e6 buyers, m = 1e4 goods,
exactly 100 uniformly random goods per buyer, u ~ LogNormal(0, 1) and
w ~ U(0.5, 1.5) in float32.  The prices come from the FP64 CPU oracle only
(restarted PDHCG, Alg. 2 with the Sec. 5 enhancements, exact row prox of
Sec. 2.2), solved to relative KKT <= 1e-8 (Sec. 5 Criteria).  Equilibrium
prices are unique (Sec. 3, Fact 1), so any solver that reaches the
equilibrium must reproduce them.

Outputs (beside this script):
  fisher_1e8_s{seed}_prices.txt  one price per line (%.17g), good order;
  fisher_1e8_s{seed}_prices.json iterations, wall times, thread count, CPU
                                 model, final KKT residuals, and the oracle's
                                 time and iterations to relative KKT 1e-4.

Usage: python tests/golden/make_fisher_1e8_prices.py [--seed 1] [--tol 1e-8]
Takes about an hour on 8 cores (two oracle solves: to 1e-4 and to tol).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2506_06258_amd import synth  # noqa: E402


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=40000)
    ap.add_argument("--skip-1e4", action="store_true",
                    help="do not time the separate solve to rel. KKT 1e-4")
    args = ap.parse_args()
    oracle.build(force=False)

    t0 = time.time()
    mk = synth.fisher_1e8(args.seed)
    print(f"market {mk.name}: nnz={mk.nnz}, generated in {time.time() - t0:.1f}s", flush=True)
    u = mk.u.astype(np.float64)
    w = mk.w.astype(np.float64)
    meta = {"market": mk.name, "n": mk.n, "m": mk.m, "nnz": mk.nnz, "seed": args.seed,
            "threads": oracle.num_threads(), "cpu_model": cpu_model()}

    if not args.skip_1e4:
        t1 = time.perf_counter()
        r4 = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u, w, tol=1e-4, max_iter=args.max_iter)
        dt4 = time.perf_counter() - t1
        meta["to_1e-4"] = {"seconds": dt4, "iterations": r4.iters, "status": r4.status,
                           "rel_kkt": r4.rel_kkt, "restarts": r4.restarts}
        print(f"to 1e-4: {dt4:.1f}s, {r4.iters} iterations, kkt {r4.rel_kkt:.3e}", flush=True)

    t1 = time.perf_counter()
    r = oracle.solve(mk.n, mk.m, mk.row_ptr, mk.col, u, w, tol=args.tol, max_iter=args.max_iter,
                     verbose=1)
    dt = time.perf_counter() - t1
    print(f"to {args.tol:g}: {dt:.1f}s, {r.iters} iterations, status {r.status}, "
          f"kkt {r.rel_kkt:.3e}", flush=True)
    if r.status != oracle.OK:
        raise SystemExit(f"oracle did not reach {args.tol:g} (status {r.status})")
    # certificate on the returned point (same metric, recomputed)
    uh, _ = oracle.normalize_rows(mk.row_ptr, u)
    k, parts = oracle.kkt(mk.n, mk.m, mk.row_ptr, mk.col, uh, w, r.x, r.p)
    meta.update({"tol": args.tol, "seconds": dt, "iterations": r.iters, "restarts": r.restarts,
                 "rel_kkt": k, "rel_primal": parts[0], "rel_dual": parts[1],
                 "rel_gap": parts[2], "sum_p": float(r.p.sum()), "sum_w": float(w.sum())})
    base = os.path.join(HERE, f"fisher_1e8_s{args.seed}_prices")
    np.savetxt(base + ".txt", r.p, fmt="%.17g",
               header=f"equilibrium prices of {mk.name} (FP64 oracle, rel. KKT {k:.3e})")
    with open(base + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    main()
