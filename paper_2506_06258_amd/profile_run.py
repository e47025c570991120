"""Workloads for rocprofv3 runs and the summaries kept with the sources.

  python -m paper_2506_06258_amd.profile_run copy  [--mib 1024] [--reps 4]
  python -m paper_2506_06258_amd.profile_run solve [--iters 64]
  python -m paper_2506_06258_amd.profile_run skewed [--iters 40]
  python -m paper_2506_06258_amd.profile_run exchange
  python -m paper_2506_06258_amd.profile_run backward [--unroll 64]
  python -m paper_2506_06258_amd.profile_run ksweep
  python -m paper_2506_06258_amd.profile_run jd
  python -m paper_2506_06258_amd.profile_run longrows [--iters 24]
  python -m paper_2506_06258_amd.profile_run table2 [--seeds 3]
  python -m paper_2506_06258_amd.profile_run pdhg
  python -m paper_2506_06258_amd.profile_run theory [--K 256] [--restarts 16]
  python -m paper_2506_06258_amd.profile_run summarize --stats DIR
  python -m paper_2506_06258_amd.profile_run counters --copy-fetch DIR --copy-write DIR \
        --fetch DIR --write DIR [--mib 1024] [--out FILE]

``copy`` runs torch's device-to-device copy of a float32 tensor of a known
size: the calibration kernel for the HBM byte counters.  ``solve`` runs a
fixed number of PDHCG iterations (fixed step, no restarts, so every
iteration launches the same kernels) on the 1e8-edge market (n = 1e6
buyers, m = 1e4 goods, 100 goods per buyer); ``skewed`` the same on the
skewed market (n = 4e6, m = 2e5, 4.5e8 edges); ``exchange`` the
Arrow-Debreu fixed point on n = m = 1e5 (inner rel. KKT 1e-7, outer 1e-6).  ``summarize`` prints the
per-kernel table of a ``--kernel-trace --stats`` run; ``counters`` turns
FETCH_SIZE / WRITE_SIZE runs (KiB per dispatch) into HBM bytes per row-pass
launch, scaled by what the same counters read for the copy of known size.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# sources the row kernel is compiled from
KERNEL_SRCS = [os.path.join(HERE, "csrc", f)
               for f in ("pdhcg_kernels.hip", "pdhcg_device.h", "pdhcg_internal.h")]
ROW_KERNEL = "k_row_pass"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def run_copy(mib: int, reps: int) -> None:
    import torch

    n = mib * (1 << 20) // 4
    src = torch.rand(n, device="cuda:0", dtype=torch.float32)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {reps} x {mib} MiB", flush=True)


def run_solve(iters: int) -> None:
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    mk = synth.fisher_1e8(1)
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    prm = pdhcg.pdhcg_default_params(tol=0.0, max_iter=iters, step_mode=pdhcg.PDHCG_STEP_FIXED,
                                     restart=pdhcg.PDHCG_RESTART_NONE, eval_every=iters)
    s = M.solve(prm)
    torch.cuda.synchronize()
    print(f"solve: {s.info.iters} iterations, rel. KKT {s.info.rel_kkt:.3e}", flush=True)
    M.close()


def run_skewed(iters: int) -> None:
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    mk = synth.fisher_skewed(workers=12)
    print(f"skewed market: nnz={mk.nnz}", flush=True)
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    prm = pdhcg.pdhcg_default_params(tol=0.0, max_iter=iters, step_mode=pdhcg.PDHCG_STEP_FIXED,
                                     restart=pdhcg.PDHCG_RESTART_NONE, eval_every=iters, timing=1)
    s = M.solve(prm)
    torch.cuda.synchronize()
    i = s.info
    print(f"skewed: {i.iters} iterations, row pass "
          f"{1e3 * i.row_pass_seconds / max(i.row_pass_launches, 1):.3f} ms", flush=True)
    M.close()


def run_exchange() -> None:
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    mk = synth.arrow_debreu_1e5()
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    inner = pdhcg.pdhcg_default_params(tol=1e-7, max_iter=200000)
    res = M.arrow_debreu(mk.e_row_ptr, mk.e_col, mk.e_val, np.ones(mk.n, np.float32), inner,
                         outer_tol=1e-6, outer_max=400)
    torch.cuda.synchronize()
    print(f"exchange: status {res['status']}, {res['outer']} outer / {res['inner']} inner "
          "iterations", flush=True)
    M.close()


def run_backward(unroll: int) -> None:
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    mk = synth.fisher_1e8(1)
    dev = torch.device("cuda:0")
    M = pdhcg.Market.from_synth(mk, device=dev)
    s = M.solve(tol=1e-4, max_iter=20000)
    g = torch.randn(mk.m, device=dev, generator=torch.Generator(device=dev).manual_seed(7))
    M.backward(s.x, s.p, s.info.omega, g, unroll=unroll, ckpt_every=16)
    torch.cuda.synchronize()
    print(f"backward: {unroll} unrolled steps", flush=True)
    M.close()


def run_ksweep() -> None:
    """The 1e8-edge market to rel. KKT 1e-4 with the paper's k-section row
    search for k = 2 ... 64 (Sec. 2.2.1, Table 1) in both mappings (one lane
    per candidate with the row in LDS; the G lanes holding a row taking the
    candidates in turn) and with the active-set search: iterations, row-pass
    time and search rounds."""
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    mk = synth.fisher_1e8(1)
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    cases = [("active set", pdhcg.PDHCG_SEARCH_ACTIVESET, 32)]
    cases += [(f"{k}-section, one lane per candidate", pdhcg.PDHCG_SEARCH_KSECTION_WAVE, k)
              for k in (2, 4, 8, 16, 32, 64)]
    cases += [(f"{k}-section, candidates in turn", pdhcg.PDHCG_SEARCH_KSECTION, k)
              for k in (2, 4, 8, 16, 32)]
    print("| search | iterations | solve s | row pass ms | mean rounds | max rounds | rel. KKT |")
    print("|---|---|---|---|---|---|---|")
    for name, search, k in cases:
        # rounds are bounded only by the bracket width (search_rtol 1e-10)
        prm = pdhcg.pdhcg_default_params(tol=1e-4, max_iter=20000, timing=1, search=search,
                                         sections=k, max_search_rounds=200)
        M.solve(prm)  # warmup
        s = M.solve(prm)
        torch.cuda.synchronize()
        i = s.info
        print(f"| {name} | {i.iters} | {i.seconds:.4f} | "
              f"{1e3 * i.row_pass_seconds / max(i.row_pass_launches, 1):.3f} | "
              f"{i.search_rounds_mean:.2f} | {i.search_rounds_max} | {i.rel_kkt:.2e} |", flush=True)
    M.close()


def run_pdhg(iters: int) -> None:
    """Restarted PDHG (Alg. 1) on the 1e8-edge market: one solve to rel.
    KKT 1e-4 (the row kernel k_pdhg_row, 24 B/edge with no root search)."""
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    mk = synth.fisher_1e8(1)
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    prm = pdhcg.pdhcg_default_params(tol=1e-4, max_iter=iters, timing=1)
    sol, _ = M.pdhg_solve(prm)
    torch.cuda.synchronize()
    i = sol.info
    print(f"pdhg: {i.iters} iterations in {i.seconds:.3f} s, rel. KKT {i.rel_kkt:.2e}, row pass "
          f"{1e3 * i.row_pass_seconds / max(i.row_pass_launches, 1):.3f} ms", flush=True)
    M.close()


def run_theory(K: int, restarts: int) -> None:
    """Alg. 2 in the setting of Sec. 3 (fixed sigma = tau = 1/(2||K||),
    restart length K, restarts to the average) on the 1e8-edge market: the
    distance of every restart point to the equilibrium prices committed in
    tests/golden (FP64, rel. KKT 7.7e-9) and its relative KKT error."""
    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    p_star = np.loadtxt(os.path.join(ROOT, "tests", "golden", "fisher_1e8_s1_prices.txt"))
    mk = synth.fisher_1e8(1)
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    sol, dist, kkt = M.solve_fixed_restart(K, restarts, p_ref=torch.tensor(p_star, dtype=torch.float32))
    torch.cuda.synchronize()
    print(f"theory mode: K = {K}, {restarts} restarts, eta = {sol.info.eta:.4e}, "
          f"{sol.info.seconds:.2f} s", flush=True)
    print("| restart n | iterations | ||p^{n,0} - p*||_2 / ||p*||_2 | ratio to previous | rel. KKT |")
    print("|---|---|---|---|---|")
    ps = float(np.linalg.norm(p_star))
    for n in range(restarts + 1):
        ratio = "" if n == 0 else f"{dist[n] / dist[n - 1]:.3f}"
        print(f"| {n} | {n * K} | {dist[n] / ps:.3e} | {ratio} | {kkt[n]:.3e} |", flush=True)
    M.close()


def run_jd() -> None:
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    mk = synth.jd_shaped(workers=12)
    print(f"jd-shaped market: n={mk.n} m={mk.m} nnz={mk.nnz}", flush=True)
    M = pdhcg.Market.from_synth(mk, device=torch.device("cuda:0"))
    print(f"bins {M.bins()}, {M.lds_goods()} goods in LDS", flush=True)
    prm = pdhcg.pdhcg_default_params(tol=1e-4, max_iter=20000, timing=1)
    M.solve(prm)  # warmup
    s = M.solve(prm)
    torch.cuda.synchronize()
    i = s.info
    print(f"jd-shaped: {i.iters} iterations in {i.seconds:.3f} s, row pass "
          f"{1e3 * i.row_pass_seconds / max(i.row_pass_launches, 1):.3f} ms, rel. KKT {i.rel_kkt:.2e}",
          flush=True)
    M.close()


# Table 2 of the paper (Sec. 5.1): PDHCG to relative KKT 1e-4 on one
# NVIDIA H100 (Julia/CUDA), geometric means over 10 random instances:
# (n, m, q) -> (iterations, seconds).
TABLE2 = [((1000, 400, 0.2), (2612, 1.7)), ((10000, 4000, 0.02), (2758, 3.6)),
          ((100000, 4000, 0.02), (1200, 8.3)), ((1000000, 4000, 0.02), (2283, 116.3)),
          ((10000000, 4000, 0.01), (2423, 589.7))]


def run_table2(seeds: int) -> None:
    """The markets of Table 2 (synth.table2_market), restarted PDHCG to rel.
    KKT 1e-4 with default parameters: iterations and seconds per instance
    (a short solve first loads the kernels), the paper's figures beside."""
    import math

    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    dev = torch.device("cuda:0")
    print("| n | m | q | nnz | instances | iterations (geo. mean) | seconds (geo. mean) | "
          "paper iterations | paper seconds (H100) |")
    print("|---|---|---|---|---|---|---|---|---|")
    for (n, m, q), (pit, psec) in TABLE2:
        its, secs, nnz = [], [], 0
        for seed in range(seeds):
            mk = synth.table2_market(n, m, q, seed)
            nnz = mk.nnz
            M = pdhcg.Market.from_synth(mk, device=dev)
            M.solve(tol=1e-4, max_iter=64)
            torch.cuda.synchronize()
            s = M.solve(tol=1e-4, max_iter=100000)
            torch.cuda.synchronize()
            assert s.info.status == pdhcg.PDHCG_OK, s.info.status
            its.append(s.info.iters)
            secs.append(s.info.seconds)
            M.close()
            del mk
        gi = math.exp(sum(math.log(v) for v in its) / len(its))
        gs = math.exp(sum(math.log(v) for v in secs) / len(secs))
        print(f"| {n} | {m} | {q:g} | {nnz} | {seeds} | {gi:.0f} | {gs:.3f} | {pit} | {psec} |",
              flush=True)


def run_longrows(iters: int) -> None:
    """Row pass of markets whose rows all exceed 512 entries (fixed degree
    800, 1500, 3000, 6000 and 12000), every good in LDS and 1024 goods in LDS, the long
    rows in registers of teams of waves (PDHCG_TEAM=2) and on the
    one-wave-per-row kernel (PDHCG_TEAM=0): fixed-step iterations, row-pass
    time from the solver's HIP events."""
    import torch

    sys.path.insert(0, ROOT)
    from paper_2506_06258_amd import pdhcg, synth

    dev = torch.device("cuda:0")
    cases = [(120000, 800, 1500), (100000, 1500, 2500), (60000, 3000, 4000), (30000, 6000, 8000),
             (20000, 12000, 13000)]
    print("| n | entries per row | m | goods in LDS | long-row kernel | row pass ms | G entries/s |")
    print("|---|---|---|---|---|---|---|")
    for n, d, m in cases:
        mk = synth.fixed_degree_market(n, m, d, 7, "uniform").as_float32()
        for hot in (None, 1024):
            for team in ("2", "0"):
                os.environ["PDHCG_TEAM"] = team
                if hot:
                    os.environ["PDHCG_HOT"] = str(hot)
                M = pdhcg.Market.from_synth(mk, device=dev)
                os.environ.pop("PDHCG_HOT", None)
                os.environ.pop("PDHCG_TEAM", None)
                prm = pdhcg.pdhcg_default_params(tol=0.0, max_iter=iters, timing=1,
                                                 eval_every=100000, step_mode=0, restart=0)
                M.solve(prm)
                s = M.solve(prm)
                per = s.info.row_pass_seconds / max(s.info.row_pass_launches, 1)
                kern = "teams of waves" if team == "2" else "one wave per row"
                print(f"| {n} | {d} | {m} | {M.lds_goods()} | {kern} | {per * 1e3:.3f} | "
                      f"{mk.nnz / per / 1e9:.1f} |", flush=True)
                M.close()


def _rows(path_glob: str):
    files = sorted(glob.glob(path_glob, recursive=True))
    if not files:
        raise SystemExit(f"no file matches {path_glob}")
    with open(files[0], newline="") as f:
        return list(csv.DictReader(f))


def _key(row: dict, *names: str) -> str:
    for n in names:
        for k in row:
            if k.lower() == n.lower():
                return k
    raise KeyError(names)


def short_name(name: str) -> str:
    base = name.split("(")[0]
    for tok in ("pdhcg::", "void "):
        base = base.replace(tok, "")
    return base.strip()


def summarize(stats_dir: str) -> str:
    rows = _rows(os.path.join(stats_dir, "**", "*kernel_stats.csv"))
    kn = _key(rows[0], "Name", "Kernel_Name")
    lines = ["| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append("| {} | {} | {:.3f} | {:.2f} | {:.2f} | {:.2f} | {:.2f} |".format(
            short_name(r[kn]), r[_key(r, "Calls")], float(r[_key(r, "TotalDurationNs")]) / 1e6,
            float(r[_key(r, "AverageNs")]) / 1e3, float(r[_key(r, "MinNs")]) / 1e3,
            float(r[_key(r, "MaxNs")]) / 1e3, float(r[_key(r, "Percentage")])))
    return "\n".join(lines)


def counter_per_dispatch(run_dir: str, counter: str, kernel: str) -> list[float]:
    rows = _rows(os.path.join(run_dir, "**", "*counter_collection.csv"))
    kn = _key(rows[0], "Kernel_Name")
    cn = _key(rows[0], "Counter_Name")
    cv = _key(rows[0], "Counter_Value")
    di = _key(rows[0], "Dispatch_Id", "Dispatch_ID")
    per = {}
    for r in rows:
        if kernel in r[kn] and r[cn] == counter:
            per[r[di]] = per.get(r[di], 0.0) + float(r[cv])
    if not per:
        raise SystemExit(f"no {counter} rows for a kernel named like {kernel} in {run_dir}")
    return list(per.values())


def counters(args) -> dict:
    copy_bytes = args.mib * (1 << 20)
    cf = statistics.median(counter_per_dispatch(args.copy_fetch, "FETCH_SIZE", args.copy_kernel))
    cw = statistics.median(counter_per_dispatch(args.copy_write, "WRITE_SIZE", args.copy_kernel))
    rf = counter_per_dispatch(args.fetch, "FETCH_SIZE", ROW_KERNEL)
    rw = counter_per_dispatch(args.write, "WRITE_SIZE", ROW_KERNEL)
    f_scale = copy_bytes / (cf * 1024.0)  # bytes per counted KiB
    w_scale = copy_bytes / (cw * 1024.0)
    fetch = statistics.median(rf) * 1024.0 * f_scale
    write = statistics.median(rw) * 1024.0 * w_scale
    return {
        "kernel": ROW_KERNEL,
        "workload": "1e8-edge Fisher market (n=1e6, m=1e4, 100 goods per buyer), fixed step",
        "kernel_source_sha256_16": kernel_source_hash(),
        "copy_calibration": {"bytes": copy_bytes, "fetch_kib": cf, "write_kib": cw,
                             "fetch_scale": f_scale, "write_scale": w_scale},
        "row_pass_dispatches": len(rf),
        "fetch_kib_median": statistics.median(rf),
        "write_kib_median": statistics.median(rw),
        "fetch_bytes_per_launch": fetch,
        "write_bytes_per_launch": write,
        "bytes_per_launch": fetch + write,
    }


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("copy")
    c.add_argument("--mib", type=int, default=1024)
    c.add_argument("--reps", type=int, default=4)
    s = sub.add_parser("solve")
    s.add_argument("--iters", type=int, default=64)
    k2 = sub.add_parser("skewed")
    k2.add_argument("--iters", type=int, default=40)
    sub.add_parser("exchange")
    sub.add_parser("ksweep")
    sub.add_parser("jd")
    t2 = sub.add_parser("table2")
    t2.add_argument("--seeds", type=int, default=3)
    lr = sub.add_parser("longrows")
    lr.add_argument("--iters", type=int, default=24)
    pg = sub.add_parser("pdhg")
    pg.add_argument("--iters", type=int, default=200000)
    th = sub.add_parser("theory")
    th.add_argument("--K", type=int, default=256)
    th.add_argument("--restarts", type=int, default=16)
    bw = sub.add_parser("backward")
    bw.add_argument("--unroll", type=int, default=64)
    m = sub.add_parser("summarize")
    m.add_argument("--stats", required=True)
    k = sub.add_parser("counters")
    k.add_argument("--copy-fetch", required=True)
    k.add_argument("--copy-write", required=True)
    k.add_argument("--fetch", required=True)
    k.add_argument("--write", required=True)
    k.add_argument("--mib", type=int, default=1024)
    k.add_argument("--copy-kernel", default="copy")
    k.add_argument("--out", default=None)
    a = ap.parse_args()
    if a.cmd == "copy":
        run_copy(a.mib, a.reps)
    elif a.cmd == "solve":
        run_solve(a.iters)
    elif a.cmd == "skewed":
        run_skewed(a.iters)
    elif a.cmd == "exchange":
        run_exchange()
    elif a.cmd == "backward":
        run_backward(a.unroll)
    elif a.cmd == "ksweep":
        run_ksweep()
    elif a.cmd == "jd":
        run_jd()
    elif a.cmd == "table2":
        run_table2(a.seeds)
    elif a.cmd == "longrows":
        run_longrows(a.iters)
    elif a.cmd == "pdhg":
        run_pdhg(a.iters)
    elif a.cmd == "theory":
        run_theory(a.K, a.restarts)
    elif a.cmd == "summarize":
        print(summarize(a.stats))
    else:
        res = counters(a)
        text = json.dumps(res, indent=1)
        if a.out:
            with open(a.out, "w") as f:
                f.write(text + "\n")
        print(text)


if __name__ == "__main__":
    main()
