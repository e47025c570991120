"""Seeded synthetic linear Fisher / Arrow-Debreu market instances.

This module only draws inputs: sparsity patterns, utilities, budgets and
endowments.  It holds none of the solver's arithmetic, so the CPU oracle and
the HIP path can both be fed from it without sharing any of the method.

Every generator is deterministic in its ``seed`` (numpy PCG64) and returns a
:class:`Market` whose CSR rows list strictly increasing good indices, which is
the layout the C ABI expects.

Workloads (shapes follow the paper's synthetic experiments, Sec. 5.1 and 5.3:
many more buyers than goods, sparse utilities):

* ``bernoulli_market``  - each (i, j) is an edge with probability ``density``;
  buyers or goods left without an edge receive one uniformly random edge
  (Assumption 1 of Sec. 2 then holds).
* ``fixed_degree_market`` - every buyer values exactly ``d`` distinct goods
  drawn uniformly without replacement.
* ``zipf_market`` - skewed buyer degrees and popularity-skewed goods.
* ``batch_markets`` - many independent markets of uneven sizes.
* ``arrow_debreu_market`` - a utility matrix plus a sparse endowment matrix
  whose columns sum to one (Sec. 4).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Market:
    """A linear Fisher market in CSR form (buyers are rows, goods columns)."""

    n: int
    m: int
    row_ptr: np.ndarray  # int32 [n+1]
    col: np.ndarray  # int32 [nnz], strictly increasing inside each row
    u: np.ndarray  # utilities u_ij > 0 on the stored entries
    w: np.ndarray  # budgets w_i > 0 [n]
    name: str = ""
    # Arrow-Debreu endowments (CSR, same n x m shape), optional
    e_row_ptr: Optional[np.ndarray] = None
    e_col: Optional[np.ndarray] = None
    e_val: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64 [nnz])."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def as_float32(self) -> "Market":
        """Same market with u, w (and E) rounded to float32.

        Parity tests hand the rounded values to both sides (the oracle reads
        them as float64), so both solve exactly the same instance."""
        return Market(
            self.n, self.m, self.row_ptr, self.col,
            self.u.astype(np.float32), self.w.astype(np.float32), self.name,
            self.e_row_ptr, self.e_col,
            None if self.e_val is None else self.e_val.astype(np.float32),
            dict(self.meta))


def _csr_from_mask(mask: np.ndarray):
    rows, cols = np.nonzero(mask)  # row-major order: cols increase per row
    n = mask.shape[0]
    counts = np.bincount(rows, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return row_ptr.astype(np.int32), cols.astype(np.int32)


def bernoulli_market(n: int, m: int, density: float, seed: int,
                     u_low: float = 0.01, u_high: float = 1.0,
                     w_mode: str = "ones", dtype=np.float64,
                     name: str = "") -> Market:
    """Each (i, j) is an edge with probability ``density``.

    Buyers or goods without an edge get one uniformly random edge.
    u ~ Uniform(u_low, u_high); budgets are all one (``w_mode='ones'``,
    the equal-income case of Sec. 1) or Uniform(0.5, 1.5)
    (``w_mode='uniform'``)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((n, m)) < density
    empty_rows = np.nonzero(~mask.any(axis=1))[0]
    if empty_rows.size:
        mask[empty_rows, rng.integers(0, m, size=empty_rows.size)] = True
    empty_cols = np.nonzero(~mask.any(axis=0))[0]
    if empty_cols.size:
        mask[rng.integers(0, n, size=empty_cols.size), empty_cols] = True
    row_ptr, col = _csr_from_mask(mask)
    u = rng.uniform(u_low, u_high, size=col.size).astype(dtype)
    if w_mode == "ones":
        w = np.ones(n, dtype=dtype)
    elif w_mode == "uniform":
        w = rng.uniform(0.5, 1.5, size=n).astype(dtype)
    else:
        raise ValueError(f"unknown w_mode {w_mode!r}")
    return Market(n, m, row_ptr, col, u, w, name or f"bernoulli-{n}x{m}-q{density}-s{seed}")


def _distinct_sorted_rows(rng, n: int, d: int, m: int) -> np.ndarray:
    """n rows of d distinct goods in [0, m), each row sorted.

    Draw with replacement, then redraw repeated values until every row is
    duplicate-free.  The procedure is symmetric under relabelling the goods,
    so every row is a uniformly random d-subset."""
    if d > m:
        raise ValueError("d > m")
    C = rng.integers(0, m, size=(n, d), dtype=np.int32)
    C.sort(axis=1)
    while True:
        dup = np.zeros(C.shape, dtype=bool)
        dup[:, 1:] = C[:, 1:] == C[:, :-1]
        bad = np.nonzero(dup.any(axis=1))[0]
        if bad.size == 0:
            return C
        sub = C[bad]
        sdup = dup[bad]
        sub[sdup] = rng.integers(0, m, size=int(sdup.sum()), dtype=np.int32)
        sub.sort(axis=1)
        C[bad] = sub


def fixed_degree_market(n: int, m: int, d: int, seed: int,
                        u_dist: str = "lognormal", w_low: float = 0.5,
                        w_high: float = 1.5, dtype=np.float32,
                        name: str = "") -> Market:
    """Every buyer values exactly ``d`` distinct uniformly random goods.

    u ~ LogNormal(0, 1) (``u_dist='lognormal'``) or Uniform(0.01, 1);
    w ~ Uniform(w_low, w_high)."""
    rng = np.random.default_rng(seed)
    C = _distinct_sorted_rows(rng, n, d, m)
    col = C.reshape(-1)
    deg = np.bincount(col, minlength=m)
    if (deg == 0).any():
        raise RuntimeError("a good received no buyer; raise n*d relative to m")
    row_ptr = (np.arange(n + 1, dtype=np.int64) * d).astype(np.int32)
    if u_dist == "lognormal":
        u = np.exp(rng.standard_normal(col.size, dtype=np.float32 if dtype == np.float32 else np.float64))
    elif u_dist == "uniform":
        u = rng.uniform(0.01, 1.0, size=col.size)
    else:
        raise ValueError(u_dist)
    u = u.astype(dtype)
    w = rng.uniform(w_low, w_high, size=n).astype(dtype)
    return Market(n, m, row_ptr, col, u, w, name or f"fixdeg-{n}x{m}-d{d}-s{seed}")


def table2_market(n: int, m: int, q: float, seed: int, dtype=np.float32) -> Market:
    """The synthetic Fisher markets of the paper's Table 2 (Sec. 5.1): buyer i
    values each good independently with probability q (row degree
    d_i ~ Binomial(m, q), at least 1, goods uniform and distinct), u_ij ~ U(0, 1)
    on the stored entries, w_i ~ U(0, 1)."""
    rng = np.random.default_rng([seed, 2])
    deg = np.maximum(rng.binomial(m, q, size=n), 1).astype(np.int64)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(deg, out=row_ptr[1:])
    col = np.empty(int(row_ptr[-1]), np.int32)
    order = np.argsort(deg, kind="stable")
    sdeg = deg[order]
    bounds = np.flatnonzero(np.diff(sdeg)) + 1
    for grp in np.split(order, bounds):
        d = int(deg[grp[0]])
        C = _distinct_sorted_rows(rng, grp.size, d, m)
        idx = (row_ptr[grp][:, None] + np.arange(d)[None, :]).reshape(-1)
        col[idx] = C.reshape(-1)
    if (np.bincount(col, minlength=m) == 0).any():
        raise RuntimeError("a good received no buyer; raise n q")
    u = rng.uniform(0.0, 1.0, size=col.size).astype(dtype)
    u = np.maximum(u, np.finfo(np.float32).tiny).astype(dtype)
    w = rng.uniform(0.0, 1.0, size=n).astype(dtype)
    w = np.maximum(w, np.finfo(np.float32).tiny).astype(dtype)
    return Market(n, m, row_ptr.astype(np.int32), col, u, w, f"table2-{n}x{m}-q{q:g}-s{seed}")


def _zipf_rows(args):
    """Goods of one block of rows of zipf_market (see there)."""
    seed, block, d, m, ranking = args
    rng = np.random.default_rng([seed, 7, block])
    n = d.size
    logm = np.log(m + 1.0)

    def draw(cnt):
        # inverse CDF of the density 1/x on [1, m + 1): rank = floor(x) - 1
        x = np.exp(rng.uniform(0.0, logm, size=cnt))
        return ranking[np.minimum(np.floor(x).astype(np.int64) - 1, m - 1)]

    rows = np.repeat(np.arange(n, dtype=np.int64), d)
    keys = np.unique(rows * m + draw(rows.size))
    for rnd in range(65):
        short = d - np.bincount(keys // m, minlength=n)
        if not short.any():
            break
        r2 = np.repeat(np.arange(n, dtype=np.int64), short)
        g2 = draw(r2.size) if rnd < 64 else rng.integers(0, m, size=r2.size)
        k2 = np.unique(r2 * m + g2)
        pos = np.minimum(np.searchsorted(keys, k2), keys.size - 1)
        k2 = k2[keys[pos] != k2]
        # at most the shortfall of each row, chosen in random order
        pri = rng.random(k2.size)
        order = np.lexsort((pri, k2 // m))
        k2 = k2[order]
        r = k2 // m
        first = np.searchsorted(r, np.arange(n))
        k2 = k2[(np.arange(k2.size) - first[r]) < short[r]]
        keys = np.union1d(keys, k2)
    u = np.exp(rng.standard_normal(keys.size))
    return keys // m, keys % m, u


def zipf_market(n: int, m: int, seed: int, a: float = 1.5, dmin: int = 5, dmax: int = 20000,
                dtype=np.float32, name: str = "", workers: int = 0,
                block_rows: int = 1 << 16, uniform_degrees: bool = False) -> Market:
    """Skewed buyer degrees and popularity-skewed goods.

    Degrees d = dmin - 1 + K with K ~ Zipf(a), redrawn while d > dmax (the
    reading of "Zipf(1.5) truncated to [5, 20000]" that gives a mean degree
    of about 112).  Each buyer's d distinct goods are drawn with probability
    proportional to 1/(rank + 1) over a random ranking of the goods: draws
    with replacement, repeated goods dropped and the shortfall drawn again
    (at most 64 rounds, then uniformly random goods fill what is left).
    Goods that no buyer drew receive one random buyer (Assumption 1).
    u ~ LogNormal(0, 1), w ~ U(0.5, 1.5).  Blocks of ``block_rows`` rows
    have generators of their own, so ``workers`` (processes, 0 = serial)
    does not change the result."""
    rng = np.random.default_rng(seed)
    d = np.empty(n, np.int64)
    if uniform_degrees:  # degrees uniform on [dmin, dmax] instead
        d[:] = rng.integers(dmin, dmax + 1, size=n)
    todo = np.arange(0 if uniform_degrees else n)
    while todo.size:
        k = rng.zipf(a, size=todo.size)
        ok = k <= dmax - dmin + 1
        d[todo[ok]] = dmin - 1 + k[ok]
        todo = todo[~ok]
    d = np.minimum(d, m)
    ranking = rng.permutation(m).astype(np.int64)  # rank -> good
    w = rng.uniform(0.5, 1.5, size=n).astype(dtype)
    jobs = [(seed, b, d[b * block_rows:(b + 1) * block_rows], m, ranking)
            for b in range((n + block_rows - 1) // block_rows)]
    if workers > 1 and len(jobs) > 1:
        # fresh interpreters, not forks: callers may already hold a GPU
        # context, which a forked child must not inherit
        from multiprocessing import get_context
        with get_context("spawn").Pool(workers) as pool:
            parts = pool.map(_zipf_rows, jobs)
    else:
        parts = [_zipf_rows(j) for j in jobs]
    counts = np.zeros(n, np.int64)
    for b, (r, _, _) in enumerate(parts):
        counts[b * block_rows:b * block_rows + jobs[b][2].size] = np.bincount(r, minlength=jobs[b][2].size)
    col = np.concatenate([c for _, c, _ in parts]).astype(np.int32)
    u = np.concatenate([x for _, _, x in parts]).astype(dtype)
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    missing = np.nonzero(np.bincount(col, minlength=m) == 0)[0]
    if missing.size:
        # one random buyer for every good nobody drew, inserted in column order
        rows = np.repeat(np.arange(n, dtype=np.int64), counts)
        buyers = rng.integers(0, n, size=missing.size)
        keys = np.concatenate([rows * m + col, buyers * m + missing])
        vals = np.concatenate([u, np.exp(rng.standard_normal(missing.size)).astype(dtype)])
        keys, idx = np.unique(keys, return_index=True)
        u = vals[idx]
        col = (keys % m).astype(np.int32)
        np.cumsum(np.bincount(keys // m, minlength=n), out=row_ptr[1:])
    return Market(n, m, row_ptr.astype(np.int32), col, u, w,
                  name or f"zipf-{n}x{m}-a{a}-d{dmin}..{dmax}-s{seed}")


def fisher_skewed(seed: int = 2, n: int = 4_000_000, m: int = 200_000,
                  workers: int = 8) -> Market:
    """The skewed workload: n=4e6 buyers, m=2e5 goods, Zipf(1.5) degrees in
    [5, 20000], 1/rank popularity of goods (about 4.5e8 edges)."""
    return zipf_market(n, m, seed, 1.5, 5, 20000, np.float32,
                       name=f"fisher-skewed-{n}x{m}-s{seed}", workers=workers)


def jd_shaped(seed: int = 5, n: int = 2_560_000, m: int = 27_000, workers: int = 8) -> Market:
    """A market of the shape of the e-commerce data of Sec. 5.2 (shape only,
    no data): n = 2.56e6 buyers, m = 27,000 goods, 3-70 goods per buyer
    (uniform), goods drawn with probability proportional to 1/rank,
    u ~ LogNormal(0, 1), w ~ U(0.5, 1.5)."""
    return zipf_market(n, m, seed, 1.5, 3, 70, np.float32, name=f"jd-shaped-{n}x{m}-s{seed}",
                       workers=workers, uniform_degrees=True)


# Named workloads.  "small" is the case the oracle finishes in seconds; the
# "1e8" market is the headline throughput workload.
def fisher_small(seed: int = 0) -> Market:
    """n=1000 buyers, m=500 goods, 10% Bernoulli density (~5e4 edges),
    u ~ U(0.01, 1) in float64, equal budgets w_i = 1."""
    return bernoulli_market(1000, 500, 0.10, seed, 0.01, 1.0, "ones",
                            np.float64, name=f"fisher-1000x500-q0.1-s{seed}")


def fisher_1e8(seed: int = 1, n: int = 1_000_000, m: int = 10_000, d: int = 100) -> Market:
    """n=1e6 buyers, m=1e4 goods, exactly 100 goods per buyer (1e8 edges),
    u ~ LogNormal(0, 1), w ~ U(0.5, 1.5), float32."""
    return fixed_degree_market(n, m, d, seed, "lognormal", 0.5, 1.5, np.float32,
                               name=f"fisher-{n}x{m}-d{d}-s{seed}")


def arrow_debreu_market(n: int, m: int, deg_u: int, deg_e: int, seed: int,
                        dtype=np.float32, name: str = "") -> Market:
    """Exchange market (Sec. 4): every agent values ``deg_u`` distinct
    uniform goods with u ~ LogNormal(0, 1) and owns ``deg_e`` distinct
    uniform goods with weights ~ U(0, 1); a good nobody owns gets one random
    owner; then every column of E is normalised to sum one (Sec. 4).
    Initial budgets w^0 = 1."""
    rng = np.random.default_rng(seed)
    Cu = _distinct_sorted_rows(rng, n, deg_u, m)
    col = Cu.reshape(-1)
    if (np.bincount(col, minlength=m) == 0).any():
        raise RuntimeError("a good received no buyer; raise n*deg_u relative to m")
    row_ptr = (np.arange(n + 1, dtype=np.int64) * deg_u).astype(np.int32)
    u = np.exp(rng.standard_normal(col.size)).astype(dtype)
    Ce = _distinct_sorted_rows(rng, n, deg_e, m)
    ev = rng.uniform(0.0, 1.0, Ce.shape)
    rows_e = np.repeat(np.arange(n), deg_e)
    cols_e = Ce.reshape(-1)
    vals_e = ev.reshape(-1)
    owned = np.bincount(cols_e, minlength=m) > 0
    orphans = np.nonzero(~owned)[0]
    if orphans.size:
        rows_e = np.concatenate([rows_e, rng.integers(0, n, orphans.size)])
        cols_e = np.concatenate([cols_e, orphans])
        vals_e = np.concatenate([vals_e, rng.uniform(0.0, 1.0, orphans.size)])
    order = np.lexsort((cols_e, rows_e))
    rows_e, cols_e, vals_e = rows_e[order], cols_e[order], vals_e[order]
    colsum = np.bincount(cols_e, weights=vals_e, minlength=m)
    vals_e = vals_e / colsum[cols_e]
    e_row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows_e, minlength=n), out=e_row_ptr[1:])
    mk = Market(n, m, row_ptr, col, u, np.ones(n, dtype=dtype),
                name or f"ad-{n}x{m}-du{deg_u}-de{deg_e}-s{seed}",
                e_row_ptr.astype(np.int32), cols_e.astype(np.int32), vals_e.astype(dtype))
    return mk


def arrow_debreu_1e5(seed: int = 4) -> Market:
    """The exchange workload: n = m = 1e5 agents and goods, 50 utility
    edges per agent (5e6), 5 endowed goods per agent, columns of E
    normalised to one (Sec. 4)."""
    return arrow_debreu_market(100_000, 100_000, 50, 5, seed)


@dataclass
class MarketBatch:
    """Independent Fisher markets concatenated: market b owns rows
    row_off[b]..row_off[b+1] (local row pointers concatenated in row_ptr,
    each starting at 0), edges edge_off[b]..edge_off[b+1] (local good ids in
    col) and goods good_off[b]..good_off[b+1]."""

    count: int
    n: np.ndarray  # int32 [count]
    m: np.ndarray  # int32 [count]
    row_ptr: np.ndarray  # int32 [sum(n) + count] local row pointers
    col: np.ndarray  # int32 [sum nnz] local good ids
    u: np.ndarray  # float32 [sum nnz]
    w: np.ndarray  # float32 [sum n]
    name: str = ""

    @property
    def nnz(self) -> np.ndarray:
        return np.array([self.market(b).nnz for b in range(self.count)])

    def offsets(self):
        n, m = self.n.astype(np.int64), self.m.astype(np.int64)
        rp_off = np.concatenate([[0], np.cumsum(n + 1)])
        row_off = np.concatenate([[0], np.cumsum(n)])
        good_off = np.concatenate([[0], np.cumsum(m)])
        nnz = self.row_ptr[rp_off[1:] - 1].astype(np.int64)
        edge_off = np.concatenate([[0], np.cumsum(nnz)])
        return rp_off, row_off, good_off, edge_off

    def market(self, b: int) -> Market:
        rp_off, row_off, good_off, edge_off = self.offsets()
        rp = self.row_ptr[rp_off[b]:rp_off[b + 1]]
        e0, e1 = edge_off[b], edge_off[b + 1]
        return Market(int(self.n[b]), int(self.m[b]), rp, self.col[e0:e1], self.u[e0:e1],
                      self.w[row_off[b]:row_off[b + 1]], f"{self.name}[{b}]")


def _sample_market(rng, n: int, m: int, q: float):
    """A random pattern with round(n m q) edges placed uniformly (at least
    one per buyer and per good), u ~ U(0.01, 1), w ~ U(0.5, 1.5)."""
    k = max(1, int(round(n * m * q)))
    pos = np.sort(rng.choice(n * m, size=k, replace=False))
    rows, cols = pos // m, pos % m
    have_r = np.bincount(rows, minlength=n) > 0
    have_c = np.bincount(cols, minlength=m) > 0
    extra_r = np.nonzero(~have_r)[0]
    extra_c = np.nonzero(~have_c)[0]
    add = [(r, int(rng.integers(0, m))) for r in extra_r] + \
          [(int(rng.integers(0, n)), c) for c in extra_c]
    if add:
        pos = np.unique(np.concatenate([pos, np.array([r * m + c for r, c in add], np.int64)]))
        rows, cols = pos // m, pos % m
    row_ptr = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    u = rng.uniform(0.01, 1.0, pos.size).astype(np.float32)
    w = rng.uniform(0.5, 1.5, n).astype(np.float32)
    return row_ptr.astype(np.int32), cols.astype(np.int32), u, w


def batch_markets(count: int, seed: int, n_range=(64, 8192), m_range=(16, 2048),
                  q_range=(0.05, 0.30)) -> MarketBatch:
    """``count`` independent markets: n, m log-uniform over the ranges,
    density q ~ U(q_range), u ~ U(0.01, 1), w ~ U(0.5, 1.5), float32.
    Market b uses its own generator seeded with (seed, b)."""
    ns, ms, rps, cols, us, ws = [], [], [], [], [], []
    for b in range(count):
        rng = np.random.default_rng([seed, b])
        n = int(round(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1])))))
        m = int(round(np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1])))))
        q = float(rng.uniform(*q_range))
        rp, c, u, w = _sample_market(rng, n, m, q)
        ns.append(n); ms.append(m); rps.append(rp); cols.append(c); us.append(u); ws.append(w)
    return MarketBatch(count, np.array(ns, np.int32), np.array(ms, np.int32),
                       np.concatenate(rps), np.concatenate(cols), np.concatenate(us),
                       np.concatenate(ws), f"batch-{count}-s{seed}")


def batch_from_markets(markets, name: str = "") -> MarketBatch:
    """Concatenate independent markets into a MarketBatch."""
    return MarketBatch(len(markets), np.array([mk.n for mk in markets], np.int32),
                       np.array([mk.m for mk in markets], np.int32),
                       np.concatenate([np.asarray(mk.row_ptr, np.int32) for mk in markets]),
                       np.concatenate([np.asarray(mk.col, np.int32) for mk in markets]),
                       np.concatenate([np.asarray(mk.u, np.float32) for mk in markets]),
                       np.concatenate([np.asarray(mk.w, np.float32) for mk in markets]),
                       name or f"batch-of-{len(markets)}")
