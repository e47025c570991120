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
