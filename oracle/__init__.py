"""FP64 CPU oracle for restarted PDHCG (Alg. 2) and restarted PDHG (Alg. 1)
on linear Fisher markets.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  The GPU solver
(``paper_2506_06258_amd``) never imports it and it never imports the GPU
solver; the two share no code.  The arithmetic lives in ``pdhcg_oracle.c``
(plain C, double precision); this module only marshals numpy arrays.

Parity unpinned: nothing in this package (every function has a pin in
``tests/test_oracle_*.py``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdhcg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, MAX_ITER, ERR_ARG, ERR_ASSUMPTION, ERR_NUMERIC, ERR_OOM = 0, 1, -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (portable -O2, OpenMP, IEEE math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class OraParams(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_iter", C.c_int64), ("eval_every", C.c_int32),
        ("restart", C.c_int32), ("beta_sufficient", C.c_double),
        ("beta_necessary", C.c_double), ("beta_artificial", C.c_double),
        ("theta", C.c_double), ("omega_check_every", C.c_int32),
        ("omega_bound", C.c_double), ("eta0", C.c_double), ("omega0", C.c_double),
        ("output", C.c_int32), ("prox", C.c_int32), ("sections", C.c_int32),
        ("prox_eps", C.c_double), ("normalize_rows", C.c_int32), ("verbose", C.c_int32),
        ("step_mode", C.c_int32),
    ]


class OraInfo(C.Structure):
    _fields_ = [
        ("rel_kkt", C.c_double), ("rel_primal", C.c_double), ("rel_dual", C.c_double),
        ("rel_gap", C.c_double), ("eta", C.c_double), ("omega", C.c_double),
        ("iters", C.c_int64), ("restarts", C.c_int32), ("status", C.c_int32),
        ("accepted", C.c_int64), ("emax_last", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        dp, ip64, ip32 = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int32)
        L.ora_default_params.argtypes = [C.POINTER(OraParams)]
        L.ora_num_threads.restype = C.c_int
        L.ora_validate.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp]
        L.ora_validate.restype = C.c_int
        L.ora_kkt.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, dp, dp, dp]
        L.ora_kkt.restype = C.c_double
        L.ora_row_root_exact.argtypes = [C.c_int, dp, dp, dp, C.c_void_p]
        L.ora_row_root_exact.restype = C.c_double
        L.ora_row_prox_exact.argtypes = [C.c_int, dp, dp, dp, C.c_double, C.c_double, dp,
                                         C.c_void_p, dp]
        L.ora_row_prox_exact.restype = C.c_double
        L.ora_row_prox_bisect.argtypes = [C.c_int, dp, dp, dp, C.c_double, C.c_double,
                                          C.c_double, C.c_int, dp, dp, C.POINTER(C.c_int)]
        L.ora_row_prox_bisect.restype = C.c_double
        L.ora_row_prox_ksection.argtypes = [C.c_int, dp, dp, dp, C.c_double, C.c_double,
                                            C.c_int, C.c_double, C.c_int, dp, dp,
                                            C.POINTER(C.c_int), dp, dp]
        L.ora_row_prox_ksection.restype = C.c_double
        L.ora_solve.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, C.POINTER(OraParams),
                                C.c_int, dp, dp, dp, C.POINTER(OraInfo)]
        L.ora_solve.restype = C.c_int
        L.ora_arrow_debreu.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, ip64, ip32, dp,
                                       C.POINTER(OraParams), C.c_double, C.c_int, dp, dp, dp,
                                       C.POINTER(C.c_int), C.POINTER(C.c_int64),
                                       C.POINTER(C.c_double)]
        L.ora_arrow_debreu.restype = C.c_int
        L.ora_implicit_grad.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, dp, dp, dp,
                                        C.c_double, dp, dp, C.POINTER(C.c_int)]
        L.ora_implicit_grad.restype = C.c_int
        L.ora_unrolled_grad.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, dp, dp, C.c_double,
                                        C.c_double, C.c_int, dp, dp, dp, dp]
        L.ora_unrolled_grad.restype = C.c_int
        L.ora_kkt_ty.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, dp, dp, dp, dp, dp]
        L.ora_kkt_ty.restype = C.c_double
        L.ora_pdhg_step.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, dp, dp, dp, dp, dp, dp,
                                    C.c_double, C.c_double, dp, dp, dp, dp]
        L.ora_pdhg_step.restype = None
        L.ora_pdhg_solve.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, C.POINTER(OraParams),
                                     dp, dp, dp, dp, C.POINTER(OraInfo)]
        L.ora_pdhg_solve.restype = C.c_int
        L.ora_fixed_restart.argtypes = [C.c_int, C.c_int, ip64, ip32, dp, dp, C.c_int, C.c_int,
                                        C.c_double, dp, dp, dp, dp, dp]
        L.ora_fixed_restart.restype = C.c_int
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def num_threads() -> int:
    return int(lib().ora_num_threads())


def default_params(**kw) -> OraParams:
    prm = OraParams()
    lib().ora_default_params(C.byref(prm))
    for k, v in kw.items():
        if not hasattr(prm, k):
            raise KeyError(k)
        setattr(prm, k, v)
    return prm


def _csr(row_ptr, col):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col, dtype=np.int32))


def validate(n, m, row_ptr, col, u, w) -> int:
    rp, cl = _csr(row_ptr, col)
    u, w = _d(u), _d(w)
    return int(lib().ora_validate(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                  _ptr(u, C.c_double), _ptr(w, C.c_double)))


def kkt(n, m, row_ptr, col, u, w, x, p):
    """Relative KKT error (r_primal, r_dual, r_gap) of (x, p) on utilities u."""
    rp, cl = _csr(row_ptr, col)
    u, w, x, p = _d(u), _d(w), _d(x), _d(p)
    out = np.zeros(3)
    r = lib().ora_kkt(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(u, C.c_double),
                      _ptr(w, C.c_double), _ptr(x, C.c_double), _ptr(p, C.c_double),
                      _ptr(out, C.c_double))
    return float(r), out


def kkt_ty(n, m, row_ptr, col, u, w, x, t, p, y):
    """Relative KKT error (r_primal, r_dual, r_gap) of a point (x, t, p, y) of
    the reformulated program (Sec. 2.1), on utilities u."""
    rp, cl = _csr(row_ptr, col)
    u, w, x, t, p, y = _d(u), _d(w), _d(x), _d(t), _d(p), _d(y)
    out = np.zeros(3)
    r = lib().ora_kkt_ty(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(u, C.c_double),
                         _ptr(w, C.c_double), _ptr(x, C.c_double), _ptr(t, C.c_double),
                         _ptr(p, C.c_double), _ptr(y, C.c_double), _ptr(out, C.c_double))
    return float(r), out


def pdhg_step(n, m, row_ptr, col, u, w, x, t, p, y, c_prev, g_prev, tau, sigma):
    """One PDHG iteration of Alg. 1 (eqs. update:py, update:t, update:x) on
    utilities u from (x, t, p, y) with the previous column sums c_prev and
    utility residuals g_prev = t - Ux; returns (x', t', p', y')."""
    rp, cl = _csr(row_ptr, col)
    u, w, x, t, p, y = _d(u), _d(w), _d(x), _d(t), _d(p), _d(y)
    c_prev, g_prev = _d(c_prev), _d(g_prev)
    x2, t2, p2, y2 = np.zeros_like(x), np.zeros(n), np.zeros(m), np.zeros(n)
    lib().ora_pdhg_step(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(u, C.c_double),
                        _ptr(w, C.c_double), _ptr(x, C.c_double), _ptr(t, C.c_double),
                        _ptr(p, C.c_double), _ptr(y, C.c_double), _ptr(c_prev, C.c_double),
                        _ptr(g_prev, C.c_double), float(tau), float(sigma),
                        _ptr(x2, C.c_double), _ptr(t2, C.c_double), _ptr(p2, C.c_double),
                        _ptr(y2, C.c_double))
    return x2, t2, p2, y2


@dataclass
class PdhgSolution:
    p: np.ndarray
    x: np.ndarray
    t: np.ndarray  # normalised units (u_i / max_j u_ij)
    y: np.ndarray  # normalised units
    status: int
    rel_kkt: float
    rel_primal: float
    rel_dual: float
    rel_gap: float
    iters: int
    restarts: int
    eta: float
    omega: float
    accepted: int
    emax_last: float


def pdhg_solve(n, m, row_ptr, col, u, w, params: OraParams | None = None,
               **kw) -> PdhgSolution:
    """Restarted PDHG in FP64 (Alg. 1 with the Sec. 5 enhancements)."""
    rp, cl = _csr(row_ptr, col)
    u, w = _d(u), _d(w)
    prm = params if params is not None else default_params(**kw)
    if params is not None:
        for k, v in kw.items():
            setattr(prm, k, v)
    p, x, t, y = np.zeros(m), np.zeros(int(rp[-1])), np.zeros(n), np.zeros(n)
    info = OraInfo()
    st = lib().ora_pdhg_solve(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(u, C.c_double),
                              _ptr(w, C.c_double), C.byref(prm), _ptr(p, C.c_double),
                              _ptr(x, C.c_double), _ptr(t, C.c_double), _ptr(y, C.c_double),
                              C.byref(info))
    return PdhgSolution(p, x, t, y, int(st), info.rel_kkt, info.rel_primal, info.rel_dual,
                        info.rel_gap, int(info.iters), int(info.restarts), info.eta, info.omega,
                        int(info.accepted), info.emax_last)


def fixed_restart(n, m, row_ptr, col, u, w, K, R, eta=0.0, p_ref=None):
    """Alg. 2 with fixed sigma = tau = eta (<= 0: 1/(2||K||)) and restart
    length K, R restarts to the average (the setting of Sec. 3).  Returns
    (status, p, x, dist[R+1], kkt[R+1]) with dist[n] = |p^{n,0} - p_ref|_2
    (zeros without p_ref) and kkt[n] the relative KKT error of the n-th
    restart point."""
    rp, cl = _csr(row_ptr, col)
    u, w = _d(u), _d(w)
    p, x = np.zeros(m), np.zeros(int(rp[-1]))
    dist, kk = np.zeros(R + 1), np.zeros(R + 1)
    pr = _d(p_ref) if p_ref is not None else None
    st = lib().ora_fixed_restart(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                 _ptr(u, C.c_double), _ptr(w, C.c_double), int(K), int(R),
                                 float(eta), _ptr(pr, C.c_double) if pr is not None else None,
                                 _ptr(dist, C.c_double) if pr is not None else None,
                                 _ptr(kk, C.c_double), _ptr(p, C.c_double), _ptr(x, C.c_double))
    return int(st), p, x, dist, kk


def normalize_rows(row_ptr, u):
    """u_hat = u / max_j u_ij per row (the preprocessing of Sec. 5)."""
    u = _d(u)
    rp = np.asarray(row_ptr, dtype=np.int64)
    lens = np.diff(rp)
    mx = np.zeros(len(rp) - 1)
    nz = lens > 0
    mx[nz] = np.maximum.reduceat(u, rp[:-1][nz])
    return u / np.repeat(mx, lens), mx


def row_prox_exact(u, xk, pg, w, tau):
    """Exact solution of one row subproblem; returns (x, s*)."""
    u, xk, pg = _d(u), _d(xk), _d(pg)
    d = u.size
    x = np.zeros(d)
    ab = np.zeros(2 * max(d, 1))
    work = (C.c_double * (3 * max(d, 1)))()
    s = lib().ora_row_prox_exact(d, _ptr(u, C.c_double), _ptr(xk, C.c_double),
                                 _ptr(pg, C.c_double), float(w), float(tau),
                                 _ptr(x, C.c_double), C.cast(work, C.c_void_p),
                                 _ptr(ab, C.c_double))
    return x, float(s)


def row_prox_bisect(u, xk, pg, w, tau, eps=1e-13, max_rounds=200):
    u, xk, pg = _d(u), _d(xk), _d(pg)
    d = u.size
    x = np.zeros(d)
    ab = np.zeros(2 * max(d, 1))
    rounds = C.c_int(0)
    s = lib().ora_row_prox_bisect(d, _ptr(u, C.c_double), _ptr(xk, C.c_double),
                                  _ptr(pg, C.c_double), float(w), float(tau), eps,
                                  max_rounds, _ptr(x, C.c_double), _ptr(ab, C.c_double),
                                  C.byref(rounds))
    return x, float(s), rounds.value


def row_prox_ksection(u, xk, pg, w, tau, K=32, eps=1e-13, max_rounds=200):
    """k-section search; returns (x, s, rounds, L, U) with the final bracket."""
    u, xk, pg = _d(u), _d(xk), _d(pg)
    d = u.size
    x = np.zeros(d)
    ab = np.zeros(2 * max(d, 1))
    rounds = C.c_int(0)
    Lo, Hi = C.c_double(0), C.c_double(0)
    s = lib().ora_row_prox_ksection(d, _ptr(u, C.c_double), _ptr(xk, C.c_double),
                                    _ptr(pg, C.c_double), float(w), float(tau), int(K), eps,
                                    max_rounds, _ptr(x, C.c_double), _ptr(ab, C.c_double),
                                    C.byref(rounds), C.byref(Lo), C.byref(Hi))
    return x, float(s), rounds.value, Lo.value, Hi.value


def row_prox_all(row_ptr, col, uh, w, x_in, p, tau):
    """Exact prox of every row (u already normalised); returns (x, s[n])."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col)
    uh, w, x_in, p = _d(uh), _d(w), _d(x_in), _d(p)
    n = rp.size - 1
    x = np.zeros_like(x_in)
    s = np.zeros(n)
    for i in range(n):
        a, b = rp[i], rp[i + 1]
        x[a:b], s[i] = row_prox_exact(uh[a:b], x_in[a:b], p[col[a:b]], w[i], tau)
    return x, s


@dataclass
class Solution:
    p: np.ndarray
    x: np.ndarray
    t: np.ndarray
    status: int
    rel_kkt: float
    rel_primal: float
    rel_dual: float
    rel_gap: float
    iters: int
    restarts: int
    eta: float
    omega: float
    accepted: int = 0
    emax_last: float = float("nan")


def solve(n, m, row_ptr, col, u, w, params: OraParams | None = None, p0=None, x0=None,
          **kw) -> Solution:
    """Restarted PDHCG in FP64 (Alg. 2 with the Sec. 5 enhancements)."""
    rp, cl = _csr(row_ptr, col)
    u, w = _d(u), _d(w)
    prm = params if params is not None else default_params(**kw)
    if params is not None:
        for k, v in kw.items():
            setattr(prm, k, v)
    warm = p0 is not None and x0 is not None
    p = _d(p0).copy() if warm else np.zeros(m)
    x = _d(x0).copy() if warm else np.zeros(int(rp[-1]))
    t = np.zeros(n)
    info = OraInfo()
    st = lib().ora_solve(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32), _ptr(u, C.c_double),
                         _ptr(w, C.c_double), C.byref(prm), int(warm), _ptr(p, C.c_double),
                         _ptr(x, C.c_double), _ptr(t, C.c_double), C.byref(info))
    return Solution(p, x, t, int(st), info.rel_kkt, info.rel_primal, info.rel_dual,
                    info.rel_gap, int(info.iters), int(info.restarts), info.eta, info.omega,
                    int(info.accepted), info.emax_last)


def solve_market(mk, **kw) -> Solution:
    return solve(mk.n, mk.m, mk.row_ptr, mk.col, mk.u, mk.w, **kw)


def arrow_debreu(n, m, row_ptr, col, u, e_row_ptr, e_col, e_val, w0, inner: OraParams,
                 outer_tol=1e-6, outer_max=100):
    """Alg. 4 fixed point; returns dict(p, w, x, status, outer, inner, change)."""
    rp, cl = _csr(row_ptr, col)
    erp, ecl = _csr(e_row_ptr, e_col)
    u, ev = _d(u), _d(e_val)
    w = _d(w0).copy()
    p = np.zeros(m)
    x = np.zeros(int(rp[-1]))
    oi, ii, ch = C.c_int(0), C.c_int64(0), C.c_double(0)
    st = lib().ora_arrow_debreu(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                _ptr(u, C.c_double), _ptr(erp, C.c_int64), _ptr(ecl, C.c_int32),
                                _ptr(ev, C.c_double), C.byref(inner), float(outer_tol),
                                int(outer_max), _ptr(w, C.c_double), _ptr(p, C.c_double),
                                _ptr(x, C.c_double), C.byref(oi), C.byref(ii), C.byref(ch))
    return dict(p=p, w=w, x=x, status=int(st), outer=oi.value, inner=ii.value,
                change=ch.value)


def implicit_grad(n, m, row_ptr, col, u, w, x, p, dL_dp, act_tol=1e-9):
    """dL/du (on the stored pattern) and dL/dw of a loss L(p) at the
    equilibrium (x, p), by the implicit function theorem on the equilibrium
    conditions over the active support.  Returns (status, dL_du, dL_dw, dim)."""
    rp, cl = _csr(row_ptr, col)
    u, w, x, p, g = _d(u), _d(w), _d(x), _d(p), _d(dL_dp)
    du = np.zeros(int(rp[-1]))
    dw = np.zeros(n)
    dim = C.c_int(0)
    st = lib().ora_implicit_grad(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                 _ptr(u, C.c_double), _ptr(w, C.c_double), _ptr(x, C.c_double),
                                 _ptr(p, C.c_double), _ptr(g, C.c_double), float(act_tol),
                                 _ptr(du, C.c_double), _ptr(dw, C.c_double), C.byref(dim))
    return int(st), du, dw, dim.value


def unrolled_grad(n, m, row_ptr, col, u, w, x0, p0, tau, sigma, K, dL_dp):
    """Reverse mode through K fixed-step PDHCG iterations from (x0, p0) for a
    loss of the final prices.  Returns (status, dL_du, dL_dw, p_K)."""
    rp, cl = _csr(row_ptr, col)
    u, w, x0, p0, g = _d(u), _d(w), _d(x0), _d(p0), _d(dL_dp)
    du = np.zeros(int(rp[-1]))
    dw = np.zeros(n)
    pK = np.zeros(m)
    st = lib().ora_unrolled_grad(n, m, _ptr(rp, C.c_int64), _ptr(cl, C.c_int32),
                                 _ptr(u, C.c_double), _ptr(w, C.c_double), _ptr(x0, C.c_double),
                                 _ptr(p0, C.c_double), float(tau), float(sigma), int(K),
                                 _ptr(g, C.c_double), _ptr(du, C.c_double), _ptr(dw, C.c_double),
                                 _ptr(pK, C.c_double))
    return int(st), du, dw, pK
