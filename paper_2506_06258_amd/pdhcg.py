"""Thin ctypes binding of ``libpdhcg.so`` (the C ABI in ``include/pdhcg.h``).

The functions named ``pdhcg_*`` take the same arguments as their C
counterparts, with torch CUDA (HIP) tensors in place of device pointers; they
only check dtypes/devices and marshal pointers.  Every step of the solver
runs in the HIP library; there is no CPU fallback: if the library is missing
the import fails.

``Market`` is a small convenience wrapper around a market handle.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdhcg.so")

PDHCG_OK, PDHCG_MAX_ITER = 0, 1
PDHCG_ERR_ARG, PDHCG_ERR_ASSUMPTION, PDHCG_ERR_NUMERIC = -1, -2, -3
PDHCG_ERR_OOM, PDHCG_ERR_HIP, PDHCG_ERR_UNSUPPORTED = -4, -5, -6
PDHCG_SEARCH_ACTIVESET, PDHCG_SEARCH_KSECTION, PDHCG_SEARCH_KSECTION_WAVE = 0, 1, 2
PDHCG_STEP_FIXED, PDHCG_STEP_ADAPTIVE = 0, 1
PDHCG_RESTART_NONE, PDHCG_RESTART_ADAPTIVE = 0, 1
PDHCG_OUTPUT_CANDIDATE, PDHCG_OUTPUT_CURRENT, PDHCG_OUTPUT_AVERAGE = 0, 1, 2

# Every function the header declares (checked by the test-suite).
EXPORTS = (
    "pdhcg_abi_version", "pdhcg_status_string", "pdhcg_last_error",
    "pdhcg_default_params", "pdhcg_validate_host", "pdhcg_market_create",
    "pdhcg_set_budgets", "pdhcg_solve", "pdhcg_solve_fixed_restart", "pdhcg_pdhg_solve",
    "pdhcg_kkt", "pdhcg_row_prox",
    "pdhcg_arrow_debreu", "pdhcg_backward", "pdhcg_backward_noalloc", "pdhcg_market_bins",
    "pdhcg_market_lds_goods",
    "pdhcg_market_destroy",
    "pdhcg_batch_create", "pdhcg_batch_solve", "pdhcg_batch_autotune", "pdhcg_batch_backward",
    "pdhcg_batch_layout",
    "pdhcg_batch_destroy",
)


class pdhcg_params(C.Structure):
    _fields_ = [
        ("tol", C.c_double), ("max_iter", C.c_int64), ("eval_every", C.c_int32),
        ("search", C.c_int32), ("sections", C.c_int32), ("max_search_rounds", C.c_int32),
        ("search_rtol", C.c_double), ("step_mode", C.c_int32), ("restart", C.c_int32),
        ("beta_sufficient", C.c_double), ("beta_necessary", C.c_double),
        ("beta_artificial", C.c_double), ("theta", C.c_double),
        ("omega_check_every", C.c_int32), ("output", C.c_int32),
        ("omega_bound", C.c_double), ("eta0", C.c_double), ("omega0", C.c_double),
        ("normalize_rows", C.c_int32), ("verbose", C.c_int32), ("timing", C.c_int32),
    ]


class pdhcg_info(C.Structure):
    _fields_ = [
        ("rel_kkt", C.c_double), ("rel_primal", C.c_double), ("rel_dual", C.c_double),
        ("rel_gap", C.c_double), ("eta", C.c_double), ("omega", C.c_double),
        ("seconds", C.c_double), ("iters", C.c_int64), ("accepted", C.c_int64),
        ("restarts", C.c_int32), ("status", C.c_int32), ("evals", C.c_int32),
        ("search_rounds_max", C.c_int32), ("search_rounds_mean", C.c_double),
        ("row_pass_seconds", C.c_double), ("row_pass_launches", C.c_int64),
    ]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class pdhcg_batch_schedule(C.Structure):
    _fields_ = [("wg_per_cu", C.c_int32), ("shape_policy", C.c_int32), ("trials", C.c_int32),
                ("best_trial_seconds", C.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib() -> C.CDLL:
    """Load libpdhcg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2506_06258_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    sig = {
        "pdhcg_abi_version": (i32, []),
        "pdhcg_status_string": (C.c_char_p, [i32]),
        "pdhcg_last_error": (C.c_char_p, []),
        "pdhcg_default_params": (None, [C.POINTER(pdhcg_params)]),
        "pdhcg_validate_host": (i32, [i32, i32, i64, vp, vp, vp, vp]),
        "pdhcg_market_create": (i32, [i32, i32, i64, vp, vp, vp, vp, vp, C.POINTER(vp)]),
        "pdhcg_set_budgets": (i32, [vp, vp]),
        "pdhcg_solve": (i32, [vp, C.POINTER(pdhcg_params), i32, vp, vp, vp,
                              C.POINTER(pdhcg_info)]),
        "pdhcg_pdhg_solve": (i32, [vp, C.POINTER(pdhcg_params), i32, vp, vp, vp, vp,
                                   C.POINTER(pdhcg_info)]),
        "pdhcg_solve_fixed_restart": (i32, [vp, i32, i32, dbl, vp, C.POINTER(dbl),
                                            C.POINTER(dbl), vp, vp, C.POINTER(pdhcg_info)]),
        "pdhcg_kkt": (i32, [vp, vp, vp, C.POINTER(pdhcg_info)]),
        "pdhcg_row_prox": (i32, [vp, vp, vp, dbl, C.POINTER(pdhcg_params), vp, vp]),
        "pdhcg_arrow_debreu": (i32, [vp, vp, vp, vp, i64, C.POINTER(pdhcg_params), dbl, i32,
                                     vp, vp, vp, C.POINTER(i32), C.POINTER(i64),
                                     C.POINTER(pdhcg_info)]),
        "pdhcg_backward": (i32, [vp, vp, vp, dbl, i32, i32, vp, vp, vp]),
        "pdhcg_backward_noalloc": (i32, [vp, vp, vp, dbl, i32, i32, vp, vp, vp]),
        "pdhcg_market_bins": (i32, [vp, i32, vp, vp, vp]),
        "pdhcg_market_lds_goods": (i32, [vp]),
        "pdhcg_market_destroy": (None, [vp]),
        "pdhcg_batch_create": (i32, [i32, vp, vp, vp, vp, vp, vp, vp, C.POINTER(vp)]),
        "pdhcg_batch_solve": (i32, [vp, C.POINTER(pdhcg_params), vp, vp, vp]),
        "pdhcg_batch_autotune": (i32, [vp, C.POINTER(pdhcg_params), i32,
                                       C.POINTER(pdhcg_batch_schedule)]),
        "pdhcg_batch_backward": (i32, [vp, vp, vp, vp, i32, i32, vp, vp, vp]),
        "pdhcg_batch_layout": (i32, [vp, vp, vp]),
        "pdhcg_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class PDHCGError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.pdhcg_status_string(status).decode()
        detail = L.pdhcg_last_error().decode()
        super().__init__(f"{where}: {msg} ({status}){': ' + detail if detail else ''}")
        self.status = status


def _check(status: int, where: str, ok=(PDHCG_OK,)) -> int:
    if status not in ok:
        raise PDHCGError(status, where)
    return status


def _dev_ptr(t: Optional[torch.Tensor], dtype, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return C.c_void_p(t.data_ptr())


def _host_ptr(a, name: str):
    import numpy as np
    if not isinstance(a, np.ndarray) or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"{name} must be a C-contiguous numpy array")
    return C.c_void_p(a.ctypes.data)


def pdhcg_default_params(**overrides) -> pdhcg_params:
    prm = pdhcg_params()
    lib().pdhcg_default_params(C.byref(prm))
    for k, v in overrides.items():
        if not hasattr(prm, k):
            raise KeyError(k)
        setattr(prm, k, v)
    return prm


def pdhcg_abi_version() -> int:
    return int(lib().pdhcg_abi_version())


def pdhcg_status_string(status: int) -> str:
    return lib().pdhcg_status_string(status).decode()


def pdhcg_last_error() -> str:
    return lib().pdhcg_last_error().decode()


def pdhcg_validate_host(n, m, nnz, row_ptr, col, u, w) -> int:
    """Host-memory validation (numpy int32/float32 arrays); returns a status."""
    import numpy as np
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    uu = np.ascontiguousarray(u, dtype=np.float32)
    ww = np.ascontiguousarray(w, dtype=np.float32)
    return int(lib().pdhcg_validate_host(int(n), int(m), int(nnz), _host_ptr(rp, "row_ptr"),
                                         _host_ptr(cl, "col"), _host_ptr(uu, "u"),
                                         _host_ptr(ww, "w")))


def _stream_handle(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def pdhcg_market_create(n, m, nnz, row_ptr, col, u, w, stream=None) -> C.c_void_p:
    h = C.c_void_p()
    st = lib().pdhcg_market_create(int(n), int(m), int(nnz),
                                   _dev_ptr(row_ptr, torch.int32, "row_ptr"),
                                   _dev_ptr(col, torch.int32, "col"),
                                   _dev_ptr(u, torch.float32, "u"),
                                   _dev_ptr(w, torch.float32, "w"),
                                   _stream_handle(stream), C.byref(h))
    _check(st, "pdhcg_market_create")
    return h


def pdhcg_market_destroy(h) -> None:
    if h:
        lib().pdhcg_market_destroy(h)


def pdhcg_set_budgets(h, w) -> None:
    _check(lib().pdhcg_set_budgets(h, _dev_ptr(w, torch.float32, "w")), "pdhcg_set_budgets")


def pdhcg_solve(h, params: pdhcg_params, warm: int, p, x, t=None) -> pdhcg_info:
    info = pdhcg_info()
    st = lib().pdhcg_solve(h, C.byref(params), int(warm), _dev_ptr(p, torch.float32, "p"),
                           _dev_ptr(x, torch.float32, "x"), _dev_ptr(t, torch.float32, "t"),
                           C.byref(info))
    _check(st, "pdhcg_solve", ok=(PDHCG_OK, PDHCG_MAX_ITER))
    return info


def pdhcg_pdhg_solve(h, params: pdhcg_params, warm: int, p, x, t=None, y=None) -> pdhcg_info:
    info = pdhcg_info()
    st = lib().pdhcg_pdhg_solve(h, C.byref(params), int(warm), _dev_ptr(p, torch.float32, "p"),
                                _dev_ptr(x, torch.float32, "x"), _dev_ptr(t, torch.float32, "t"),
                                _dev_ptr(y, torch.float32, "y"), C.byref(info))
    _check(st, "pdhcg_pdhg_solve", ok=(PDHCG_OK, PDHCG_MAX_ITER))
    return info


def pdhcg_solve_fixed_restart(h, K: int, restarts: int, eta: float, p_ref, p, x):
    """Returns (info, dist[restarts+1], kkt[restarts+1]) (numpy)."""
    info = pdhcg_info()
    dist = np.zeros(restarts + 1)
    kk = np.zeros(restarts + 1)
    _check(lib().pdhcg_solve_fixed_restart(
        h, int(K), int(restarts), float(eta), _dev_ptr(p_ref, torch.float32, "p_ref"),
        dist.ctypes.data_as(C.POINTER(C.c_double)), kk.ctypes.data_as(C.POINTER(C.c_double)),
        _dev_ptr(p, torch.float32, "p"), _dev_ptr(x, torch.float32, "x"), C.byref(info)),
        "pdhcg_solve_fixed_restart")
    return info, dist, kk


def pdhcg_kkt(h, p, x) -> pdhcg_info:
    info = pdhcg_info()
    _check(lib().pdhcg_kkt(h, _dev_ptr(p, torch.float32, "p"), _dev_ptr(x, torch.float32, "x"),
                           C.byref(info)), "pdhcg_kkt")
    return info


def pdhcg_row_prox(h, x_in, p, tau: float, params: Optional[pdhcg_params], x_out, s_out=None):
    prm = C.byref(params) if params is not None else None
    _check(lib().pdhcg_row_prox(h, _dev_ptr(x_in, torch.float32, "x_in"),
                                _dev_ptr(p, torch.float32, "p"), float(tau), prm,
                                _dev_ptr(x_out, torch.float32, "x_out"),
                                _dev_ptr(s_out, torch.float32, "s_out")), "pdhcg_row_prox")


def pdhcg_backward(h, x, p, omega: float, unroll: int, ckpt_every: int, dL_dp, dL_du, dL_dw):
    _check(lib().pdhcg_backward(h, _dev_ptr(x, torch.float32, "x"), _dev_ptr(p, torch.float32, "p"),
                                float(omega), int(unroll), int(ckpt_every),
                                _dev_ptr(dL_dp, torch.float32, "dL_dp"),
                                _dev_ptr(dL_du, torch.float32, "dL_du"),
                                _dev_ptr(dL_dw, torch.float32, "dL_dw")), "pdhcg_backward")


def pdhcg_backward_noalloc(h, x, p, omega: float, unroll: int, ckpt_every: int, dL_dp, dL_du,
                           dL_dw):
    _check(lib().pdhcg_backward_noalloc(h, _dev_ptr(x, torch.float32, "x"),
                                        _dev_ptr(p, torch.float32, "p"),
                                        float(omega), int(unroll), int(ckpt_every),
                                        _dev_ptr(dL_dp, torch.float32, "dL_dp"),
                                        _dev_ptr(dL_du, torch.float32, "dL_du"),
                                        _dev_ptr(dL_dw, torch.float32, "dL_dw")),
           "pdhcg_backward_noalloc")


def pdhcg_arrow_debreu(h, e_row_ptr, e_col, e_val, e_nnz, inner: pdhcg_params, outer_tol,
                       outer_max, w, p, x):
    oi, ii, info = C.c_int32(0), C.c_int64(0), pdhcg_info()
    st = lib().pdhcg_arrow_debreu(h, _dev_ptr(e_row_ptr, torch.int32, "e_row_ptr"),
                                  _dev_ptr(e_col, torch.int32, "e_col"),
                                  _dev_ptr(e_val, torch.float32, "e_val"), int(e_nnz),
                                  C.byref(inner), float(outer_tol), int(outer_max),
                                  _dev_ptr(w, torch.float32, "w"),
                                  _dev_ptr(p, torch.float32, "p"),
                                  _dev_ptr(x, torch.float32, "x"), C.byref(oi), C.byref(ii),
                                  C.byref(info))
    _check(st, "pdhcg_arrow_debreu", ok=(PDHCG_OK, PDHCG_MAX_ITER))
    return st, oi.value, ii.value, info


def pdhcg_market_bins(h, cap: int = 64):
    import numpy as np
    G = np.zeros(cap, np.int32)
    E = np.zeros(cap, np.int32)
    R = np.zeros(cap, np.int32)
    nb = lib().pdhcg_market_bins(h, cap, _host_ptr(G, "G"), _host_ptr(E, "E"), _host_ptr(R, "R"))
    if nb < 0:
        _check(nb, "pdhcg_market_bins")
    k = min(nb, cap)
    return list(zip(G[:k].tolist(), E[:k].tolist(), R[:k].tolist()))


def pdhcg_market_lds_goods(h) -> int:
    r = lib().pdhcg_market_lds_goods(h)
    if r < 0:
        _check(r, "pdhcg_market_lds_goods")
    return r


@dataclass
class Solution:
    p: torch.Tensor
    x: torch.Tensor
    t: torch.Tensor
    info: pdhcg_info


class Market:
    """A market handle over torch device tensors (CSR int32, float32 values)."""

    def __init__(self, row_ptr, col, u, w, m: Optional[int] = None, device="cuda", stream=None):
        dev = torch.device(device)
        self.row_ptr = torch.as_tensor(row_ptr, dtype=torch.int32).to(dev).contiguous()
        self.col = torch.as_tensor(col, dtype=torch.int32).to(dev).contiguous()
        u_t = torch.as_tensor(u).to(dev, torch.float32).contiguous()
        w_t = torch.as_tensor(w).to(dev, torch.float32).contiguous()
        self.n = int(self.row_ptr.numel() - 1)
        self.nnz = int(self.col.numel())
        self.m = int(m) if m is not None else int(self.col.max().item()) + 1
        self.device = dev
        self.stream = stream
        self._h = pdhcg_market_create(self.n, self.m, self.nnz, self.row_ptr, self.col, u_t, w_t,
                                      stream)

    @classmethod
    def from_synth(cls, mk, device="cuda", stream=None) -> "Market":
        return cls(mk.row_ptr, mk.col, mk.u, mk.w, m=mk.m, device=device, stream=stream)

    def close(self):
        if getattr(self, "_h", None):
            pdhcg_market_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self, **kw) -> pdhcg_params:
        return pdhcg_default_params(**kw)

    def solve(self, params: Optional[pdhcg_params] = None, p0=None, x0=None, **kw) -> Solution:
        prm = params if params is not None else pdhcg_default_params(**kw)
        p = torch.empty(self.m, dtype=torch.float32, device=self.device)
        x = torch.empty(self.nnz, dtype=torch.float32, device=self.device)
        t = torch.empty(self.n, dtype=torch.float32, device=self.device)
        warm = p0 is not None and x0 is not None
        if warm:
            p.copy_(torch.as_tensor(p0, dtype=torch.float32))
            x.copy_(torch.as_tensor(x0, dtype=torch.float32))
        info = pdhcg_solve(self._h, prm, int(warm), p, x, t)
        return Solution(p, x, t, info)

    def pdhg_solve(self, params: Optional[pdhcg_params] = None, **kw):
        """Restarted PDHG (pdhcg_pdhg_solve): (Solution, y) with t and y in
        the caller's units."""
        prm = params if params is not None else pdhcg_default_params(**kw)
        p = torch.empty(self.m, dtype=torch.float32, device=self.device)
        x = torch.empty(self.nnz, dtype=torch.float32, device=self.device)
        t = torch.empty(self.n, dtype=torch.float32, device=self.device)
        y = torch.empty(self.n, dtype=torch.float32, device=self.device)
        info = pdhcg_pdhg_solve(self._h, prm, 0, p, x, t, y)
        return Solution(p, x, t, info), y

    def solve_fixed_restart(self, K: int, restarts: int, eta: float = 0.0, p_ref=None):
        """Alg. 2 with fixed steps and restart length (pdhcg_solve_fixed_restart):
        (Solution without t, dist, kkt)."""
        p = torch.empty(self.m, dtype=torch.float32, device=self.device)
        x = torch.empty(self.nnz, dtype=torch.float32, device=self.device)
        pr = None
        if p_ref is not None:
            pr = torch.as_tensor(p_ref).to(self.device, torch.float32).contiguous()
        info, dist, kk = pdhcg_solve_fixed_restart(self._h, K, restarts, eta, pr, p, x)
        return Solution(p, x, None, info), dist, kk

    def set_budgets(self, w) -> None:
        w_t = torch.as_tensor(w).to(self.device, torch.float32).contiguous()
        pdhcg_set_budgets(self._h, w_t)

    def kkt(self, p, x) -> pdhcg_info:
        return pdhcg_kkt(self._h, p.contiguous(), x.contiguous())

    def row_prox(self, x_in, p, tau: float, params: Optional[pdhcg_params] = None):
        x_out = torch.empty_like(x_in)
        s_out = torch.empty(self.n, dtype=torch.float32, device=self.device)
        pdhcg_row_prox(self._h, x_in.contiguous(), p.contiguous(), tau, params, x_out, s_out)
        return x_out, s_out

    def bins(self):
        return pdhcg_market_bins(self._h)

    def lds_goods(self) -> int:
        """Goods whose column data the row kernels keep in LDS (m: all)."""
        return pdhcg_market_lds_goods(self._h)

    def backward(self, x, p, omega: float, dL_dp, unroll: int = 1024, ckpt_every: int = 32,
                 out=None, noalloc: bool = False):
        """(dL/du, dL/dw) by reverse mode through `unroll` fixed-step
        iterations from (x, p); see pdhcg_backward.  noalloc: call
        pdhcg_backward_noalloc (the library's fixed workspace); out: optional
        (du, dw) tensors to write into."""
        if out is None:
            du = torch.empty(self.nnz, dtype=torch.float32, device=self.device)
            dw = torch.empty(self.n, dtype=torch.float32, device=self.device)
        else:
            du, dw = out
        g = torch.as_tensor(dL_dp).to(self.device, torch.float32).contiguous()
        fn = pdhcg_backward_noalloc if noalloc else pdhcg_backward
        fn(self._h, x.contiguous(), p.contiguous(), omega, unroll, ckpt_every, g, du, dw)
        return du, dw

    def arrow_debreu(self, e_row_ptr, e_col, e_val, w0, inner: Optional[pdhcg_params] = None,
                     outer_tol: float = 1e-6, outer_max: int = 100):
        inner = inner if inner is not None else pdhcg_default_params()
        erp = torch.as_tensor(e_row_ptr, dtype=torch.int32).to(self.device).contiguous()
        ecl = torch.as_tensor(e_col, dtype=torch.int32).to(self.device).contiguous()
        ev = torch.as_tensor(e_val).to(self.device, torch.float32).contiguous()
        w = torch.as_tensor(w0).to(self.device, torch.float32).contiguous().clone()
        p = torch.empty(self.m, dtype=torch.float32, device=self.device)
        x = torch.empty(self.nnz, dtype=torch.float32, device=self.device)
        st, outer, inner_it, info = pdhcg_arrow_debreu(self._h, erp, ecl, ev, ecl.numel(), inner,
                                                       outer_tol, outer_max, w, p, x)
        return dict(status=st, p=p, w=w, x=x, outer=outer, inner=inner_it, info=info)


def pdhcg_batch_create(count, n, m, row_ptr_cat, col_cat, u_cat, w_cat, stream=None):
    """n, m: host int32 arrays; the CSR arrays are device tensors."""
    import numpy as np
    nn = np.ascontiguousarray(n, dtype=np.int32)
    mm = np.ascontiguousarray(m, dtype=np.int32)
    h = C.c_void_p()
    st = lib().pdhcg_batch_create(int(count), _host_ptr(nn, "n"), _host_ptr(mm, "m"),
                                  _dev_ptr(row_ptr_cat, torch.int32, "row_ptr_cat"),
                                  _dev_ptr(col_cat, torch.int32, "col_cat"),
                                  _dev_ptr(u_cat, torch.float32, "u_cat"),
                                  _dev_ptr(w_cat, torch.float32, "w_cat"),
                                  _stream_handle(stream), C.byref(h))
    _check(st, "pdhcg_batch_create")
    return h


def pdhcg_batch_solve(h, params: pdhcg_params, p_cat, x_cat, count: int):
    infos = (pdhcg_info * count)()
    st = lib().pdhcg_batch_solve(h, C.byref(params), _dev_ptr(p_cat, torch.float32, "p_cat"),
                                 _dev_ptr(x_cat, torch.float32, "x_cat"), infos)
    _check(st, "pdhcg_batch_solve", ok=(PDHCG_OK, PDHCG_MAX_ITER))
    return st, list(infos)


def pdhcg_batch_autotune(h, params: Optional[pdhcg_params], trial_iters: int
                         ) -> pdhcg_batch_schedule:
    out = pdhcg_batch_schedule()
    _check(lib().pdhcg_batch_autotune(h, C.byref(params) if params is not None else None,
                                      int(trial_iters), C.byref(out)), "pdhcg_batch_autotune")
    return out


def pdhcg_batch_backward(h, x_cat, p_cat, omega, unroll: int, ckpt_every: int, dL_dp_cat,
                         dL_du_cat, dL_dw_cat) -> None:
    import numpy as np
    om = np.ascontiguousarray(omega, dtype=np.float64)
    _check(lib().pdhcg_batch_backward(h, _dev_ptr(x_cat, torch.float32, "x_cat"),
                                      _dev_ptr(p_cat, torch.float32, "p_cat"), _host_ptr(om, "omega"),
                                      int(unroll), int(ckpt_every),
                                      _dev_ptr(dL_dp_cat, torch.float32, "dL_dp_cat"),
                                      _dev_ptr(dL_du_cat, torch.float32, "dL_du_cat"),
                                      _dev_ptr(dL_dw_cat, torch.float32, "dL_dw_cat")),
           "pdhcg_batch_backward")


def pdhcg_batch_layout(h, count: int):
    import numpy as np
    g = np.zeros(count + 1, np.int64)
    e = np.zeros(count + 1, np.int64)
    _check(lib().pdhcg_batch_layout(h, _host_ptr(g, "good_off"), _host_ptr(e, "edge_off")),
           "pdhcg_batch_layout")
    return g, e


def pdhcg_batch_destroy(h) -> None:
    if h:
        lib().pdhcg_batch_destroy(h)


class Batch:
    """Many independent markets solved in one persistent launch."""

    def __init__(self, batch, device="cuda", stream=None):
        dev = torch.device(device)
        self.count = int(batch.count)
        self.device = dev
        rp = torch.as_tensor(batch.row_ptr, dtype=torch.int32).to(dev).contiguous()
        col = torch.as_tensor(batch.col, dtype=torch.int32).to(dev).contiguous()
        u = torch.as_tensor(batch.u).to(dev, torch.float32).contiguous()
        w = torch.as_tensor(batch.w).to(dev, torch.float32).contiguous()
        self._h = pdhcg_batch_create(self.count, batch.n, batch.m, rp, col, u, w, stream)
        self.n_total = int(w.numel())
        self.good_off, self.edge_off = pdhcg_batch_layout(self._h, self.count)

    def close(self):
        if getattr(self, "_h", None):
            pdhcg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, params: Optional[pdhcg_params] = None, **kw):
        prm = params if params is not None else pdhcg_default_params(**kw)
        p = torch.empty(int(self.good_off[-1]), dtype=torch.float32, device=self.device)
        x = torch.empty(int(self.edge_off[-1]), dtype=torch.float32, device=self.device)
        st, infos = pdhcg_batch_solve(self._h, prm, p, x, self.count)
        return st, p, x, infos

    def backward(self, x, p, omega, dL_dp, unroll: int = 1024, ckpt_every: int = 32):
        """(dL/du, dL/dw), concatenated like the inputs, for every market
        (pdhcg_batch_backward); omega: each market's primal weight."""
        du = torch.empty(int(self.edge_off[-1]), dtype=torch.float32, device=self.device)
        dw = torch.empty(self.n_total, dtype=torch.float32, device=self.device)
        g = torch.as_tensor(dL_dp).to(self.device, torch.float32).contiguous()
        pdhcg_batch_backward(self._h, x.contiguous(), p.contiguous(), omega, unroll, ckpt_every, g,
                             du, dw)
        return du, dw

    def autotune(self, params: Optional[pdhcg_params] = None, trial_iters: int = 64):
        """Time the schedule candidates and keep the fastest (pdhcg_batch_autotune)."""
        return pdhcg_batch_autotune(self._h, params, trial_iters)


class FisherPrices(torch.autograd.Function):
    """Equilibrium prices of a linear Fisher market as a differentiable
    function of the utilities (CSR values) and budgets.

    ``p = FisherPrices.apply(u, w, row_ptr, col, m, params, unroll, ckpt_every)``

    Forward: restarted PDHCG (pdhcg_solve) with ``params`` (a pdhcg_params
    or None for the defaults).  Backward: pdhcg_backward from the solution
    with the solve's primal weight, ``unroll`` fixed-step iterations with a
    checkpoint every ``ckpt_every``; gradients for u and w (float32), None
    for the structure arguments."""

    @staticmethod
    def forward(ctx, u, w, row_ptr, col, m, params=None, unroll=1024, ckpt_every=32):
        M = Market(row_ptr, col, u.detach(), w.detach(), m=m, device=u.device)
        sol = M.solve(params)
        if sol.info.status not in (PDHCG_OK, PDHCG_MAX_ITER):
            M.close()
            raise PDHCGError(sol.info.status, "FisherPrices.forward")
        ctx.market = M
        ctx.omega = sol.info.omega
        ctx.unroll, ctx.ckpt = int(unroll), int(ckpt_every)
        ctx.save_for_backward(sol.x, sol.p)
        ctx.u_dtype, ctx.w_dtype = u.dtype, w.dtype
        return sol.p

    @staticmethod
    def backward(ctx, grad_p):
        x, p = ctx.saved_tensors
        M = ctx.market
        du, dw = M.backward(x, p, ctx.omega, grad_p.float(), ctx.unroll, ctx.ckpt)
        M.close()
        return (du.to(ctx.u_dtype), dw.to(ctx.w_dtype), None, None, None, None, None, None)
