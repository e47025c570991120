"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/pdhcg.h, its structs have the layout the header gives,
defaults follow Sec. 5, and host-side validation returns the documented
status codes."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2506_06258_amd import pdhcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pdhcg.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pdhcg_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = pdhcg.lib()
    names = declared_functions()
    assert set(names) == set(pdhcg.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", pdhcg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (pdhcg_[a-z_]+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)


def _c_layout(struct_name, fields):
    prog = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void){",
            f'printf("%zu\\n", sizeof({struct_name}));']
    for f in fields:
        prog.append(f'printf("%zu\\n", offsetof({struct_name}, {f}));')
    prog.append("return 0;}")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        exe = os.path.join(d, "l")
        open(c, "w").write("\n".join(prog))
        subprocess.run(["gcc", "-o", exe, c], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True,
                                                check=True).stdout.split()]
    return vals[0], vals[1:]


@pytest.mark.parametrize("cls,name", [(pdhcg.pdhcg_params, "pdhcg_params"),
                                      (pdhcg.pdhcg_info, "pdhcg_info"),
                                      (pdhcg.pdhcg_batch_schedule, "pdhcg_batch_schedule")])
def test_struct_layout_matches_header(cls, name):
    fields = [f for f, _ in cls._fields_]
    size, offs = _c_layout(name, fields)
    assert C.sizeof(cls) == size
    assert [getattr(cls, f).offset for f in fields] == offs


def test_defaults_follow_paper():
    prm = pdhcg.pdhcg_default_params()
    assert prm.tol == 1e-4
    assert (prm.beta_sufficient, prm.beta_necessary, prm.beta_artificial) == (0.2, 0.8, 0.2)
    assert prm.theta == 0.2
    assert prm.omega_check_every == 3
    assert prm.sections == 32
    assert prm.normalize_rows == 1
    assert prm.step_mode == pdhcg.PDHCG_STEP_ADAPTIVE
    assert prm.restart == pdhcg.PDHCG_RESTART_ADAPTIVE
    assert pdhcg.pdhcg_abi_version() == 1


def test_status_strings():
    for st in (0, 1, -1, -2, -3, -4, -5, -6):
        assert pdhcg.pdhcg_status_string(st)
    assert pdhcg.pdhcg_status_string(12345) == "unknown status"


def _ok_market():
    row_ptr = np.array([0, 2, 3], np.int32)
    col = np.array([0, 1, 1], np.int32)
    u = np.array([1.0, 0.5, 2.0], np.float32)
    w = np.array([1.0, 1.0], np.float32)
    return row_ptr, col, u, w


def test_validate_host_accepts_valid_market():
    rp, col, u, w = _ok_market()
    assert pdhcg.pdhcg_validate_host(2, 2, 3, rp, col, u, w) == pdhcg.PDHCG_OK


@pytest.mark.parametrize("mutate,code", [
    (lambda rp, c, u, w: (rp, np.array([1, 0, 1], np.int32), u, w), pdhcg.PDHCG_ERR_ARG),
    (lambda rp, c, u, w: (rp, np.array([0, 0, 1], np.int32), u, w), pdhcg.PDHCG_ERR_ARG),
    (lambda rp, c, u, w: (rp, np.array([0, 2, 1], np.int32), u, w), pdhcg.PDHCG_ERR_ARG),
    (lambda rp, c, u, w: (rp, c, np.array([1, -1, 2], np.float32), w), pdhcg.PDHCG_ERR_ARG),
    (lambda rp, c, u, w: (rp, c, np.array([1, np.nan, 2], np.float32), w), pdhcg.PDHCG_ERR_ARG),
    (lambda rp, c, u, w: (rp, c, u, np.array([1, 0], np.float32)), pdhcg.PDHCG_ERR_ARG),
    (lambda rp, c, u, w: (rp, c, u, np.array([1, np.inf], np.float32)), pdhcg.PDHCG_ERR_ARG),
    (lambda rp, c, u, w: (rp, c, np.array([0, 0, 2], np.float32), w), pdhcg.PDHCG_ERR_ASSUMPTION),
    (lambda rp, c, u, w: (rp, c, np.array([1, 0.5, 0], np.float32), w), pdhcg.PDHCG_ERR_ASSUMPTION),
])
def test_validate_host_rejects(mutate, code):
    rp, col, u, w = mutate(*_ok_market())
    assert pdhcg.pdhcg_validate_host(2, 2, 3, rp, col, u, w) == code
    assert pdhcg.pdhcg_last_error()


def test_validate_host_rejects_empty_buyer():
    rp = np.array([0, 2, 2], np.int32)
    col = np.array([0, 1], np.int32)
    u = np.array([1.0, 0.5], np.float32)
    w = np.array([1.0, 1.0], np.float32)
    assert pdhcg.pdhcg_validate_host(2, 2, 2, rp, col, u, w) == pdhcg.PDHCG_ERR_ASSUMPTION


def test_validate_host_rejects_good_without_buyer():
    rp, col, u, w = _ok_market()
    assert pdhcg.pdhcg_validate_host(2, 3, 3, rp, col, u, w) == pdhcg.PDHCG_ERR_ASSUMPTION


def test_validate_host_rejects_bad_sizes():
    rp, col, u, w = _ok_market()
    assert pdhcg.pdhcg_validate_host(0, 2, 3, rp, col, u, w) == pdhcg.PDHCG_ERR_ARG
    assert pdhcg.pdhcg_validate_host(2, 2, 4, rp, col, u, w) == pdhcg.PDHCG_ERR_ARG


def test_null_handles_are_rejected_without_gpu():
    L = pdhcg.lib()
    prm = pdhcg.pdhcg_default_params()
    assert L.pdhcg_solve(None, C.byref(prm), 0, None, None, None, None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_kkt(None, None, None, None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_set_budgets(None, None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_market_lds_goods(None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_row_prox(None, None, None, 1.0, None, None, None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_backward(None, None, None, 1.0, 8, 4, None, None, None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_market_bins(None, 0, None, None, None) == pdhcg.PDHCG_ERR_ARG
    sch = pdhcg.pdhcg_batch_schedule()
    assert L.pdhcg_batch_autotune(None, C.byref(prm), 8, C.byref(sch)) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_batch_solve(None, C.byref(prm), None, None, None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_batch_layout(None, None, None) == pdhcg.PDHCG_ERR_ARG
    assert L.pdhcg_batch_backward(None, None, None, None, 8, 4, None, None, None) == pdhcg.PDHCG_ERR_ARG
    L.pdhcg_market_destroy(None)
    L.pdhcg_batch_destroy(None)
