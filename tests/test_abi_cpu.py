"""Host-side checks of the C ABI that need no GPU: the built library loads,
exports every function include/pswflr.h declares, the ctypes structs match
the header, and argument errors are reported before any device call."""
import ctypes
import os
import re

import pytest

from paper_2606_06617_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pswflr.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(pswflr_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("pswflr_plan_create", "pswflr_plan_info", "pswflr_plan_destroy", "pswflr_execute",
              "pswflr_backward", "pswflr_execute_batch", "pswflr_batch_workspace",
              "pswflr_status_string", "pswflr_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for n in _declared():
        assert hasattr(L, n), n


def test_status_strings():
    L = _lib.lib()
    for s in range(7):
        assert L.pswflr_status_string(s)


def _create(**kw):
    L = _lib.lib()
    base = dict(box=(20.0, 20.0, 20.0), ps=[1], r_c=5.0, c=12.024, tol=1e-5, grid=(32, 32, 32),
                support=6, c_spread=16.4, tile=None)
    base.update(kw)
    prm = _lib.make_params(base["box"], base["ps"], base["r_c"], base["c"], base["tol"], base["grid"],
                           base["support"], base["c_spread"], base["tile"])
    h = ctypes.c_void_p()
    return L.pswflr_plan_create(ctypes.byref(prm), 100, ctypes.byref(h))


@pytest.mark.parametrize("kw,status", [
    (dict(ps=[7]), 1),
    (dict(ps=[0]), 1),
    (dict(box=(0.0, 20.0, 20.0)), 1),
    (dict(r_c=-1.0), 1),
    (dict(support=9), 1),
    (dict(grid=(32, 32, 31)), 2),      # odd M_z
    (dict(grid=(32, 14, 32)), 2),      # 7 is not a supported radix
    (dict(grid=(8, 8, 8)), 1),         # Nyquist: k_c h / pi >= 1
    (dict(tile=(5, 16, 16)), 1),       # tile does not divide the grid
    (dict(tile=(32, 32, 32)), 2),      # too many spreading blocks
])
def test_argument_errors_before_device(kw, status):
    assert _create(**kw) == status


def test_struct_layout_matches_header():
    # offsets the C side relies on (x86-64 SysV layout of pswflr_params)
    assert _lib.Params.box.offset == 264      # 4 + 4*64, padded to 8
    assert ctypes.sizeof(_lib.IO) == 7 * 8
