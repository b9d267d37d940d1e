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




SKEWED = ((12.0, 0.0, 0.0), (3.0, 11.0, 0.0), (-2.0, 2.5, 10.0))


@pytest.mark.parametrize("cell,status", [
    (((12.0, 0.0, 0.0), (24.0, 0.0, 0.0), (0.0, 0.0, 10.0)), 1),     # singular
    (((12.0, 0.0, 0.0), (0.0, float("nan"), 0.0), (0.0, 0.0, 10.0)), 1),
    (((12.0, 0.0, 0.0), (12.0, 1e-3, 0.0), (0.0, 0.0, 10.0)), 1),    # degenerate: reduce the basis
])
def test_cell_errors_before_device(cell, status):
    assert _create(box=cell, grid=(24, 24, 24)) == status


def test_cell_nyquist_uses_lattice_vector_lengths():
    # |a_1| = 11.4 A on 10 points: k_c h / pi = 2.4048 * 1.14 / pi > 0.87 is
    # fine; on 8 points it exceeds 1
    assert _create(box=SKEWED, grid=(24, 8, 24)) == 1


def test_struct_layout_matches_header(tmp_path):
    # offsets and sizes of the parameter and info structs as the C compiler
    # lays them out, against the ctypes mirrors
    src = tmp_path / "layout.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "pswflr.h"\n'
        'int main(void) { printf("%zu %zu %zu %zu %zu %zu %zu\\n", offsetof(pswflr_params, box), '
        'offsetof(pswflr_params, flags), offsetof(pswflr_params, cell), sizeof(pswflr_params), '
        'offsetof(pswflr_info, cell), sizeof(pswflr_info), sizeof(pswflr_io)); return 0; }\n')
    exe = str(tmp_path / "layout")
    import subprocess
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", exe], check=True)
    got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [_lib.Params.box.offset, _lib.Params.flags.offset, _lib.Params.cell.offset,
                   ctypes.sizeof(_lib.Params), _lib.Info.cell.offset, ctypes.sizeof(_lib.Info),
                   ctypes.sizeof(_lib.IO)]
