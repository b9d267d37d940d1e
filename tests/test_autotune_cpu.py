"""The autotuner's model of the kernels' tile limits agrees with the
library's own validation: over every tile shape that divides a grid, the
tiles it calls feasible pass plan validation (the CPU-only run then stops
at the device allocation) and the others are refused as unsupported."""
import ctypes
import itertools

import pytest

from paper_2606_06617_amd import _lib, autotune

UNSUPPORTED, DEVICE = 2, 4


def _status(grid, P, tile):
    prm = _lib.make_params((20.0, 20.0, 20.0), [1], 5.0, 12.024, 1e-5, grid, P, 0.0, tile)
    h = ctypes.c_void_p()
    return _lib.lib().pswflr_plan_create(ctypes.byref(prm), 100, ctypes.byref(h))


@pytest.mark.parametrize("grid,P", [((32, 32, 32), 6), ((48, 40, 36), 8), ((40, 36, 48), 4)])
def test_feasibility_model_matches_library(grid, P):
    divs = [autotune._divisors(m) for m in grid]
    seen_ok = 0
    for tile in itertools.product(*divs):
        want = autotune.tile_feasible(grid, tile, P)
        got = _status(grid, P, tile)
        assert got in (UNSUPPORTED, DEVICE), (tile, got)
        assert (got == DEVICE) == want, (grid, P, tile, got, want)
        seen_ok += want
    assert seen_ok > 0


def test_cache_is_reread_only_when_the_file_changes(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("PSWFLR_AUTOTUNE_CACHE", str(path))
    key = autotune.key_for("gfx950", (40, 40, 40), 8, 2, 3000)
    assert autotune.lookup("gfx950", (40, 40, 40), 8, 2, 3000) is None
    path.write_text('{"%s": {"tile": [8, 8, 8]}}' % key)
    assert autotune.lookup("gfx950", (40, 40, 40), 8, 2, 3000)["tile"] == [8, 8, 8]
    path.write_text('{"%s": {"tile": [8, 8, 20]}}' % key)      # same size, new contents
    import os
    st = os.stat(path)
    os.utime(path, ns=(st.st_atime_ns, st.st_mtime_ns + 1_000_000))
    assert autotune.lookup("gfx950", (40, 40, 40), 8, 2, 3000)["tile"] == [8, 8, 20]
    monkeypatch.setenv("PSWFLR_AUTOTUNE", "0")
    assert autotune.cached_tile((40, 40, 40), 8, 2, 3000) is None
