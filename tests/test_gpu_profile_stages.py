"""Per-stage timing through the C ABI: with a stage mask only the named
stages carry event records and report launches; the results are the same
with timing on, off or restricted; a mask bit past the last stage is an
argument error."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu

NUM_STAGES, GATHER, SPREAD = 10, 9, 2


def _read(L, plan):
    from paper_2606_06617_amd import _lib
    ms = (ctypes.c_double * NUM_STAGES)()
    cnt = (ctypes.c_int64 * NUM_STAGES)()
    _lib.check(L.pswflr_profile_read(plan.handle, ms, cnt))
    return np.array(ms[:]), np.array(cnt[:])


def test_stage_mask_times_only_named_stages():
    from paper_2606_06617_amd import _lib
    from paper_2606_06617_amd.api import Plan
    L = _lib.lib()
    w = wl.random_box(3000, ps=(1, 6), seed=7)
    print("case profile mask n 3000 grid 32^3", flush=True)
    plan = Plan(w["box"], w["ps"], r_c=5.0, c=12.024, grid=(32, 32, 32), support=6, max_atoms=3000,
                autotune=False)
    pos, q = torch.from_numpy(w["pos"]).cuda(), torch.from_numpy(w["q"]).cuda()
    ref = plan.execute(pos, q, forces=True, virial=True)
    torch.cuda.synchronize()

    _lib.check(L.pswflr_profile_stages(plan.handle, (1 << GATHER) | (1 << SPREAD)))
    for _ in range(3):
        out = plan.execute(pos, q, forces=True, virial=True)
    ms, cnt = _read(L, plan)
    _lib.check(L.pswflr_profile_stages(plan.handle, 0))
    assert cnt[GATHER] == 3 and cnt[SPREAD] >= 3
    assert all(cnt[s] == 0 for s in range(NUM_STAGES) if s not in (GATHER, SPREAD))
    assert ms[GATHER] > 0 and ms[SPREAD] > 0
    for k in ("energy", "forces", "virial"):
        assert torch.equal(out[k], ref[k]), k

    # every stage, then off: nothing is left to read
    _lib.check(L.pswflr_profile_enable(plan.handle, 1))
    plan.execute(pos, q, forces=True, virial=True)
    _, cnt = _read(L, plan)
    assert all(cnt[s] >= 1 for s in (0, 2, 3, 4, 5, 6, 7, 8, 9))
    _lib.check(L.pswflr_profile_enable(plan.handle, 0))
    plan.execute(pos, q, forces=True, virial=True)
    _, cnt = _read(L, plan)
    assert cnt.sum() == 0

    # a bit past the last stage is refused and leaves timing off
    st = L.pswflr_profile_stages(plan.handle, 1 << NUM_STAGES)
    assert st != 0
    plan.execute(pos, q, forces=True, virial=True)
    _, cnt = _read(L, plan)
    assert cnt.sum() == 0
