"""The allocation-free entry point (pswflr_execute_noalloc) through the C
ABI on the GPU: for callers that cannot allocate device memory.  Its
results must equal pswflr_execute's with a caller workspace bit for bit
(same kernels, same order) on two calls in a row on one plan, the second
with fewer atoms (the scratch keeps the first call's contents, so anything
not cleared would show), and plans whose workspace exceeds the scratch are
refused with a workspace error."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2606_06617_amd import _lib
from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr() if t is not None else 0)


def _noalloc(plan, pos, q):
    N, C = pos.shape[0], plan.C
    dev = pos.device
    e = torch.empty(3 * C + 1, dtype=torch.float64, device=dev)
    f = torch.empty((N, 3), dtype=torch.float32, device=dev)
    v = torch.empty(6, dtype=torch.float64, device=dev)
    p = torch.empty((C, N), dtype=torch.float32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(_lib.lib().pswflr_execute_noalloc(plan.handle, st, N, _ptr(pos), _ptr(q), _ptr(e), _ptr(f),
                                                 _ptr(v), _ptr(p)))
    torch.cuda.synchronize()
    return {"energy": e, "forces": f, "virial": v, "potential": p}


def test_noalloc_equals_execute_twice_shrinking():
    from paper_2606_06617_amd.api import Plan
    w = wl.random_box(3000, ps=(1, 6), seed=61, aspect=(1.0, 1.1, 0.9))
    plan = Plan(w["box"], w["ps"], r_c=5.0, c=12.024, grid=(40, 45, 36), support=8, max_atoms=3000)
    assert plan.workspace_bytes <= 64 << 20
    pos = torch.from_numpy(w["pos"]).cuda()
    q = torch.from_numpy(w["q"]).cuda()
    for n in (3000, 1700):
        print("case noalloc N", n, flush=True)
        pn, qn = pos[:n].contiguous(), q[:, :n].contiguous()
        a = _noalloc(plan, pn, qn)
        b = plan.execute(pn, qn, forces=True, virial=True, potential=True)
        torch.cuda.synchronize()
        for k in ("energy", "forces", "virial", "potential"):
            assert torch.equal(a[k], b[k]), (n, k)
        assert np.isfinite(a["energy"].cpu().numpy()).all()


def test_noalloc_refuses_plans_beyond_the_scratch():
    from paper_2606_06617_amd.api import Plan
    big = Plan((200.0, 200.0, 200.0), (1, 6), r_c=5.0, c=12.024, grid=(256, 256, 256), support=8,
               max_atoms=10)
    assert big.workspace_bytes > 64 << 20
    pos = torch.zeros((10, 3), dtype=torch.float32, device="cuda")
    q = torch.zeros((2, 10), dtype=torch.float32, device="cuda")
    with pytest.raises(_lib.PswflrError, match="scratch"):
        _noalloc(big, pos, q)
