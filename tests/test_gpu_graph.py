"""The evaluation captured once as a HIP graph (through torch's graph
capture on a side stream) and replayed: every replay, with eager work and
synchronisations between them, must reproduce the eager call bit for bit
(the path records only kernel launches: no memset nodes, no allocation)."""
import numpy as np
import pytest
import torch

from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_graph_replays_equal_eager():
    from paper_2606_06617_amd.api import Plan
    w = wl.water(nmol=500, L=24.8)
    N, C = w["pos"].shape[0], len(w["ps"])
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(w["pos"]).to(dev)
    q = torch.from_numpy(w["q"]).to(dev)
    plan = Plan(w["box"], w["ps"], r_c=5.0, c=12.024, grid=(40, 40, 40), support=8, max_atoms=N)
    ws = plan.new_workspace(dev)
    out = {"energy": torch.empty(3 * C + 1, dtype=torch.float64, device=dev),
           "forces": torch.empty((N, 3), dtype=torch.float32, device=dev),
           "virial": torch.empty(6, dtype=torch.float64, device=dev)}
    side = torch.cuda.Stream(device=dev)
    print("case graph capture and replay: water", N, "atoms", flush=True)
    with torch.cuda.stream(side):
        plan.execute(pos, q, workspace=ws, out=out, stream=side)
    side.synchronize()
    ref = {k: v.clone() for k, v in out.items()}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        plan.execute(pos, q, workspace=ws, out=out, stream=side)
    side.synchronize()
    for rep in range(4):
        for v in out.values():
            v.fill_(np.nan)
        # eager work of the program between replays
        other = plan.execute(pos, q * 0.5)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k in out:
            assert torch.equal(out[k], ref[k]), (rep, k)
        assert not torch.equal(other["energy"], ref["energy"])
