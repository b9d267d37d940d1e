"""Plan tables are pooled, not freed: a plan destroyed while its last call is
still queued must not hand its device table to the next plan before that
call has run.  Plan A is evaluated on a busy stream and dropped at once;
plan B (same table size, so a pool candidate) is built and run on another
stream while A's call is still in flight.  A's results must equal its
evaluation on an idle device, bit for bit."""
import pytest
import torch

from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_destroyed_plan_table_not_reused_while_in_flight():
    from paper_2606_06617_amd.api import Plan
    w = wl.random_box(20000, ps=(1, 6), seed=51)
    grid = (96, 96, 96)
    print("case plan reuse, grid", grid, flush=True)
    pos = torch.from_numpy(w["pos"]).cuda()
    q = torch.from_numpy(w["q"]).cuda()
    ref_plan = Plan(w["box"], w["ps"], grid=grid, support=8, max_atoms=pos.shape[0])
    ref = ref_plan.execute(pos, q, forces=True, virial=True)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items() if torch.is_tensor(v)}
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    outs = []
    for rep in range(4):
        with torch.cuda.stream(sa):
            pa = Plan(w["box"], w["ps"], grid=grid, support=8, max_atoms=pos.shape[0])
            for _ in range(3):                    # keep stream A busy
                out = pa.execute(pos, q, forces=True, virial=True, stream=sa)
            outs.append(out)
            del pa                                 # destroyed with its calls still queued
        with torch.cuda.stream(sb):
            w2 = wl.random_box(20000, ps=(1, 6), seed=60 + rep)
            pb = Plan(w2["box"], w2["ps"], grid=grid, support=8, max_atoms=20000)
            pb.execute(torch.from_numpy(w2["pos"]).cuda(), torch.from_numpy(w2["q"]).cuda(),
                       forces=True, virial=True, stream=sb)
            del pb
    torch.cuda.synchronize()
    for out in outs:
        for k in ("energy", "forces", "virial"):
            assert torch.equal(out[k], ref[k]), k
