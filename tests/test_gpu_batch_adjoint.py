"""The batched flat-array calls and the batched adjoint on the GPU: every
structure of a batch equals its standalone call bit for bit (forward with
forces, virial and potentials; energy-only forward followed by the batched
backward against the single-structure backward), and the batched gradients
through torch.autograd against the oracle's potentials and forces (the
derivatives of the direct Fourier sum) for a few structures."""
import numpy as np
import pytest
import torch

from oracle import reciprocal
from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _setup(k=10):
    from paper_2606_06617_amd.api import Batch, Plan
    structs = wl.diff_batch()[:k]
    plans = [Plan(st["box"], st["ps"], r_c=5.0, c=12.024, grid=st["grid"], support=8, max_atoms=st["pos"].shape[0])
             for st in structs]
    inputs = [(torch.from_numpy(st["pos"]).cuda(), torch.from_numpy(st["q"]).cuda()) for st in structs]
    batch = Batch(plans, [p.shape[0] for p, _ in inputs])
    pos, q = Batch.concat(inputs)
    return structs, plans, inputs, batch, pos, q


def test_flat_batch_equals_standalone_bitwise():
    structs, plans, inputs, batch, pos, q = _setup()
    print("case flat batch of", batch.n, "structures,", batch.atoms, "atoms", flush=True)
    out = batch.execute(pos, q, forces=True, virial=True, potential=True)
    torch.cuda.synchronize()
    a0 = q0 = e0 = 0
    for i, (plan, (p, c)) in enumerate(zip(plans, inputs)):
        ref = plan.execute(p, c, forces=True, virial=True, potential=True)
        torch.cuda.synchronize()
        N, C = p.shape[0], plan.C
        assert torch.equal(out["energy"][e0:e0 + 3 * C + 1], ref["energy"])
        assert torch.equal(out["forces"][a0:a0 + N], ref["forces"])
        assert torch.equal(out["virial"][i], ref["virial"])
        assert torch.equal(out["potential"][q0:q0 + C * N].view(C, N), ref["potential"])
        a0 += N
        q0 += C * N
        e0 += 3 * C + 1


def test_batched_adjoint_equals_single_backward_bitwise():
    structs, plans, inputs, batch, pos, q = _setup()
    ws = batch.new_workspace("cuda")
    batch.execute(pos, q, forces=False, virial=False, potential=False, workspace=ws)
    g = torch.linspace(0.5, 1.5, sum(batch.Cs), dtype=torch.float64, device="cuda")
    gq, gp = batch.backward(ws, pos, q, g)
    torch.cuda.synchronize()
    a0 = q0 = c0 = 0
    for plan, (p, c) in zip(plans, inputs):
        N, C = p.shape[0], plan.C
        w1 = plan.new_workspace("cuda")
        plan.execute(p, c, forces=False, virial=False, potential=False, workspace=w1)
        rq, rp = plan.backward(w1, p, c, g[c0:c0 + C])
        torch.cuda.synchronize()
        assert torch.equal(gq[q0:q0 + C * N].view(C, N), rq)
        assert torch.equal(gp[a0:a0 + N], rp)
        a0 += N
        q0 += C * N
        c0 += C


def test_autograd_batch_gradients_against_oracle():
    from paper_2606_06617_amd.api import lr_energy_batch
    structs, plans, inputs, batch, pos, q = _setup(k=4)
    posr = pos.clone().requires_grad_(True)
    qr = q.clone().requires_grad_(True)
    e = lr_energy_batch(posr, qr, batch)
    weights = torch.tensor([1.0, -0.5, 2.0, 0.25], dtype=torch.float64, device="cuda")
    (e * weights).sum().backward()
    torch.cuda.synchronize()
    a0 = q0 = 0
    for i, (st, plan) in enumerate(zip(structs, plans)):
        N, C = st["pos"].shape[0], plan.C
        r = reciprocal.evaluate(st["pos"].astype(np.float64), st["q"].astype(np.float64), st["box"], st["ps"],
                                12.024, 5.0)
        Er = float((r["Ek"] + r["E0"]).sum())
        assert abs(float(e[i].detach()) - Er) <= 1e-5 * abs(Er)
        w = float(weights[i])
        gq = qr.grad[q0:q0 + C * N].view(C, N).cpu().numpy().astype(np.float64)
        gp = posr.grad.view(-1, 3)[a0:a0 + N].cpu().numpy().astype(np.float64)
        assert np.sqrt(np.mean((gq - w * r["phi"]) ** 2)) <= 1e-4 * np.sqrt(np.mean((w * r["phi"]) ** 2))
        assert np.sqrt(np.mean((gp + w * r["F"]) ** 2)) <= 1e-4 * np.sqrt(np.mean((w * r["F"]) ** 2))
        a0 += N
        q0 += C * N
