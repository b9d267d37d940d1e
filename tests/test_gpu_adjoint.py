"""The hand-written adjoint behind torch.autograd.Function (energy-only
forward, scaled inverse transforms + gather in backward) against the
forward path's own forces/potentials, the FP64 oracle's gradients (which
the CPU suite pins to finite differences), and a chain rule through
learned charges."""
import numpy as np
import pytest
import torch

from oracle import reciprocal
from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu

C_MOL, RC = 12.024, 5.0


def _rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


def _setup(w, grid, P):
    from paper_2606_06617_amd.api import Plan
    print("case", w["name"], grid, P, flush=True)
    pos = torch.from_numpy(w["pos"]).cuda()
    q = torch.from_numpy(w["q"]).cuda()
    plan = Plan(w["box"], w["ps"], r_c=RC, c=C_MOL, grid=grid, support=P, max_atoms=pos.shape[0])
    return plan, pos, q


def test_adjoint_matches_forward_outputs():
    from paper_2606_06617_amd.api import lr_energy
    w = wl.water(nmol=300, L=20.0)
    plan, pos, q = _setup(w, (32, 32, 32), 8)
    ref = plan.execute(pos, q, forces=True, virial=False, potential=True)
    p = pos.clone().requires_grad_(True)
    qq = q.clone().requires_grad_(True)
    E = lr_energy(p, qq, plan)
    E.backward()
    torch.cuda.synchronize()
    e = ref["energy"].cpu().numpy()[:-1].reshape(-1, 3)
    assert abs(E.item() - (e[:, 0] + e[:, 1]).sum()) <= 1e-12 * abs(E.item())
    assert torch.allclose(p.grad, -ref["forces"], rtol=1e-6, atol=1e-7 * ref["forces"].abs().max().item())
    assert torch.allclose(qq.grad, ref["potential"], rtol=1e-6, atol=1e-7 * ref["potential"].abs().max().item())


def test_adjoint_against_oracle_gradients():
    from paper_2606_06617_amd.api import lr_energy
    w = wl.random_box(800, ps=(1, 6), seed=41, neutral=False)
    plan, pos, q = _setup(w, (24, 24, 24), 8)
    p = pos.clone().requires_grad_(True)
    qq = q.clone().requires_grad_(True)
    lr_energy(p, qq, plan).backward()
    torch.cuda.synchronize()
    r = reciprocal.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), w["box"], w["ps"],
                            C_MOL, RC)
    assert _rel_rms(-p.grad.cpu().numpy().astype(np.float64), r["F"]) < 1e-4
    assert _rel_rms(qq.grad.cpu().numpy().astype(np.float64), r["phi"]) < 1e-4


def test_chain_rule_through_learned_charges():
    # q = theta * base (a per-channel scale, as an MLIP head would output);
    # dE/dtheta_c = sum_i base_ci dE/dq_ci = 2 E_c / theta_c for a quadratic E
    from paper_2606_06617_amd.api import lr_energy
    w = wl.random_box(500, ps=(1, 6), seed=42)
    plan, pos, q = _setup(w, (24, 24, 24), 8)
    theta = torch.tensor([0.7, 1.3], device="cuda", requires_grad=True)
    qs = theta[:, None] * q
    E = lr_energy(pos, qs.contiguous(), plan)
    E.backward()
    torch.cuda.synchronize()
    ref = plan.execute(pos, (theta.detach()[:, None] * q).contiguous(), forces=False, virial=False)
    e = ref["energy"].cpu().numpy()[:-1].reshape(-1, 3)
    ec = e[:, 0] + e[:, 1]
    want = 2.0 * ec / theta.detach().cpu().numpy()
    assert np.allclose(theta.grad.cpu().numpy(), want, rtol=2e-5)


def test_second_call_reuses_plan_and_scales_gradient():
    from paper_2606_06617_amd.api import lr_energy
    w = wl.random_box(300, ps=(1,), seed=43)
    plan, pos, q = _setup(w, (20, 20, 20), 6)
    g1 = None
    for scale in (1.0, -2.5):
        p = pos.clone().requires_grad_(True)
        (scale * lr_energy(p, q, plan)).backward()
        torch.cuda.synchronize()
        if g1 is None:
            g1 = p.grad.clone()
        else:
            # linear in the upstream gradient up to FP32 rounding of the scaled transforms
            err = ((p.grad + 2.5 * g1).norm() / (2.5 * g1).norm()).item()
            assert err < 1e-6, err
