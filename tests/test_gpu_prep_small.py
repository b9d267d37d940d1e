"""Structures of up to 2048 atoms bin, order and sum their charges in one
single-workgroup launch; larger ones, and batched calls, take the
multi-launch path.  The two paths must agree bit for bit: the records, the
order inside each tile (ascending caller index) and the fixed-order charge
sums are the same.  Compared here through a standalone call against a
batched call of the same structure, at sizes around the threshold, for a
crowded structure (every atom in one tile), and against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import reciprocal
from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu

C_MOL, RC = 12.024, 5.0


def _both(w, support=6):
    from paper_2606_06617_amd.api import Plan, execute_batch
    n = w["pos"].shape[0]
    plan = Plan(w["box"], w["ps"], r_c=RC, c=C_MOL, grid=w["grid"], support=support, max_atoms=max(1, n),
                autotune=False)
    pos, q = torch.from_numpy(w["pos"]).cuda(), torch.from_numpy(w["q"]).cuda()
    alone = plan.execute(pos, q, forces=True, virial=True, potential=True)
    outs, _ = execute_batch([plan], [(pos, q)], potential=True)
    torch.cuda.synchronize()
    return alone, outs[0]


@pytest.mark.parametrize("n", [1, 37, 2047, 2048, 2049])
def test_one_launch_prep_equals_batched_path(n):
    w = wl.random_box(n, ps=(1, 6), seed=100 + n)
    w["grid"] = (48, 48, 48) if n > 1000 else (24, 24, 24)
    print("case n", n, "grid", w["grid"], flush=True)
    alone, batched = _both(w)
    for k in ("energy", "forces", "virial", "potential"):
        assert torch.equal(alone[k], batched[k]), k


def test_one_launch_prep_crowded_tile():
    # every atom inside one tile: the in-tile order is decided by counting
    rng = np.random.default_rng(5)
    n = 2000
    box = np.array([20.0, 20.0, 20.0])
    pos = (rng.uniform(0.0, 0.8, size=(n, 3)) + 3.0).astype(np.float32)
    q = rng.normal(0.0, 0.5, size=(2, n))
    q -= q.mean(axis=1, keepdims=True)
    w = {"pos": pos, "q": q.astype(np.float32), "box": box, "ps": [1, 6], "grid": (32, 32, 32)}
    print("case crowded n", n, flush=True)
    alone, batched = _both(w)
    for k in ("energy", "forces", "virial", "potential"):
        assert torch.equal(alone[k], batched[k]), k
    r = reciprocal.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), box, w["ps"], C_MOL, RC)
    e = alone["energy"].cpu().numpy()[:-1].reshape(-1, 3)
    Eg, Er = e[:, 0] + e[:, 1], r["Ek"] + r["E0"]
    assert np.all(np.abs(Eg - Er) <= 1e-5 * np.abs(Er)), (Eg, Er)
    F = alone["forces"].cpu().numpy().astype(np.float64)
    assert np.sqrt(np.mean((F - r["F"]) ** 2)) <= 1e-4 * np.sqrt(np.mean(r["F"] ** 2))
