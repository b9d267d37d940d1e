"""Batched execution (one launch per stage over many uneven structures):
every structure's result equals its standalone evaluation bit for bit (the
kernels see only that structure's buffers and reduce in a fixed order), and
matches the FP64 oracle to the parity bar."""
import numpy as np
import pytest
import torch

from oracle import reciprocal
from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu

C_MOL, RC = 12.024, 5.0


def _plans(ws_list, support=8):
    from paper_2606_06617_amd.api import Plan
    return [Plan(w["box"], w["ps"], r_c=RC, c=C_MOL, grid=w["grid"], support=support,
                 max_atoms=w["pos"].shape[0]) for w in ws_list]


def test_batch_equals_standalone_bitwise():
    from paper_2606_06617_amd.api import execute_batch
    structs = wl.diff_batch(nstruct=12, seed=7, nmin=200, nmax=2500)
    print("batch of", len(structs), [w["pos"].shape[0] for w in structs], flush=True)
    plans = _plans(structs)
    inputs = [(torch.from_numpy(w["pos"]).cuda(), torch.from_numpy(w["q"]).cuda()) for w in structs]
    outs, _ = execute_batch(plans, inputs, potential=True)
    torch.cuda.synchronize()
    for plan, (pos, q), o in zip(plans, inputs, outs):
        ref = plan.execute(pos, q, forces=True, virial=True, potential=True)
        torch.cuda.synchronize()
        for k in ("energy", "forces", "virial", "potential"):
            assert torch.equal(o[k], ref[k]), k


def test_batch_against_oracle_and_mixed_sizes():
    from paper_2606_06617_amd.api import execute_batch
    structs = wl.diff_batch(nstruct=5, seed=8, nmin=200, nmax=1200)
    structs.append(wl.random_box(0, ps=(1, 6), seed=1))   # an empty structure in the mix
    structs[-1]["grid"] = (16, 16, 16)
    structs[-1]["box"] = np.array([10.0, 10.0, 10.0])
    plans = _plans(structs)
    inputs = [(torch.from_numpy(w["pos"]).cuda(), torch.from_numpy(w["q"]).cuda()) for w in structs]
    outs, _ = execute_batch(plans, inputs)
    torch.cuda.synchronize()
    for w, o in zip(structs[:-1], outs[:-1]):
        r = reciprocal.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), w["box"], w["ps"],
                                C_MOL, RC)
        e = o["energy"].cpu().numpy()[:-1].reshape(-1, 3)
        Eg, Er = e[:, 0] + e[:, 1], r["Ek"] + r["E0"]
        assert np.all(np.abs(Eg - Er) <= 1e-5 * np.abs(Er))
        F = o["forces"].cpu().numpy().astype(np.float64)
        assert np.sqrt(np.mean((F - r["F"]) ** 2)) <= 1e-4 * np.sqrt(np.mean(r["F"] ** 2))
    assert np.all(outs[-1]["energy"].cpu().numpy() == 0.0)


def test_batch_mixed_supports_and_crowded_entry_bitwise():
    # entries with every support from 3 to 8 (one kernel variant each in the
    # spread, a per-entry switch in the gather) and a crowded box whose tiles
    # hold hundreds of atoms (many spread flushes and gather passes)
    from paper_2606_06617_amd.api import Plan, execute_batch
    structs = wl.diff_batch(nstruct=6, seed=9, nmin=200, nmax=1500)
    supports = [3, 4, 5, 6, 7, 8]
    rng = np.random.default_rng(405)
    N, L = 900, 18.0
    pos = ((rng.uniform(-2.0, 2.0, (N, 3)) + np.array([9.0, 0.2, 17.7])) % L).astype(np.float32)
    q = rng.normal(0.0, 1.0, (2, N))
    q = (q - q.mean(axis=1, keepdims=True)).astype(np.float32)
    structs.append({"pos": pos, "q": q, "box": np.array([L, L, L]), "ps": (1, 6), "grid": (36, 36, 36)})
    supports.append(8)
    print("batch supports", supports, "atoms", [w["pos"].shape[0] for w in structs], flush=True)
    plans = [Plan(w["box"], w["ps"], r_c=RC, c=C_MOL, grid=w["grid"], support=P, max_atoms=w["pos"].shape[0])
             for w, P in zip(structs, supports)]
    inputs = [(torch.from_numpy(w["pos"]).cuda(), torch.from_numpy(w["q"]).cuda()) for w in structs]
    outs, _ = execute_batch(plans, inputs, potential=True)
    torch.cuda.synchronize()
    for P, plan, (p, qq), o in zip(supports, plans, inputs, outs):
        ref = plan.execute(p, qq, forces=True, virial=True, potential=True)
        torch.cuda.synchronize()
        for k in ("energy", "forces", "virial", "potential"):
            assert torch.equal(o[k], ref[k]), (P, k)
    w = structs[-1]
    r = reciprocal.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), w["box"], w["ps"], C_MOL, RC)
    e = outs[-1]["energy"].cpu().numpy()[:-1].reshape(-1, 3)
    assert np.all(np.abs(e[:, 0] + e[:, 1] - r["Ek"] - r["E0"]) <= 1e-5 * np.abs(r["Ek"] + r["E0"]))
    F = outs[-1]["forces"].cpu().numpy().astype(np.float64)
    assert np.sqrt(np.mean((F - r["F"]) ** 2)) <= 1e-4 * np.sqrt(np.mean(r["F"] ** 2))
