"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded FP32 inputs.

Bars (FP32 on the GPU, FP64 oracle):
  * against the direct structure-factor sum (the plain definition):
    relative energy <= 1e-5, relative RMS force <= 1e-4, virial <= 1e-4
    (max-abs relative to max |W|), potentials RMS <= 1e-4;
  * against the oracle's mesh algorithm at the same (grid, P, c_s), which
    isolates FP32 rounding from the method's own approximation:
    energy <= 2e-6, forces <= 2e-5, potentials <= 2e-5.
"""
import numpy as np
import pytest
import torch

from oracle import mesh, reciprocal
from paper_2606_06617_amd import workloads as wl

pytestmark = pytest.mark.gpu

C_MOL, RC = 12.024, 5.0
# window bandwidth given to both sides of the mesh comparisons (about 2.6 P,
# the usual choice for a PSWF window of P points); the GPU-vs-mesh bars do
# not depend on it being the planner's optimum
CS_OF_P = {2: 5.2, 3: 7.8, 4: 10.4, 5: 13.0, 6: 15.6, 7: 18.2, 8: 20.8}


def _gpu(w, grid, P, cs=0.0, potential=True, c=C_MOL, rc=RC):
    from paper_2606_06617_amd.api import Plan
    print("case", w["name"], "grid", grid, "P", P, flush=True)
    pos = torch.from_numpy(w["pos"]).cuda()
    q = torch.from_numpy(w["q"]).cuda()
    plan = Plan(w["box"], w["ps"], r_c=rc, c=c, grid=grid, support=P, c_spread=cs,
                max_atoms=max(1, pos.shape[0]))
    out = plan.execute(pos, q, forces=True, virial=True, potential=potential)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if torch.is_tensor(v) else v) for k, v in out.items() if k != "workspace"}
    e = res["energy"][:-1].reshape(-1, 3)
    W = res["virial"]
    return {
        "Ek": e[:, 0], "E0": e[:, 1], "Eself": e[:, 2], "Elr": float(res["energy"][-1]),
        "F": res["forces"].astype(np.float64),
        "W": np.array([[W[0], W[3], W[4]], [W[3], W[1], W[5]], [W[4], W[5], W[2]]]),
        "phi": res["potential"].astype(np.float64) if potential else None, "plan": plan,
    }


def _rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


def _compare(g, r, eE, eF, eW, eP):
    Eg = g["Ek"] + g["E0"]
    Er = r["Ek"] + r["E0"]
    rel_e = np.abs(Eg - Er) / np.maximum(np.abs(Er), 1e-300)
    assert np.all(rel_e <= eE), (rel_e, Eg, Er)
    # E_lr, summed on the device in channel order
    assert abs(g["Elr"] - Eg.sum()) <= 1e-12 * np.abs(Eg).sum()
    assert np.allclose(g["E0"], r["E0"], rtol=1e-9, atol=1e-12)
    assert np.allclose(g["Eself"], r["Eself"], rtol=1e-9)
    ef = _rel_rms(g["F"], r["F"])
    assert ef <= eF, ef
    ew = np.abs(g["W"] - r["W"]).max() / np.abs(r["W"]).max()
    assert ew <= eW, ew
    if g["phi"] is not None:
        ep = _rel_rms(g["phi"], r["phi"])
        assert ep <= eP, ep
    return rel_e, ef, ew


def _direct(w):
    return reciprocal.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), w["box"],
                               w["ps"], C_MOL, RC)


def test_rock_salt_512_vs_direct_sum():
    w = wl.nacl()
    g = _gpu(w, (32, 32, 32), 6)
    _compare(g, _direct(w), 1e-5, 1e-4, 1e-4, 1e-4)


def test_water_3000_two_channels_vs_direct_sum():
    w = wl.water()
    g = _gpu(w, (48, 48, 48), 8)
    _compare(g, _direct(w), 1e-5, 1e-4, 1e-4, 1e-4)


def test_random_box_vs_mesh_algorithm():
    # same grid, P and c_s as the oracle's mesh: only FP32 rounding differs
    w = wl.random_box(700, ps=(1, 6), seed=21, aspect=(1.0, 1.2, 0.9))
    grid = (24, 30, 20)
    cs = CS_OF_P[8]
    g = _gpu(w, grid, 8, cs=cs)
    assert g["plan"].info["c_spread"] == cs
    r = mesh.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), w["box"], w["ps"],
                      C_MOL, RC, grid, 8, cs)
    _compare(g, r, 2e-6, 2e-5, 2e-5, 2e-5)


@pytest.mark.parametrize("P", [2, 3, 4, 5, 6, 7, 8])
def test_every_support_vs_mesh_algorithm(P):
    w = wl.random_box(300, ps=(1,), seed=30 + P)
    grid = (20, 24, 18)
    cs = CS_OF_P[P]
    g = _gpu(w, grid, P, cs=cs)
    assert g["plan"].info["c_spread"] == cs
    r = mesh.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), w["box"], w["ps"],
                      C_MOL, RC, grid, P, cs)
    _compare(g, r, 2e-6, 2e-5, 2e-5, 2e-5)


def test_all_exponents_charged_ragged_grid():
    # six channels p = 1..6, non-neutral, anisotropic cell, grid edges with
    # factors 2, 3 and 5 that leave ragged tiles and transform lengths
    w = wl.random_box(900, ps=(1, 2, 3, 4, 5, 6), seed=22, aspect=(1.0, 1.3, 0.8), neutral=False)
    grid = (30, 40, 36)
    g = _gpu(w, grid, 8)
    _compare(g, _direct(w), 1e-5, 1e-4, 1e-4, 1e-4)


def test_empty_and_single_atom():
    w = wl.random_box(1, ps=(1, 6), seed=23, neutral=False, density=1e-3)
    g = _gpu(w, (16, 16, 16), 6)
    r = _direct(w)
    # a single charge: E_k is its self-image interaction in k-space
    assert np.allclose(g["Ek"] + g["E0"], r["Ek"] + r["E0"], rtol=1e-5)
    empty = dict(w)
    empty["pos"] = np.zeros((0, 3), np.float32)
    empty["q"] = np.zeros((2, 0), np.float32)
    from paper_2606_06617_amd.api import Plan
    plan = Plan(w["box"], w["ps"], r_c=RC, c=C_MOL, grid=(16, 16, 16), support=6, max_atoms=4)
    out = plan.execute(torch.zeros((0, 3), device="cuda"), torch.zeros((2, 0), device="cuda"))
    torch.cuda.synchronize()
    assert np.all(out["energy"].cpu().numpy() == 0.0)


def test_bitwise_reproducible():
    from paper_2606_06617_amd.api import Plan
    w = wl.water(nmol=400, L=22.0)
    pos = torch.from_numpy(w["pos"]).cuda()
    q = torch.from_numpy(w["q"]).cuda()
    plan = Plan(w["box"], w["ps"], r_c=RC, c=C_MOL, grid=(36, 36, 36), support=8, max_atoms=pos.shape[0])
    a = plan.execute(pos, q, potential=True)
    b = plan.execute(pos, q, potential=True)
    torch.cuda.synchronize()
    for k in ("energy", "forces", "virial", "potential"):
        assert torch.equal(a[k], b[k]), k


def test_grid_translation_invariance():
    # shifting every atom by a whole number of grid spacings permutes the
    # grid: energies agree to rounding, forces are unchanged
    from paper_2606_06617_amd.api import Plan
    w = wl.random_box(500, ps=(1,), seed=24)
    grid = (24, 24, 24)
    plan = Plan(w["box"], w["ps"], r_c=RC, c=C_MOL, grid=grid, support=8, max_atoms=500)
    h = w["box"] / np.array(grid)
    p0 = w["pos"].astype(np.float64)
    p1 = np.mod(p0 + 5 * h, w["box"]).astype(np.float32)
    a = plan.execute(torch.from_numpy(w["pos"]).cuda(), torch.from_numpy(w["q"]).cuda())
    b = plan.execute(torch.from_numpy(p1).cuda(), torch.from_numpy(w["q"]).cuda())
    torch.cuda.synchronize()
    ea, eb = a["energy"].cpu().numpy(), b["energy"].cpu().numpy()
    assert abs(ea[0] - eb[0]) <= 1e-5 * abs(ea[0])
    assert _rel_rms(b["forces"].cpu().numpy(), a["forces"].cpu().numpy()) < 1e-4


def test_crowded_tiles_vs_mesh_and_direct_sum():
    # 1200 atoms packed into a 4 A cube that straddles the periodic corner of
    # an 18 A box: a few tiles hold hundreds of atoms each, so the spread
    # flushes its candidate list many times per tile and the gather takes
    # several passes of atoms over the same tile (with idle waves in the
    # last one); the wrap across three faces exercises periodic indexing
    rng = np.random.default_rng(404)
    N, L = 1200, 18.0
    pos = (rng.uniform(-2.0, 2.0, (N, 3)) + np.array([0.3, 17.9, 0.1])) % L
    q = rng.normal(0.0, 1.0, (2, N))
    q -= q.mean(axis=1, keepdims=True)
    w = {"name": "crowded", "pos": pos.astype(np.float32), "q": q.astype(np.float32),
         "box": (L, L, L), "ps": (1, 6)}
    grid = (36, 36, 36)
    cs = CS_OF_P[8]
    g = _gpu(w, grid, 8, cs=cs)
    B = np.array(g["plan"].info["tile"])
    x = w["pos"].astype(np.float64) / L * np.array(grid)
    start = np.ceil(x - 4.0).astype(np.int64) % np.array(grid)
    cell = start // B
    nc = -(-np.array(grid) // B)
    cnt = np.bincount((cell[:, 0] * nc[1] + cell[:, 1]) * nc[2] + cell[:, 2])
    assert cnt.max() > 256, (B, cnt.max())
    r = mesh.evaluate(w["pos"].astype(np.float64), w["q"].astype(np.float64), w["box"], w["ps"],
                      C_MOL, RC, grid, 8, cs)
    _compare(g, r, 2e-6, 2e-5, 2e-5, 2e-5)
    _compare(g, _direct(w), 1e-5, 1e-4, 1e-4, 1e-4)
