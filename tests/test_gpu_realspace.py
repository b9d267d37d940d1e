"""The real-space complement on the GPU (pswflr_realspace, Eq. realLR with
the mollifier of Eqs. G1, G6, G) against the FP64 oracle, and the complete
split E_real + E_k + E_0 - E_self against values fixed by the mathematics:

* parity with oracle.realspace.evaluate (energy per channel, forces,
  potentials, virial) on a charged anisotropic box with p = 1, 3, 6, and
  on a box shorter than r_c (several periodic images of every atom);
* the rock-salt Madelung energy (tests/golden/madelung_nacl.txt) from the
  GPU's real-space and reciprocal parts at c = 30;
* splitting independence: the total for p = 1..6 on a charged box is the
  same at two cutoffs r_c.

FP32 on the GPU bounds the totals at ~1e-6 relative (each term carries
~1e-7 relative rounding and E_real, E_k are of the total's size), so the
totals are checked at 2e-6, the pair sums against the oracle at 1e-5."""
import os

import numpy as np
import pytest
import torch

from oracle import realspace

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _rel_rms(a, b):
    return float(np.sqrt(np.mean((a - b) ** 2)) / np.sqrt(np.mean(b ** 2)))


def _plan(box, ps, c, rc, n, grid=None, support=0):
    from paper_2606_06617_amd.api import Plan
    return Plan(box, ps, r_c=rc, c=c, tol=1e-5, grid=grid, support=support, max_atoms=max(1, n))


def _real(plan, pos, q):
    out = plan.realspace(torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda(), forces=True, virial=True,
                         potential=True)
    torch.cuda.synchronize()
    Wv = out["virial"].cpu().numpy()
    return {"E": out["energy"].cpu().numpy(), "F": out["forces"].cpu().numpy().astype(np.float64),
            "phi": out["potential"].cpu().numpy().astype(np.float64),
            "W": np.array([[Wv[0], Wv[3], Wv[4]], [Wv[3], Wv[1], Wv[5]], [Wv[4], Wv[5], Wv[2]]])}


def _compare(g, r, tol=1e-5):
    assert np.allclose(g["E"], r["Ereal"], rtol=tol, atol=0.0), (g["E"], r["Ereal"])
    assert _rel_rms(g["F"], r["F"]) <= tol
    assert _rel_rms(g["phi"], r["phi"]) <= tol
    assert np.abs(g["W"] - r["W"]).max() <= tol * np.abs(r["W"]).max()


def test_realspace_vs_oracle_charged_box():
    rng = np.random.default_rng(71)
    box = np.array([18.0, 21.0, 16.5])
    N = 700
    pos = (rng.uniform(0.0, 1.0, (N, 3)) * box).astype(np.float32)
    q = rng.normal(0.0, 0.5, (3, N)).astype(np.float32)
    print("case real space: N", N, "box", box, flush=True)
    plan = _plan(box, (1, 3, 6), 12.024, 5.0, N, grid=(24, 30, 24), support=6)
    g = _real(plan, pos, q)
    r = realspace.evaluate(pos.astype(np.float64), q.astype(np.float64), box, (1, 3, 6), 12.024, 5.0)
    _compare(g, r)
    # a second call on the same workspace gives the same bits
    assert np.array_equal(_real(plan, pos, q)["F"], g["F"])


def test_realspace_box_shorter_than_cutoff():
    rng = np.random.default_rng(72)
    box = np.array([4.5, 6.0, 5.5])
    N = 24
    pos = (rng.uniform(-1.0, 2.0, (N, 3)) * box).astype(np.float32)   # also outside the cell
    q = rng.normal(0.0, 0.5, (2, N)).astype(np.float32)
    print("case real space: box shorter than r_c", box, flush=True)
    plan = _plan(box, (1, 6), 12.024, 5.0, N, grid=(8, 10, 8), support=4)
    g = _real(plan, pos, q)
    r = realspace.evaluate(pos.astype(np.float64), q.astype(np.float64), box, (1, 6), 12.024, 5.0)
    _compare(g, r)


def _parts(plan, pos, q):
    """Per channel E_real, E_k + E_0 and E_self from the GPU."""
    tp, tq = torch.from_numpy(pos).cuda(), torch.from_numpy(q).cuda()
    e = plan.execute(tp, tq, forces=False, virial=False)["energy"]
    er = plan.realspace(tp, tq, forces=False, virial=False)["energy"]
    torch.cuda.synchronize()
    ek = e.cpu().numpy()[:-1].reshape(-1, 3)
    return er.cpu().numpy(), ek[:, 0] + ek[:, 1], ek[:, 2]


def _total(plan, pos, q):
    er, elr, es = _parts(plan, pos, q)
    return er + elr - es


def test_rock_salt_madelung_from_gpu_split():
    from paper_2606_06617_amd import workloads as wl
    lines = [ln for ln in open(os.path.join(ROOT, "tests", "golden", "madelung_nacl.txt"))
             if ln.strip() and not ln.startswith("#")]
    madelung = float(lines[0].split()[0])
    a = 5.64
    w = wl.nacl(jitter=0.0, a=a)
    N = w["pos"].shape[0]
    e_ref = -(N / 2) * madelung / (a / 2)          # -M e^2 / r0 per ion pair
    print("case Madelung: rock salt", N, "atoms, c = 30", flush=True)
    plan = _plan(w["box"], [1], 30.0, 5.0, N)
    tot = _total(plan, w["pos"], w["q"])[0]
    print("   total %.10f reference %.10f rel %.2e" % (tot, e_ref, abs(tot - e_ref) / abs(e_ref)), flush=True)
    assert abs(tot - e_ref) <= 2e-6 * abs(e_ref), (tot, e_ref)


def test_splitting_independence_all_exponents():
    rng = np.random.default_rng(73)
    box = np.array([12.0, 12.0, 12.0])
    N = 60
    pos = (rng.uniform(0.0, 1.0, (N, 3)) * box).astype(np.float32)
    q = rng.normal(0.0, 0.5, (6, N)).astype(np.float32)          # charged: exercises E_0
    ps = [1, 2, 3, 4, 5, 6]
    print("case splitting independence p = 1..6", flush=True)
    # the reciprocal part of a plan at tol = 1e-5 is accurate to about
    # 1e-5 of its own size, and the total is a difference of parts larger
    # than itself (the self term of p = 5 at these cutoffs is many times
    # the total): the bar is 1e-5 of the largest part
    p1 = _parts(_plan(box, ps, 30.0, 2.5, N), pos, q)
    p2 = _parts(_plan(box, ps, 30.0, 3.0, N), pos, q)
    t1, t2 = p1[0] + p1[1] - p1[2], p2[0] + p2[1] - p2[2]
    scale = np.max(np.abs(np.stack(p1 + p2)), axis=0)
    print("   totals r_c 2.5:", np.array2string(t1, precision=9), flush=True)
    print("   totals r_c 3.0:", np.array2string(t2, precision=9), flush=True)
    print("   |diff| / largest part:", np.array2string(np.abs(t1 - t2) / scale, precision=2), flush=True)
    assert np.all(np.abs(t1 - t2) <= 1e-5 * scale), (t1, t2, scale)
