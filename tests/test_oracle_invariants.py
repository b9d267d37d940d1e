"""Physics pins for the oracle's energy, forces, potentials and virial.

Each pin uses something other than the oracle's own formulas: a closed-form
lattice constant (rock-salt Madelung), independent summation methods
(textbook Ewald, brute-force image sums), invariance of the total energy
under the arbitrary splitting parameters (c, r_c), and finite differences."""
import os

import numpy as np
import pytest

from oracle import brute, ewald, kernels, realspace, reciprocal
from paper_2606_06617_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _madelung():
    with open(os.path.join(GOLDEN, "madelung_nacl.txt")) as f:
        return float([ln for ln in f if ln.strip() and not ln.startswith("#")][0])


def _small_cell(seed, n=16, charged=True, aspect=(1.0, 1.1, 0.9), L=8.0):
    rng = np.random.default_rng(seed)
    box = np.array(aspect) * L
    pos = rng.uniform(0, 1, (n, 3)) * box
    q = rng.normal(0, 1, n)
    if not charged:
        q -= q.mean()
    return pos, q, box


def test_rock_salt_madelung_energy():
    w = wl.nacl(jitter=0.0)
    pos = w["pos"].astype(np.float64)
    q = w["q"][0].astype(np.float64)
    a = 5.64
    ref = -0.5 * pos.shape[0] * _madelung() / (a / 2)
    E = realspace.total_energy(pos, q, w["box"], 1, 30.0, 5.0)
    assert E == pytest.approx(ref, rel=1e-11)
    # at the paper's working bandwidth the band-limited reading leaves an
    # O(psi(1)) = 7e-5 discrepancy in the total (not in the k-space part)
    E12 = realspace.total_energy(pos, q, w["box"], 1, 12.024, 5.0)
    assert E12 == pytest.approx(ref, rel=1e-4)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("charged", [False, True])
def test_splitting_independence(p, charged):
    pos, q, box = _small_cell(10 + p, charged=charged)
    Es = [realspace.total_energy(pos, q, box, p, c, rc)
          for c, rc in [(30.0, 2.5), (30.0, 3.0), (25.0, 3.5)]]
    assert np.ptp(Es) < 1e-8 * max(1.0, abs(Es[0])), Es


@pytest.mark.parametrize("p,rtol", [(4, 2e-4), (5, 1e-5), (6, 1e-7)])
def test_brute_force_image_sums(p, rtol):
    rng = np.random.default_rng(1)
    L = 6.0
    box = np.array([L, L, L])
    pos = rng.uniform(0, 1, (8, 3)) * box
    q = rng.normal(0, 1, 8)
    Eb = brute.image_sum(pos, q, box, p, 25 * L)
    Ep = realspace.total_energy(pos, q, box, p, 30.0, 2.9)
    assert Ep == pytest.approx(Eb, rel=rtol)


def test_textbook_ewald_p1():
    pos, q, box = _small_cell(3, n=12, charged=False, L=7.0)
    Ee = ewald.ewald_energy(pos, q, box, alpha=1.2, r_cut=6.5, k_cut=13.0)
    Ep = realspace.total_energy(pos, q, box, 1, 30.0, 3.0)
    assert Ep == pytest.approx(Ee, rel=1e-9)


def _ek(pos, q, box, p, c=12.024, rc=5.0):
    return reciprocal.reciprocal_channel(pos, q, box, p, c, rc, forces=False,
                                         potential=False, virial=False)["E"]


@pytest.mark.parametrize("p", [1, 3, 6])
def test_forces_are_minus_gradient(p):
    pos, q, box = _small_cell(4, n=10, charged=(p == 6), L=9.0)
    r = reciprocal.reciprocal_channel(pos, q, box, p, 12.024, 3.0)
    h = 1e-5
    for i in (0, 3, 7):
        for a in range(3):
            pp = pos.copy()
            pm = pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = -(_ek(pp, q, box, p, rc=3.0) - _ek(pm, q, box, p, rc=3.0)) / (2 * h)
            assert r["F"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(r["F"]).max())


@pytest.mark.parametrize("p", [1, 2, 3, 6])
def test_potential_is_charge_derivative(p):
    pos, q, box = _small_cell(5, n=10, charged=True, L=9.0)
    res = reciprocal.evaluate(pos, q[None, :], box, [p], 12.024, 3.0)
    h = 1e-6

    def etot(qq):
        r = reciprocal.evaluate(pos, qq[None, :], box, [p], 12.024, 3.0,
                                forces=False, potential=False, virial=False)
        return r["Ek"][0] + r["E0"][0]
    for i in (0, 4, 9):
        qp = q.copy()
        qm = q.copy()
        qp[i] += h
        qm[i] -= h
        fd = (etot(qp) - etot(qm)) / (2 * h)
        assert res["phi"][0, i] == pytest.approx(fd, rel=1e-6, abs=1e-9)


@pytest.mark.parametrize("p", [1, 3, 5, 6])
def test_virial_is_minus_strain_derivative(p):
    pos, q, box = _small_cell(6, n=10, charged=(p >= 3), L=9.0)
    c, rc = 12.024, 3.0
    res = reciprocal.evaluate(pos, q[None, :], box, [p], c, rc)
    h = 1e-6

    def etot(eps):
        # affine strain x -> (1 + eps) x of an orthorhombic cell (diagonal eps)
        s = 1.0 + eps
        r = reciprocal.evaluate(pos * s, q[None, :], box * s, [p], c, rc,
                                forces=False, potential=False, virial=False)
        return r["Ek"][0] + r["E0"][0]
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = -(etot(e) - etot(-e)) / (2 * h)
        assert res["W"][a, a] == pytest.approx(fd, rel=1e-6)
    # off-diagonal: W_ab = sum_i r_ia F_ib is not the k-space form, but a
    # shear of the sample keeps E_k invariant when the reciprocal lattice is
    # sheared along; checked by symmetry instead
    assert np.allclose(res["W"], res["W"].T, atol=1e-12 * np.abs(res["W"]).max())


def test_invariances():
    pos, q, box = _small_cell(7, n=12, charged=False, L=9.0)
    c, rc = 12.024, 3.0
    r0 = reciprocal.evaluate(pos, q[None, :], box, [1], c, rc)
    # zero net force (Newton's third law holds in k-space)
    assert np.abs(r0["F"].sum(0)).max() < 1e-12 * np.abs(r0["F"]).max()
    # translation invariance of energy and forces
    sh = np.array([0.37, -1.21, 2.5])
    r1 = reciprocal.evaluate(pos + sh, q[None, :], box, [1], c, rc)
    assert r1["Ek"][0] == pytest.approx(r0["Ek"][0], rel=1e-12)
    assert np.allclose(r1["F"], r0["F"], atol=1e-12 * np.abs(r0["F"]).max())
    # quadratic in the charges, potentials linear
    r2 = reciprocal.evaluate(pos, 2.5 * q[None, :], box, [1], c, rc)
    assert r2["Ek"][0] == pytest.approx(6.25 * r0["Ek"][0], rel=1e-12)
    assert np.allclose(r2["phi"], 2.5 * r0["phi"], rtol=1e-12, atol=1e-14)


def test_perfect_lattice_has_zero_force():
    w = wl.nacl(jitter=0.0)
    pos = w["pos"].astype(np.float64)
    r = reciprocal.evaluate(pos, w["q"].astype(np.float64), w["box"], [1], 12.024, 5.0)
    # positions are the FP32-rounded lattice (~1e-7 A off the ideal sites);
    # forces on the 0.1 A-jittered crystal are O(1) in the same units
    assert np.abs(r["F"]).max() < 1e-7
    rj = reciprocal.evaluate(wl.nacl()["pos"].astype(np.float64),
                             w["q"].astype(np.float64), w["box"], [1], 12.024, 5.0)
    assert np.sqrt(np.mean(rj["F"] ** 2)) > 1e-2
