"""Pins of the oracle in general (triclinic) cells, the cell tensor of the
Fig. 1 caption: the complete split E_real + E_k + E_0 - E_self of Eq. realLR
with the general-cell real-space image sum (oracle.realspace) and the
general-cell Fourier sum (oracle.cellsum) against values the mathematics
fixes:

* the rock-salt Madelung energy, with the crystal described by its
  face-centred primitive (triclinic) cell;
* independence of the total from the splitting (c, r_c) for p = 1..6 on a
  charged skewed cell;
* the real-space potentials, forces and virial invariant under a change of
  lattice basis (the same lattice described by other vectors), and equal
  to derivatives of the energy (finite differences in positions, in strain
  of the cell and positions, and in charges)."""
import os

import numpy as np
import pytest

from oracle import realspace
from paper_2606_06617_amd import workloads as wl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SKEW = np.array([[8.0, 0.0, 0.0], [2.5, 8.8, 0.0], [-1.5, 1.8, 7.2]])


def _madelung():
    with open(os.path.join(GOLDEN, "madelung_nacl.txt")) as f:
        return float([ln for ln in f if ln.strip() and not ln.startswith("#")][0])


def _skew_cell(seed, n=12, charged=True):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0, 1, (n, 3)) @ SKEW
    q = rng.normal(0, 1, n)
    if not charged:
        q -= q.mean()
    return pos, q


@pytest.mark.parametrize("ncell", [1, 2])
def test_rock_salt_madelung_on_the_primitive_cell(ncell):
    # ncell = 1: two ions in a cell whose widths (a / sqrt 3) are below r_c
    a = 5.64
    w = wl.nacl_primitive(ncell=ncell, a=a)
    pos = w["pos"].astype(np.float64)
    q = w["q"][0].astype(np.float64)
    ref = -0.5 * pos.shape[0] * _madelung() / (a / 2)
    E = realspace.total_energy(pos, q, w["box"], 1, 30.0, 5.0)
    assert E == pytest.approx(ref, rel=1e-10)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_splitting_independence_in_a_skewed_cell(p):
    pos, q = _skew_cell(20 + p)
    Es = [realspace.total_energy(pos, q, SKEW, p, c, rc) for c, rc in [(30.0, 2.5), (30.0, 3.0), (25.0, 3.5)]]
    assert np.ptp(Es) < 1e-8 * max(1.0, abs(Es[0])), Es


def test_real_space_change_of_lattice_basis():
    pos, q = _skew_cell(31)
    qq = np.stack([q, q - q.mean()])
    U = np.array([[1, 0, 0], [1, 1, 0], [0, -1, 1]], dtype=np.float64)   # unimodular
    r1 = realspace.evaluate(pos, qq, SKEW, [1, 6], 12.024, 4.0)
    r2 = realspace.evaluate(pos, qq, U @ SKEW, [1, 6], 12.024, 4.0)
    for key in ("Ereal", "phi", "F", "W"):
        assert np.allclose(r1[key], r2[key], rtol=1e-12, atol=1e-12 * np.abs(r1[key]).max()), key


def test_real_space_derivatives_in_a_skewed_cell():
    pos, q = _skew_cell(32)
    p, c, rc = 3, 12.024, 4.0
    r = realspace.evaluate(pos, q[None, :], SKEW, [p], c, rc)
    h = 1e-5
    for i in (0, 5, 11):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = -(realspace.real_energy(pp, q, SKEW, p, c, rc) - realspace.real_energy(pm, q, SKEW, p, c, rc)) / (2 * h)
            assert r["F"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-8 * np.abs(r["F"]).max())
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            ep = realspace.real_energy(pos @ (np.eye(3) + e).T, q, SKEW @ (np.eye(3) + e).T, p, c, rc)
            em = realspace.real_energy(pos @ (np.eye(3) - e).T, q, SKEW @ (np.eye(3) - e).T, p, c, rc)
            fd = -(ep - em) / (2 * h)
            assert r["W"][a, b] == pytest.approx(fd, rel=1e-6, abs=1e-8 * np.abs(r["W"]).max())
    for i in (1, 7):
        qp, qm = q.copy(), q.copy()
        qp[i] += h
        qm[i] -= h
        fd = (realspace.real_energy(pos, qp, SKEW, p, c, rc) - realspace.real_energy(pos, qm, SKEW, p, c, rc)) / (2 * h)
        assert r["phi"][0, i] == pytest.approx(fd, rel=1e-6, abs=1e-9)
