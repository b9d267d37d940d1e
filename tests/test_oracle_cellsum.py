"""Pins for oracle.cellsum, the general-cell Fourier sum with separable
phase tables: against the plain direct sum (orthorhombic), a change of
lattice basis, finite differences of its own energy for forces and for the
whole virial tensor (off-diagonal entries included), and the off-diagonal
virial of oracle.reciprocal against the energy of a sheared cell."""
import numpy as np
import pytest

from oracle import cellsum, reciprocal

C_MOL = 12.024


def _cell_atoms(seed, n, H, charged):
    rng = np.random.Generator(np.random.PCG64(seed))
    frac = rng.uniform(0.0, 1.0, size=(n, 3))
    pos = frac @ H
    q = rng.normal(0.0, 0.5, size=(2, n))
    if not charged:
        q -= q.mean(axis=1, keepdims=True)
    return pos, q


TRICLINIC = np.array([[9.0, 0.0, 0.0], [2.1, 8.4, 0.0], [-1.3, 1.7, 9.6]])


@pytest.mark.parametrize("charged", [False, True])
def test_orthorhombic_equals_direct_sum(charged):
    box = np.array([9.0, 10.5, 8.2])
    pos, q = _cell_atoms(1, 14, np.diag(box), charged)
    ps = [1, 6]
    r = reciprocal.evaluate(pos, q, box, ps, C_MOL, 3.0)
    g = cellsum.evaluate(pos, q, np.diag(box), ps, C_MOL, 3.0)
    for key in ("Ek", "E0", "Eself"):
        assert np.allclose(g[key], r[key], rtol=1e-11, atol=1e-14), key
    assert np.allclose(g["phi"], r["phi"], rtol=1e-10, atol=1e-12 * np.abs(r["phi"]).max())
    assert np.allclose(g["F"], r["F"], rtol=1e-10, atol=1e-12 * np.abs(r["F"]).max())
    assert np.allclose(g["W"], r["W"], rtol=1e-10, atol=1e-12 * np.abs(r["W"]).max())


def test_sampled_atoms_match_all_atoms():
    pos, q = _cell_atoms(2, 20, TRICLINIC, True)
    full = cellsum.evaluate(pos, q, TRICLINIC, [1, 3], C_MOL, 3.0)
    idx = np.array([3, 0, 17])
    part = cellsum.evaluate(pos, q, TRICLINIC, [1, 3], C_MOL, 3.0, sample=idx)
    assert np.array_equal(part["Ek"], full["Ek"])
    assert np.allclose(part["F"], full["F"][idx], rtol=1e-13, atol=1e-15)
    assert np.allclose(part["phi"], full["phi"][:, idx], rtol=1e-13, atol=1e-15)


def test_change_of_lattice_basis():
    # the same lattice described by other basis vectors (integer matrix of
    # determinant 1): every output is the same
    pos, q = _cell_atoms(3, 12, TRICLINIC, True)
    U = np.array([[1, 0, 0], [1, 1, 0], [0, -1, 1]], dtype=np.float64)
    a = cellsum.evaluate(pos, q, TRICLINIC, [1, 6], C_MOL, 3.0)
    b = cellsum.evaluate(pos, q, U @ TRICLINIC, [1, 6], C_MOL, 3.0)
    assert np.allclose(b["Ek"], a["Ek"], rtol=1e-11)
    assert np.allclose(b["F"], a["F"], rtol=1e-9, atol=1e-11 * np.abs(a["F"]).max())
    assert np.allclose(b["phi"], a["phi"], rtol=1e-9, atol=1e-11 * np.abs(a["phi"]).max())
    assert np.allclose(b["W"], a["W"], rtol=1e-9, atol=1e-11 * np.abs(a["W"]).max())


def _etot(pos, q, H, ps, rc=3.0):
    r = cellsum.evaluate(pos, q, H, ps, C_MOL, rc, sample=np.zeros(0, np.int64), virial=False)
    return float(np.sum(r["Ek"] + r["E0"]))


@pytest.mark.parametrize("ps", [(1, 6), (3, 5)])
def test_triclinic_forces_are_minus_gradient(ps):
    pos, q = _cell_atoms(4, 10, TRICLINIC, True)
    res = cellsum.evaluate(pos, q, TRICLINIC, ps, C_MOL, 3.0)
    h = 1e-5
    for i in (0, 6):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = -(_etot(pp, q, TRICLINIC, ps) - _etot(pm, q, TRICLINIC, ps)) / (2 * h)
            assert res["F"][i, a] == pytest.approx(fd, rel=1e-6, abs=1e-9 * np.abs(res["F"]).max())


@pytest.mark.parametrize("ps", [(1, 6), (2, 4)])
def test_triclinic_virial_is_minus_strain_derivative(ps):
    # W_ab = -dE/d eps_ab under r -> r (I + eps), H -> H (I + eps), for every
    # (a, b): the off-diagonal entries are pinned here, not by symmetry
    pos, q = _cell_atoms(5, 10, TRICLINIC, True)
    res = cellsum.evaluate(pos, q, TRICLINIC, ps, C_MOL, 3.0)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            e = np.zeros((3, 3))
            e[a, b] = h
            Fp, Fm = np.eye(3) + e, np.eye(3) - e
            fd = -(_etot(pos @ Fp, q, TRICLINIC @ Fp, ps) - _etot(pos @ Fm, q, TRICLINIC @ Fm, ps)) / (2 * h)
            assert res["W"][a, b] == pytest.approx(fd, rel=1e-6, abs=1e-8 * np.abs(res["W"]).max()), (a, b)


@pytest.mark.parametrize("p", [1, 3, 6])
def test_orthorhombic_off_diagonal_virial_against_sheared_cell(p):
    # oracle.reciprocal's off-diagonal virial against the energy of the
    # sheared (triclinic) cell
    box = np.array([9.0, 8.0, 10.0])
    pos, q = _cell_atoms(6, 10, np.diag(box), p >= 3)
    r = reciprocal.evaluate(pos, q[:1], box, [p], C_MOL, 3.0)
    h = 1e-6
    for a, b in ((0, 1), (0, 2), (1, 2), (2, 0)):
        e = np.zeros((3, 3))
        e[a, b] = h
        Fp, Fm = np.eye(3) + e, np.eye(3) - e
        H = np.diag(box)
        fd = -(_etot(pos @ Fp, q[:1], H @ Fp, [p]) - _etot(pos @ Fm, q[:1], H @ Fm, [p])) / (2 * h)
        assert r["W"][a, b] == pytest.approx(fd, rel=1e-6, abs=1e-8 * np.abs(r["W"]).max()), (a, b)


def _vjp_system():
    rng = np.random.default_rng(19)
    H = np.array([[9.0, 0.0, 0.0], [2.2, 9.5, 0.0], [-1.4, 1.9, 8.1]])
    n = 18
    pos = rng.uniform(0.0, 1.0, (n, 3)) @ H
    q = rng.normal(0.0, 0.5, (2, n))
    v = rng.normal(0.0, 1.0, (n, 3))
    return pos, q, H, (1, 6), v


def _vjp_loss(pos, q, H, ps, v):
    F = cellsum.evaluate(pos, q, H, ps, C_MOL, 5.0, virial=False)["F"]
    return float(np.sum(v * F))


def test_force_vjp_against_finite_differences_of_forces():
    # the double backward in a triclinic cell: derivatives of L = sum v . F
    # against central differences of L formed from the oracle's own forces
    pos, q, H, ps, v = _vjp_system()
    dq, dr = cellsum.force_vjp(pos, q, H, ps, C_MOL, 5.0, v)
    h = 1e-6
    for ch, j in ((0, 2), (1, 9), (0, 17)):
        qp, qm = q.copy(), q.copy()
        qp[ch, j] += h
        qm[ch, j] -= h
        fd = (_vjp_loss(pos, qp, H, ps, v) - _vjp_loss(pos, qm, H, ps, v)) / (2 * h)
        assert dq[ch, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    for j in (0, 11):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[j, a] += h
            pm[j, a] -= h
            fd = (_vjp_loss(pp, q, H, ps, v) - _vjp_loss(pm, q, H, ps, v)) / (2 * h)
            assert dr[j, a] == pytest.approx(fd, rel=1e-5, abs=1e-8)
