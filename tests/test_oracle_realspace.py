"""Pins of the oracle's real-space complement (oracle.realspace.evaluate)
and of the mollifier derivative it uses: the third derivative of psi
against the differentiated prolate equation, dG_p/dr against finite
differences of G_p (Eqs. G1, G6, G), the energy against the independent
image loop real_energy, forces and virial against finite differences of the
energy, potentials against the quadratic form and finite differences in q."""
import numpy as np
import pytest

from oracle import kernels, realspace
from oracle.pswf import PSWF

C, RC = 12.024, 5.0


def test_third_derivative_satisfies_differentiated_prolate_equation():
    # (1 - x^2) psi''' = 4 x psi'' + 2 psi' - (chi - c^2 x^2) psi' + 2 c^2 x psi
    ps = PSWF(C)
    x = np.linspace(-0.9, 0.9, 13)
    lhs = (1 - x * x) * ps.d3(x)
    rhs = 4 * x * ps.d2(x) + 2 * ps.d1(x) - (ps.chi - C * C * x * x) * ps.d1(x) + 2 * C * C * x * ps(x)
    assert np.allclose(lhs, rhs, rtol=1e-9, atol=1e-9 * np.abs(rhs).max())


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_mollifier_derivative_against_finite_differences(p):
    r = np.linspace(0.3, 4.7, 23)
    h = 1e-5
    fd = (kernels.mollifier(p, r + h, C, RC) - kernels.mollifier(p, r - h, C, RC)) / (2 * h)
    an = kernels.mollifier_deriv(p, r, C, RC)
    assert np.allclose(an, fd, rtol=1e-6, atol=1e-9)


def _system(seed=3, n=40, L=(9.0, 10.0, 8.5), ps=(1, 3, 6)):
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, 1.0, (n, 3)) * np.array(L)
    q = rng.normal(0.0, 0.5, (len(ps), n))
    return pos, q, np.array(L), list(ps)


def test_energy_equals_independent_image_loop():
    pos, q, box, ps = _system()
    r = realspace.evaluate(pos, q, box, ps, C, RC)
    for ch, p in enumerate(ps):
        assert r["Ereal"][ch] == pytest.approx(realspace.real_energy(pos, q[ch], box, p, C, RC), rel=1e-12)


def test_forces_are_minus_energy_gradient():
    pos, q, box, ps = _system(n=24)
    r = realspace.evaluate(pos, q, box, ps, C, RC)
    h = 1e-6
    for i in (0, 7, 19):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            ep = realspace.evaluate(pp, q, box, ps, C, RC)["Ereal"].sum()
            em = realspace.evaluate(pm, q, box, ps, C, RC)["Ereal"].sum()
            assert r["F"][i, a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-5, abs=1e-7)


def test_virial_is_minus_strain_derivative():
    pos, q, box, ps = _system(n=24)
    r = realspace.evaluate(pos, q, box, ps, C, RC)
    h = 1e-6
    for a in range(3):
        for b in range(3):
            eps = np.zeros((3, 3))
            eps[a, b] = h
            def energy(e):
                # affine strain of positions; the box is orthorhombic, so only
                # diagonal strains scale it (off-diagonal: images shear, the
                # pair geometry is that of the sheared positions)
                m = np.eye(3) + e
                E = 0.0
                for ch, p in enumerate(ps):
                    E += _sheared_energy(pos @ m.T, q[ch], box, m, p)
                return E
            fd = -(energy(eps) - energy(-eps)) / (2 * h)
            assert r["W"][a, b] == pytest.approx(fd, rel=1e-5, abs=1e-7)


def _sheared_energy(pos, q, box, m, p):
    """1/2 sum q_i q_j K(|r_j - r_i + m n L|) over the sheared lattice."""
    n = pos.shape[0]
    H = m @ np.diag(box)            # columns: the deformed lattice vectors
    E = 0.0
    rng = range(-2, 3)
    for ix in rng:
        for iy in rng:
            for iz in rng:
                sh = H @ np.array([ix, iy, iz], dtype=np.float64)
                d = pos[None, :, :] - pos[:, None, :] + sh
                r = np.sqrt(np.sum(d * d, axis=2))
                mask = (r < RC) & (r > 0.0)
                rr = r[mask]
                qq = (q[:, None] * q[None, :])[mask]
                E += 0.5 * np.sum(qq * (1.0 - kernels.mollifier(p, rr, C, RC)) / rr ** p)
    return E


def test_potentials_quadratic_form_and_charge_derivative():
    pos, q, box, ps = _system(n=30)
    r = realspace.evaluate(pos, q, box, ps, C, RC)
    for ch in range(len(ps)):
        assert 0.5 * np.sum(q[ch] * r["phi"][ch]) == pytest.approx(r["Ereal"][ch], rel=1e-12)
    h = 1e-6
    for ch, i in ((0, 3), (1, 11), (2, 29)):
        qp, qm = q.copy(), q.copy()
        qp[ch, i] += h
        qm[ch, i] -= h
        fd = (realspace.evaluate(pos, qp, box, ps, C, RC)["Ereal"][ch]
              - realspace.evaluate(pos, qm, box, ps, C, RC)["Ereal"][ch]) / (2 * h)
        assert r["phi"][ch, i] == pytest.approx(fd, rel=1e-6, abs=1e-9)
