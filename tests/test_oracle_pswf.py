"""Pins for oracle.pswf (the order-zero PSWF, Methods "Prolate spheroidal
wave functions").  Each check uses something other than the Legendre
representation itself: the defining integral eigen-relation by quadrature,
the prolate ODE at x = 0, and the large-c asymptote of lambda_0."""
import numpy as np
import pytest

from oracle.pswf import PSWF, ode_derivatives_at_zero

CS = [5.0, 12.024, 20.0, 30.0]


@pytest.mark.parametrize("c", CS)
def test_integral_eigen_relation(c):
    # lambda_0 psi(x) = int_{-1}^{1} psi(t) exp(i c x t) dt  (eq. psidefinit)
    ps = PSWF(c)
    t, w = np.polynomial.legendre.leggauss(300)
    xs = np.linspace(-1.0, 1.0, 41)
    rhs = np.array([np.sum(w * ps(t) * np.exp(1j * c * x * t)) for x in xs])
    assert np.max(np.abs(rhs.imag)) < 1e-13
    assert np.max(np.abs(ps.lam * ps(xs) - rhs.real)) < 1e-12


@pytest.mark.parametrize("c", CS)
def test_normalisation_and_parity(c):
    ps = PSWF(c)
    assert ps(0.0) == pytest.approx(1.0, abs=1e-15)
    x = np.linspace(0.0, 1.0, 17)
    assert np.allclose(ps(x), ps(-x), atol=1e-15)
    # C0 = int_0^1 psi by plain quadrature (not the Legendre antiderivative)
    t, w = np.polynomial.legendre.leggauss(200)
    c0 = np.sum(0.5 * w * ps(0.5 * (t + 1.0)))
    assert ps.C0 == pytest.approx(c0, rel=1e-13)
    assert ps.I0(1.0) == pytest.approx(c0, rel=1e-13)


@pytest.mark.parametrize("c", CS)
def test_derivatives_at_zero_match_prolate_ode(c):
    ps = PSWF(c)
    d = ode_derivatives_at_zero(ps.chi, c, 8)
    for n in (2, 4, 6, 8):
        assert ps.deriv_at_zero(n) == pytest.approx(d[n], rel=1e-9)


@pytest.mark.parametrize("c", CS)
def test_prolate_ode_residual(c):
    ps = PSWF(c)
    x = np.linspace(-0.95, 0.95, 39)
    res = -(1 - x * x) * ps.d2(x) + 2 * x * ps.d1(x) + c * c * x * x * ps(x) - ps.chi * ps(x)
    assert np.max(np.abs(res)) < 1e-9 * max(1.0, c * c)


def test_lambda_asymptote_and_band_concentration():
    # lambda_0 -> sqrt(2 pi / c) as c grows (psi_0 tends to a Gaussian-like bump)
    ps = PSWF(30.0)
    assert ps.lam == pytest.approx(np.sqrt(2 * np.pi / 30.0), rel=1e-12)
    # at c = 12.024 the edge value is small but not zero (the band-limited
    # reading of the Fourier-side integrals differs by O(psi(1)))
    ps = PSWF(12.024)
    assert 5e-5 < ps(1.0) < 1e-4


def test_integrals_against_quadrature():
    ps = PSWF(12.024)
    t, w = np.polynomial.legendre.leggauss(200)
    for kap in (0.0, 0.1, 0.37, 0.8, 1.0):
        u = kap + (1 - kap) * 0.5 * (t + 1)
        ww = (1 - kap) * 0.5 * w
        assert ps.J1(kap) == pytest.approx(np.sum(ww * u * ps(u)), abs=1e-14)
        assert ps.J3(kap) == pytest.approx(np.sum(ww * u ** 3 * ps(u)), abs=1e-14)
        if kap > 0:
            assert ps.L(kap) == pytest.approx(np.sum(ww * ps(u) / u), rel=1e-11)
