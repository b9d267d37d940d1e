"""Pins for oracle.kernels: the Fourier kernels of Eq. PhiH against the
Fourier transform of the real-space mollifiers of Eqs. G1, G6, G computed
by radial quadrature; the kernel derivatives against finite differences;
the printed self-energy coefficients against the r -> 0 limit of G_p/r^p."""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.special import sici

from oracle import kernels
from oracle.pswf import ode_derivatives_at_zero

C_BIG = 30.0     # psi(1) ~ 2e-12: the band-limited reading is exact to that order
RC = 2.5


def _tail(p, k, a):
    """int_a^inf r^(1-p) sin(k r) dr by integration by parts down to the
    sine/cosine integrals; p = 1 uses Abel summation (cos(k a) / k)."""
    if p == 1:
        return np.cos(k * a) / k
    si, ci = sici(k * a)
    I = {1: np.pi / 2 - si}
    J = {1: -ci}
    for n in range(2, p):
        I[n] = np.sin(k * a) / ((n - 1) * a ** (n - 1)) + k / (n - 1) * J[n - 1]
        J[n] = np.cos(k * a) / ((n - 1) * a ** (n - 1)) - k / (n - 1) * I[n - 1]
    return I[p - 1]


def _taylor_kernel(p, r, c, rc, nterm=40):
    """G_p(r)/r^p near r = 0 from the Taylor series of psi, whose derivatives
    at 0 come from the prolate ODE (not from the Legendre series).  Avoids the
    cancellation of the O(1) terms of G_p that leave an O(r^p) remainder."""
    ps = kernels.pswf(c)
    d = ode_derivatives_at_zero(ps.chi, c, 2 * nterm + 2)
    rho = np.asarray(r, dtype=np.float64) / rc
    out = np.zeros_like(rho)
    for j in range(nterm):
        a = d[2 * j] / math.factorial(2 * j)
        n = 2 * j
        one = Fraction(1)
        # exact combinatorial factor of a_{2j} in the series of G_p
        if p == 1:
            fac, power, div = one / (n + 1), n + 1, ps.C0
        elif p == 2:
            fac, power, div = (-one if j > 0 else 0 * one), n, 1.0
        elif p == 3:
            fac, power, div = one / (n + 1) - 1, n + 1, ps.C0
        elif p == 4:
            fac, power, div = (-one + Fraction(n, 2) if j > 0 else 0 * one), n, 1.0
        elif p == 5:
            fac, power, div = one / (n + 1) - 1 + Fraction(n, 3), n + 1, ps.C0
        else:
            fac = (-one + Fraction(5 * n, 8) - Fraction(n * (n - 1), 8)) if j > 0 else 0 * one
            power, div = n, 1.0
        coef = 0.0 if fac == 0 else a * float(fac) / div
        if coef == 0.0:
            continue
        out += coef * rho ** (power - p)
    return out / rc ** p


def _ft_radial(p, k, c, rc):
    """Phi_p(k) = (4 pi / k) int_0^inf G_p(r) r^(1-p) sin(k r) dr."""
    t, w = np.polynomial.legendre.leggauss(200)
    rs = 0.25 * rc
    r1 = 0.5 * rs * (t + 1.0)
    inner = np.sum(0.5 * rs * w * _taylor_kernel(p, r1, c, rc) * r1 * np.sin(k * r1))
    r2 = rs + 0.5 * (rc - rs) * (t + 1.0)
    inner += np.sum(0.5 * (rc - rs) * w * kernels.mollifier(p, r2, c, rc)
                    * r2 ** (1 - p) * np.sin(k * r2))
    return 4.0 * np.pi / k * (inner + _tail(p, k, rc))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_phi_hat_is_fourier_transform_of_mollified_kernel(p):
    kc = C_BIG / RC
    for k in (0.05 * kc, 0.2 * kc, 0.5 * kc, 0.8 * kc, 0.97 * kc):
        ref = _ft_radial(p, k, C_BIG, RC)
        got = float(kernels.phi_hat(p, np.array([k]), C_BIG, RC)[0])
        scale = max(abs(ref), abs(_ft_radial(p, 0.05 * kc, C_BIG, RC)))
        assert abs(got - ref) < 1e-8 * scale, (p, k, got, ref)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_phi_hat_vanishes_outside_band(p):
    kc = 12.024 / 5.0
    v = kernels.phi_hat(p, np.array([1.0001 * kc, 2 * kc]), 12.024, 5.0)
    assert np.all(v == 0.0)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_phi_hat_derivative_matches_finite_difference(p):
    c, rc = 12.024, 5.0
    kc = c / rc
    k = np.array([0.07, 0.3, 0.55, 0.9]) * kc
    d = 1e-5 * kc
    fd = (kernels.phi_hat(p, k + d, c, rc) - kernels.phi_hat(p, k - d, c, rc)) / (2 * d)
    an = kernels.phi_hat_deriv(p, k, c, rc)
    assert np.allclose(an, fd, rtol=2e-7, atol=2e-8 * np.max(np.abs(fd)))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_self_coefficient_is_half_limit_of_mollified_kernel(p):
    # E_self = 1/2 Q_self lim_{r->0} G_p(r)/r^p, the limit taken on the
    # Taylor series of G_p built from the ODE-derived psi^(n)(0).
    c, rc = 12.024, 5.0
    lim = float(_taylor_kernel(p, np.array([1e-9 * rc]), c, rc)[0])
    assert 0.5 * lim == pytest.approx(kernels.self_coefficient(p, c, rc), rel=1e-9)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_mollifier_matches_taylor_series(p):
    # the oracle's G_p (Legendre series of psi) against the ODE Taylor series
    c, rc = 12.024, 5.0
    r = np.array([0.15, 0.25, 0.35]) * rc
    got = kernels.mollifier(p, r, c, rc) / r ** p
    ref = _taylor_kernel(p, r, c, rc, nterm=60)
    assert np.allclose(got, ref, rtol=1e-8)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_mollifier_long_range_limit(p):
    # G_p(r)/r^p -> 1/r^p (Eq. G): exactly 1 beyond r_c, and continuous
    # at r_c up to the O(psi(1)) edge value.
    c, rc = C_BIG, RC
    assert np.all(kernels.mollifier(p, np.array([rc, 1.5 * rc]), c, rc) == 1.0)
    g = kernels.mollifier(p, np.array([rc * (1 - 1e-9)]), c, rc)[0]
    assert g == pytest.approx(1.0, abs=1e-7)
