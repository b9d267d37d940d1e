"""Order-zero prolate spheroidal wave function psi_0^c, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Methods, "Prolate spheroidal wave functions": psi_0^c is the
eigenfunction of the band-limiting operator F_c[phi](x) = int_{-1}^{1}
phi(t) exp(i c x t) dt with the largest eigenvalue lambda_0 (eq. formula,
eq. psidefinit), scaled so that psi_0^c(0) = 1.

Method.  psi_0^c is also the eigenfunction of the prolate differential
operator  L[psi] = -((1 - x^2) psi')' + c^2 x^2 psi  with the smallest
eigenvalue chi_0 (the classical commuting-operator property).  In the
normalised Legendre basis Pbar_k = sqrt(k + 1/2) P_k that operator is a
symmetric tridiagonal matrix on the even degrees (Bouwkamp's method, as
used by Xiao, Rokhlin and Yarvin, Inverse Problems 17 (2001)):

  A_kk     = k (k + 1) + c^2 (2k^2 + 2k - 1) / ((2k - 1)(2k + 3))
  A_k,k+2  = c^2 (k + 1)(k + 2) / ((2k + 3) sqrt((2k + 1)(2k + 5)))

The eigenvector gives the Legendre coefficients of psi_0^c.  Then
lambda_0 = int_{-1}^{1} psi_0^c (eq. psidefinit at x = 0) and
C_0 = int_0^1 psi_0^c = lambda_0 / 2 (eq. G1).

Pins (tests/test_oracle_pswf.py): the defining integral eigen-relation is
checked by quadrature at many x; psi''(0), psi''''(0), psi''''''(0) are
checked against the values the prolate ODE fixes at x = 0; lambda_0 is
checked against its large-c asymptote sqrt(2 pi / c).
"""
import numpy as np
from numpy.polynomial import legendre as npleg


class PSWF:
    """psi_0^c on [-1, 1] as a Legendre series, with psi_0^c(0) = 1."""

    def __init__(self, c, n_even=None):
        c = float(c)
        if not c > 0.0:
            raise ValueError("bandwidth c must be positive")
        n = int(n_even) if n_even is not None else max(48, int(1.5 * c) + 48)
        k = 2.0 * np.arange(n)
        diag = k * (k + 1.0) + c * c * (2.0 * k * k + 2.0 * k - 1.0) / (
            (2.0 * k - 1.0) * (2.0 * k + 3.0))
        kk = k[:-1]
        off = c * c * (kk + 1.0) * (kk + 2.0) / (
            (2.0 * kk + 3.0) * np.sqrt((2.0 * kk + 1.0) * (2.0 * kk + 5.0)))
        a = np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)
        evals, evecs = np.linalg.eigh(a)
        self.c = c
        self.chi = float(evals[0])
        beta = evecs[:, 0]
        coef = np.zeros(2 * n)
        coef[0::2] = beta * np.sqrt(k + 0.5)      # coefficients on P_k
        coef /= npleg.legval(0.0, coef)            # psi(0) = 1
        self.coef = coef
        # lambda_0 psi(0) = int_{-1}^{1} psi(t) dt ; only P_0 has nonzero mean.
        self.lam = 2.0 * coef[0]
        self.C0 = 0.5 * self.lam
        self._d1 = npleg.legder(coef, 1)
        self._d2 = npleg.legder(coef, 2)
        self._d3 = npleg.legder(coef, 3)
        self._int = npleg.legint(coef, lbnd=0.0)            # int_0^x psi
        self._int_x = npleg.legint(npleg.legmulx(coef), lbnd=0.0)   # int_0^x u psi
        x3 = npleg.legmulx(npleg.legmulx(npleg.legmulx(coef)))
        self._int_x3 = npleg.legint(x3, lbnd=0.0)           # int_0^x u^3 psi

    # -- values ---------------------------------------------------------
    def __call__(self, x):
        """psi_0^c(x) for |x| <= 1 (values outside are not defined here)."""
        return npleg.legval(np.asarray(x, dtype=np.float64), self.coef)

    def d1(self, x):
        return npleg.legval(np.asarray(x, dtype=np.float64), self._d1)

    def d2(self, x):
        return npleg.legval(np.asarray(x, dtype=np.float64), self._d2)

    def d3(self, x):
        return npleg.legval(np.asarray(x, dtype=np.float64), self._d3)

    def deriv_at_zero(self, n):
        """n-th derivative of psi_0^c at 0, from the Legendre series."""
        return float(npleg.legval(0.0, npleg.legder(self.coef, n)))

    # -- integrals over [0, kappa] and [kappa, 1] ------------------------
    def I0(self, kappa):
        """int_0^kappa psi(u) du."""
        return npleg.legval(np.asarray(kappa, dtype=np.float64), self._int)

    def J1(self, kappa):
        """int_kappa^1 u psi(u) du."""
        kap = np.asarray(kappa, dtype=np.float64)
        return npleg.legval(1.0, self._int_x) - npleg.legval(kap, self._int_x)

    def J3(self, kappa):
        """int_kappa^1 u^3 psi(u) du."""
        kap = np.asarray(kappa, dtype=np.float64)
        return npleg.legval(1.0, self._int_x3) - npleg.legval(kap, self._int_x3)

    def T3(self, kappa, nquad=96):
        """int_kappa^1 (psi(u) - 1)/u du  (smooth, finite at kappa = 0).

        Written as T3(0) - int_0^kappa (psi(u) - 1)/u du and the second
        integral as int_0^1 (psi(kappa s) - 1)/s ds by Gauss-Legendre.
        """
        kap = np.atleast_1d(np.asarray(kappa, dtype=np.float64))
        xs, ws = np.polynomial.legendre.leggauss(nquad)
        s = 0.5 * (xs + 1.0)
        w = 0.5 * ws
        full = np.sum(w * (self(s) - 1.0) / s)
        out = np.empty_like(kap)
        chunk = max(1, 2_000_000 // nquad)
        for i in range(0, kap.size, chunk):
            kk = kap[i:i + chunk, None]
            vals = (self(kk * s[None, :]) - 1.0) / s[None, :]
            out[i:i + chunk] = full - np.sum(w[None, :] * vals, axis=1)
        return out.reshape(np.shape(kappa)) if np.ndim(kappa) else float(out[0])

    def L(self, kappa):
        """int_kappa^1 psi(u)/u du = -ln(kappa) + T3(kappa), kappa > 0."""
        kap = np.asarray(kappa, dtype=np.float64)
        return -np.log(kap) + self.T3(kap)


def ode_derivatives_at_zero(chi, c, nmax):
    """psi^(n)(0) for even n <= nmax from the prolate ODE alone.

    Differentiating (1 - x^2) psi'' - 2 x psi' + (chi - c^2 x^2) psi = 0
    n times at x = 0 gives
        psi^(n+2)(0) = (n (n + 1) - chi) psi^(n)(0) + c^2 n (n - 1) psi^(n-2)(0).
    Independent of the Legendre representation; used as a pin.
    """
    d = {0: 1.0, 2: -chi}
    for n in range(2, nmax - 1, 2):
        d[n + 2] = (n * (n + 1) - chi) * d[n] + c * c * n * (n - 1) * d[n - 2]
    return d
