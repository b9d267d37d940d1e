"""Mollifiers, Fourier kernels, self and zero-frequency terms, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Notation: psi = psi_0^c with psi(0) = 1, C0 = int_0^1 psi, lambda0 = 2 C0,
rho = r / r_c, kappa = k r_c / c  (so k_c = c / r_c is kappa = 1).

Reading of the Fourier-side integrals (Methods, Eq. PhiH).  Every integral
of lambda0 psi(x/c) runs over x in [0, c]: psi is taken as supported on
[0, 1] on the Fourier side (band-limited reading), so
  Chat0 = int_0^c lambda0 psi(x/c) dx = lambda0 c C0,
and each kernel vanishes for k > k_c, matching the truncation |k| <= K_max
of Eq. Fourier.  With the substitution x = c u the kernels become

  Phi1 = 4 pi psi(kappa) / k^2
  Phi2 = (2 pi^2 / k) (1 - I0(kappa)/C0)
  Phi3 = (2 pi / C0) lambda0 L(kappa) = 4 pi L(kappa)
  Phi4 = -pi^2 k (1 - I0/C0) + pi^2 c J1 / (r_c C0)
  Phi5 = -(2 pi / 3) (k^2 L - c^2 J1 / r_c^2)
  Phi6 = (pi^2/12) (k^3 (1 - I0/C0) - (3 k^2 c / (2 r_c C0)) J1
                    + (c^3 / (2 r_c^3 C0)) J3)

with I0 = int_0^kappa psi, L = int_kappa^1 psi/u, J1 = int_kappa^1 u psi,
J3 = int_kappa^1 u^3 psi.  Their k-derivatives (for the virial) follow by
differentiating under the integral sign:

  Phi1' = 4 pi (kappa psi'(kappa) - 2 psi(kappa)) / k^3
  Phi2' = -Phi2 / k - 2 pi^2 kappa psi(kappa) / (C0 k^2)
  Phi3' = -4 pi psi(kappa) / k
  Phi4' = -pi^2 (1 - I0/C0)
  Phi5' = -(4 pi / 3) k L
  Phi6' = (pi^2 / 4) (k^2 (1 - I0/C0) - k c J1 / (r_c C0))

Pins: splitting independence of E_real + E_k + E_0 - E_self over (c, r_c)
for p = 1..6 (neutral and charged), the rock-salt Madelung constant (p = 1),
brute-force image sums (p = 4, 5, 6), the Fourier transform of G_p/r^p
computed by radial quadrature (p = 1, 2, 4, 6), and finite differences of
Phi_p for the derivatives (tests/test_oracle_kernels.py,
tests/test_oracle_invariants.py).
"""
import numpy as np

from .pswf import PSWF

_PSWF_CACHE = {}


def pswf(c):
    key = float(c)
    if key not in _PSWF_CACHE:
        _PSWF_CACHE[key] = PSWF(key)
    return _PSWF_CACHE[key]


def _unique_eval(fn, kappa):
    """Evaluate fn on the unique values of kappa (the oracle is slow per value)."""
    kap = np.asarray(kappa, dtype=np.float64)
    u, inv = np.unique(kap.ravel(), return_inverse=True)
    return fn(u)[inv].reshape(kap.shape)


def phi_hat(p, k, c, r_c):
    """Fourier kernel Phi_p(|k|) of G_p(r)/r^p (Eq. PhiH), zero for k > c/r_c.

    k must be > 0 for p <= 3 (singular at k = 0).
    """
    ps = pswf(c)
    k = np.asarray(k, dtype=np.float64)
    kap = k * r_c / c
    inside = kap <= 1.0
    kin = np.where(inside, kap, 1.0)

    def body(kk):
        kv = kk * c / r_c
        if p == 1:
            return 4.0 * np.pi * ps(kk) / kv ** 2
        if p == 2:
            return 2.0 * np.pi ** 2 / kv * (1.0 - ps.I0(kk) / ps.C0)
        if p == 3:
            return 4.0 * np.pi * ps.L(kk)
        if p == 4:
            return (-np.pi ** 2 * kv * (1.0 - ps.I0(kk) / ps.C0)
                    + np.pi ** 2 * c * ps.J1(kk) / (r_c * ps.C0))
        if p == 5:
            return -(2.0 * np.pi / 3.0) * (kv ** 2 * ps.L(kk) - c ** 2 * ps.J1(kk) / r_c ** 2)
        if p == 6:
            return (np.pi ** 2 / 12.0) * (
                kv ** 3 * (1.0 - ps.I0(kk) / ps.C0)
                - 3.0 * kv ** 2 * c / (2.0 * r_c * ps.C0) * ps.J1(kk)
                + c ** 3 / (2.0 * r_c ** 3 * ps.C0) * ps.J3(kk))
        raise ValueError("p must be in 1..6")

    val = _unique_eval(body, kin)
    return np.where(inside, val, 0.0)


def phi_hat_deriv(p, k, c, r_c):
    """d Phi_p / dk at |k| (closed forms in the module docstring)."""
    ps = pswf(c)
    k = np.asarray(k, dtype=np.float64)
    kap = k * r_c / c
    inside = kap <= 1.0
    kin = np.where(inside, kap, 1.0)

    def body(kk):
        kv = kk * c / r_c
        if p == 1:
            return 4.0 * np.pi * (kk * ps.d1(kk) - 2.0 * ps(kk)) / kv ** 3
        if p == 2:
            phi2 = 2.0 * np.pi ** 2 / kv * (1.0 - ps.I0(kk) / ps.C0)
            return -phi2 / kv - 2.0 * np.pi ** 2 * kk * ps(kk) / (ps.C0 * kv ** 2)
        if p == 3:
            return -4.0 * np.pi * ps(kk) / kv
        if p == 4:
            return -np.pi ** 2 * (1.0 - ps.I0(kk) / ps.C0)
        if p == 5:
            return -(4.0 * np.pi / 3.0) * kv * ps.L(kk)
        if p == 6:
            return (np.pi ** 2 / 4.0) * (kv ** 2 * (1.0 - ps.I0(kk) / ps.C0)
                                         - kv * c * ps.J1(kk) / (r_c * ps.C0))
        raise ValueError("p must be in 1..6")

    val = _unique_eval(body, kin)
    return np.where(inside, val, 0.0)


def mollifier(p, r, c, r_c):
    """G_p(r) of Eqs. G1, G6 and G; equal to 1 for r >= r_c."""
    ps = pswf(c)
    r = np.asarray(r, dtype=np.float64)
    rho = r / r_c
    inside = rho < 1.0
    x = np.where(inside, rho, 0.0)
    psi, d1, d2 = ps(x), ps.d1(x), ps.d2(x)
    if p == 1:
        g = ps.I0(x) / ps.C0
    elif p == 2:
        g = 1.0 - psi
    elif p == 3:
        g = (ps.I0(x) - x * psi) / ps.C0
    elif p == 4:
        g = 1.0 - psi + 0.5 * x * d1
    elif p == 5:
        g = (ps.I0(x) - x * psi + x * x / 3.0 * d1) / ps.C0
    elif p == 6:
        g = 1.0 - psi + 5.0 * x / 8.0 * d1 - x * x / 8.0 * d2
    else:
        raise ValueError("p must be in 1..6")
    return np.where(inside, g, 1.0)


def mollifier_deriv(p, r, c, r_c):
    """dG_p/dr of mollifier(): the rho-derivative of Eqs. G1, G6, G divided
    by r_c (each term differentiated by the product rule; G_p' = 0 for
    r >= r_c)."""
    ps = pswf(c)
    r = np.asarray(r, dtype=np.float64)
    rho = r / r_c
    inside = rho < 1.0
    x = np.where(inside, rho, 0.0)
    psi, d1, d2 = ps(x), ps.d1(x), ps.d2(x)
    if p == 1:
        g = psi / ps.C0
    elif p == 2:
        g = -d1
    elif p == 3:
        g = -x * d1 / ps.C0
    elif p == 4:
        g = -0.5 * d1 + 0.5 * x * d2
    elif p == 5:
        g = (-x * d1 / 3.0 + x * x * d2 / 3.0) / ps.C0
    elif p == 6:
        g = -3.0 * d1 / 8.0 + 3.0 * x * d2 / 8.0 - x * x * ps.d3(x) / 8.0
    else:
        raise ValueError("p must be in 1..6")
    return np.where(inside, g / r_c, 0.0)


def self_coefficient(p, c, r_c):
    """s_p with E_self^(p) = s_p * sum_i q_i^2 (Methods, self-correction term)."""
    ps = pswf(c)
    C0 = ps.C0
    d2 = ps.deriv_at_zero(2)
    d4 = ps.deriv_at_zero(4)
    d6 = ps.deriv_at_zero(6)
    psi0 = 1.0
    return {
        1: psi0 / (2.0 * C0 * r_c),
        2: -d2 / (4.0 * r_c ** 2),
        3: -d2 / (6.0 * C0 * r_c ** 3),
        4: d4 / (48.0 * r_c ** 4),
        5: d4 / (90.0 * C0 * r_c ** 5),
        6: -d6 / (1440.0 * r_c ** 6),
    }[p]


def zero_mode_coefficient(p, c, r_c, volume):
    """a_p with E_0^(p) = a_p * Q_net^2 (Methods, zero-frequency correction).

    p > 3 : Phi_p(0) / (2V).
    p = 3 : (2 pi / V) (ln(c/r_c) + int_0^1 (psi(r) - 1)/r dr)   (Eq. Correction3r),
            lengths in Angstrom.
    p = 2 : -(2 pi / V) int_0^{r_c} psi(r/r_c) dr = -(2 pi / V) r_c C0   (Eq. Correction).
    p = 1 : the printed p = 1 form does not give an energy independent of
            (c, r_c) for a charged cell; the k -> 0 limit of
            (Phi1 - 4 pi / k^2) Q^2 / (2V), equivalently the neutralising
            background seen through the real-space complement, does:
            -pi chi0 r_c^2 / (V c^2).  The infinite-boundary term is 0
            (tin-foil boundary).  Pinned by splitting independence.
    """
    ps = pswf(c)
    V = float(volume)
    if p == 1:
        return -np.pi * ps.chi * r_c ** 2 / (V * c ** 2)
    if p == 2:
        return -2.0 * np.pi * r_c * ps.C0 / V
    if p == 3:
        return 2.0 * np.pi / V * (np.log(c / r_c) + ps.T3(0.0))
    if p == 4:
        return 0.5 / V * (np.pi ** 2 * c * ps.J1(0.0) / (r_c * ps.C0))
    if p == 5:
        return 0.5 / V * ((2.0 * np.pi / 3.0) * c ** 2 * ps.J1(0.0) / r_c ** 2)
    if p == 6:
        return 0.5 / V * ((np.pi ** 2 / 12.0) * c ** 3 * ps.J3(0.0) / (2.0 * r_c ** 3 * ps.C0))
    raise ValueError("p must be in 1..6")
