"""The paper's four-step mesh algorithm in plain form, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Methods, "Accelerating atom-grid spreading with PSWFs" (Eq. EthetaLR and
the four steps after it):

 (i)   spread: g(n) = sum_j q_j [W(n h - r_j)]_*  with the separable window
       W(r) = prod_a psi_s(r_a / omega), |r_a| <= omega = P h / 2, periodised;
 (ii)  forward 3D FFT of g (numpy's FFT serves as the library primitive);
 (iii) diagonal scaling by What(k)^-2 Phi_p(k) / 2V with
       What(k) = prod_a omega lambda_s psi_s(omega k_a / c_s);
 (iv)  reduction over 0 < |k| <= k_c.

Forces (Fig. 1 caption: obtained by differentiation) use the exact adjoint:
phi_grid = dE/dg = (1/V) IDFT(K F) with K = Phi_p h^6 / What^2, gathered
with W for potentials and with grad W for forces.

Readings of the paper used here:
 * the spreading window has its own bandwidth c_s (the paper reuses the
   symbol c for both the mollifier and the window);
 * grid nodes sit at n h, n = 0..M-1; each atom touches the P nodes with
   n h - x in [-omega, omega), i.e. n = ceil(x/h - P/2) + l, l = 0..P-1;
 * rho_grid(k) = h^3 DFT(g)(k) approximates What(k) conj(S(k));
 * Nyquist frequencies |m_a| = M_a / 2 are excluded from the sum.

Pins: mesh energy and forces converge to the direct sum of oracle.reciprocal
as P grows (spectral convergence); mesh forces equal minus the finite
difference of the mesh energy (tests/test_oracle_mesh.py).
"""
import numpy as np

from . import kernels
from .pswf import PSWF

_CACHE = {}


def window_pswf(c_s):
    key = float(c_s)
    if key not in _CACHE:
        _CACHE[key] = PSWF(key)
    return _CACHE[key]


def _window_points(pos, box, M, P, c_s):
    """Per atom and axis: node indices [N,3,P], psi_s weights and derivatives."""
    ws = window_pswf(c_s)
    box = np.asarray(box, dtype=np.float64)
    M = np.asarray(M, dtype=np.int64)
    h = box / M
    x = np.mod(np.asarray(pos, dtype=np.float64), box)
    u = x / h
    n0 = np.ceil(u - 0.5 * P)
    l = np.arange(P)
    nodes = n0[:, :, None] + l[None, None, :]
    t = 2.0 * (nodes - u[:, :, None]) / P           # in [-1, 1)
    w = ws(t)
    dw = ws.d1(t) / (0.5 * P * h[None, :, None])     # d/dd of psi_s(d/omega)
    idx = np.mod(nodes.astype(np.int64), M[None, :, None])
    return idx, w, dw


def spread(pos, q, box, M, P, c_s):
    """Step (i): the periodised PSWF-window grid of one channel, [Mx, My, Mz]."""
    M = tuple(int(m) for m in M)
    idx, w, _ = _window_points(pos, box, M, P, c_s)
    q = np.asarray(q, dtype=np.float64)
    g = np.zeros(M)
    n = idx.shape[0]
    for a in range(P):
        for b in range(P):
            wab = q * w[:, 0, a] * w[:, 1, b]
            ix = idx[:, 0, a]
            iy = idx[:, 1, b]
            for cc in range(P):
                np.add.at(g, (ix, iy, idx[:, 2, cc]), wab * w[:, 2, cc])
    return g


def signed_freq(M):
    return np.fft.fftfreq(M, 1.0 / M).round().astype(np.int64)


def scaling(box, M, P, c_s, p, c, r_c):
    """Step (iii) without the 1/2V: K(m) = Phi_p h^6 / What^2 and the mode mask."""
    box = np.asarray(box, dtype=np.float64)
    ws = window_pswf(c_s)
    h = box / np.asarray(M)
    f = [signed_freq(m) for m in M]
    k1 = [2.0 * np.pi * f[a] / box[a] for a in range(3)]
    # What_a(k) / h = (P/2) lambda_s psi_s(omega k / c_s), omega k = pi P f / M
    wr = [0.5 * P * ws.lam * ws(np.pi * P * f[a] / (M[a] * c_s)) for a in range(3)]
    KX, KY, KZ = np.meshgrid(*k1, indexing="ij")
    kn = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    ok = (kn > 0) & (kn <= c / r_c)
    for a, (fa, ma) in enumerate(zip(f, M)):
        nyq = np.abs(fa) * 2 == ma
        shape = [1, 1, 1]
        shape[a] = ma
        ok &= ~nyq.reshape(shape)
    wx, wy, wz = np.meshgrid(*wr, indexing="ij")
    phi = np.zeros_like(kn)
    dphi = np.zeros_like(kn)
    phi[ok] = kernels.phi_hat(p, kn[ok], c, r_c)
    dphi[ok] = kernels.phi_hat_deriv(p, kn[ok], c, r_c)
    D = 1.0 / (wx * wy * wz) ** 2                      # h^6 / What^2
    return phi * D, dphi * D, (KX, KY, KZ, kn), ok


def evaluate(pos, q, box, ps, c, r_c, M, P, c_s):
    """All four steps plus the adjoint gather for every channel.

    q is [C, N].  Returns the same dictionary as oracle.reciprocal.evaluate,
    plus the spread grids.
    """
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    M = tuple(int(m) for m in M)
    Mt = float(np.prod(M))
    idx, w, dw = _window_points(pos, box, M, P, c_s)
    C, n = q.shape
    Ek = np.zeros(C)
    E0 = np.zeros(C)
    Es = np.zeros(C)
    phi = np.zeros((C, n))
    F = np.zeros((n, 3))
    W = np.zeros((3, 3))
    grids = []
    for ch in range(C):
        p = int(ps[ch])
        g = spread(pos, q[ch], box, M, P, c_s)
        grids.append(g)
        Fk = np.fft.fftn(g)
        K, dK, (KX, KY, KZ, kn), ok = scaling(box, M, P, c_s, p, c, r_c)
        S2 = (Fk * np.conj(Fk)).real
        Ek[ch] = np.sum(K * S2) / (2.0 * V)
        knz = np.where(ok, kn, 1.0)
        wv = S2 * dK / knz
        kv = [KX, KY, KZ]
        for a in range(3):
            for b in range(3):
                W[a, b] += np.sum(wv * kv[a] * kv[b]) / (2.0 * V)
        W += np.eye(3) * Ek[ch]
        pg = (np.fft.ifftn(K * Fk) * Mt).real / V       # dE/dg(n)
        # gather: phi_i = sum W pg, F_i = q_i sum gradW pg
        a_ = kernels.zero_mode_coefficient(p, c, r_c, V)
        qn = float(np.sum(q[ch]))
        E0[ch] = a_ * qn * qn
        Es[ch] = kernels.self_coefficient(p, c, r_c) * float(np.sum(q[ch] ** 2))
        W += E0[ch] * np.eye(3)
        pot = np.zeros(n)
        gr = np.zeros((n, 3))
        for a in range(P):
            for b in range(P):
                for cc in range(P):
                    v = pg[idx[:, 0, a], idx[:, 1, b], idx[:, 2, cc]]
                    pot += v * w[:, 0, a] * w[:, 1, b] * w[:, 2, cc]
                    gr[:, 0] += v * dw[:, 0, a] * w[:, 1, b] * w[:, 2, cc]
                    gr[:, 1] += v * w[:, 0, a] * dw[:, 1, b] * w[:, 2, cc]
                    gr[:, 2] += v * w[:, 0, a] * w[:, 1, b] * dw[:, 2, cc]
        phi[ch] = pot + 2.0 * a_ * qn
        # E depends on r_j through W(n h - r_j): dE/dr_j = -q_j sum pg gradW
        F += q[ch][:, None] * gr
    return {"Ek": Ek, "E0": E0, "Eself": Es, "phi": phi, "F": F, "W": W,
            "grids": grids}
