"""Direct structure-factor sum of the truncated Fourier energy, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Follows Eq. Fourier with the truncation |k| <= K_max = k_c = c / r_c and the
latent structure factor rho^(p)(k) = sum_i q_i exp(i k . r_i):

  E_k   = (1 / 2V) sum_{0 < |k| <= k_c} Phi_p(|k|) |S(k)|^2
  phi_i = dE_k/dq_i = (1/V) sum_k Phi_p Re(conj(S(k)) exp(i k . r_i))
  F_i   = -dE_k/dr_i = (q_i / V) sum_k Phi_p k Im(conj(S(k)) exp(i k . r_i))
  W_ab  = -dE/d(strain_ab)
        = (1/2V) sum_k |S|^2 (Phi_p delta_ab + Phi_p'(k) k_a k_b / k)

with k = 2 pi m / L (orthorhombic cell, m integer).  Only the half space of
m is enumerated; every term is even in k, so the full sum is twice it.  No
mesh is involved: this is the plain definition the mesh method approximates.

Zero-frequency terms E_0 = a_p Q_net^2 (oracle.kernels) are added by
`evaluate`; they contribute 2 a_p Q_net to every potential, nothing to the
forces and E_0 delta_ab to the virial (every a_p scales as 1/V).

`force_vjp` differentiates L = sum_i v_i . F_i once more (the double
backward of force-matching training).

Pins: forces against central finite differences of E_k, virial against
finite differences of the energy under affine strain, zero net force,
translation invariance, E(lambda q) = lambda^2 E, and the total-energy pins
of tests/test_oracle_invariants.py that use E_k; force_vjp against central
finite differences of sum_i v_i . F_i in charges and positions
(tests/test_oracle_double_backward.py).
"""
import numpy as np

from . import kernels


def half_space_modes(box, k_cut):
    """Integer vectors m in the half space with 0 < |2 pi m / L| <= k_cut."""
    box = np.asarray(box, dtype=np.float64)
    mmax = np.floor(k_cut * box / (2.0 * np.pi)).astype(int)
    ax = [np.arange(-mm, mm + 1) for mm in mmax]
    mx, my, mz = np.meshgrid(*ax, indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    half = (m[:, 2] > 0) | ((m[:, 2] == 0) & (m[:, 1] > 0)) | (
        (m[:, 2] == 0) & (m[:, 1] == 0) & (m[:, 0] > 0))
    m = m[half]
    kvec = 2.0 * np.pi * m / box[None, :]
    kn = np.sqrt(np.sum(kvec * kvec, axis=1))
    keep = kn <= k_cut
    return m[keep], kvec[keep], kn[keep]


def reciprocal_channel(pos, q, box, p, c, r_c, forces=True, potential=True,
                       virial=True, chunk=4096):
    """One channel: returns dict(E, phi[N], F[N,3], W[3,3]) of the k-space sum."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    k_cut = c / r_c
    _, kvec, kn = half_space_modes(box, k_cut)
    phi_k = kernels.phi_hat(p, kn, c, r_c)
    dphi_k = kernels.phi_hat_deriv(p, kn, c, r_c) if virial else None
    n = pos.shape[0]
    E = 0.0
    phi = np.zeros(n)
    F = np.zeros((n, 3))
    W = np.zeros((3, 3))
    for s in range(0, kn.size, chunk):
        kv = kvec[s:s + chunk]
        ph = np.exp(1j * (pos @ kv.T))            # [N, K] exp(i k . r_j)
        S = q @ ph                                # [K]
        S2 = (S * np.conj(S)).real
        fk = phi_k[s:s + chunk]
        # half space counted twice: (1/2V) * 2 = 1/V
        E += np.sum(fk * S2) / V
        if potential or forces:
            t = np.conj(S)[None, :] * ph          # conj(S) exp(i k r_i)
            if potential:
                phi += (2.0 / V) * (t.real @ fk)
            if forces:
                F += (2.0 / V) * q[:, None] * ((t.imag * fk[None, :]) @ kv)
        if virial:
            kk = kn[s:s + chunk]
            wgt = S2 * dphi_k[s:s + chunk] / kk
            W += np.einsum("k,ka,kb->ab", wgt, kv, kv) / V
            W += np.eye(3) * np.sum(fk * S2) / V
    return {"E": E, "phi": phi, "F": F, "W": W}


def force_vjp(pos, q, box, ps, c, r_c, v):
    """Derivatives of L = sum_i v_i . F_i (a force-matching loss linearised
    at upstream gradient v [N, 3]) with respect to the charges and the
    positions, from the same Fourier sum.  With T(k) = sum_i q_i (v_i . k)
    e^{i k.r_i}, L = (1/V) sum_k Phi_p Im(conj(S) T) over the whole ball, so

      dL/dq_j = (1/V) sum_k Phi_p Im(e^{-i k.r_j} T + conj(S) (v_j . k) e^{i k.r_j})
      dL/dr_j = (q_j/V) sum_k Phi_p k [-Re(e^{-i k.r_j} T) + (v_j . k) Re(conj(S) e^{i k.r_j})]

    (every term is even in k: the half space is counted twice).  E_0 does
    not depend on the positions and adds nothing.  Returns dq [C, N] and
    dr [N, 3] (summed over channels)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    v = np.asarray(v, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    C, n = q.shape
    _, kvec, kn = half_space_modes(box, c / r_c)
    dq = np.zeros((C, n))
    dr = np.zeros((n, 3))
    for ch in range(C):
        fk = kernels.phi_hat(int(ps[ch]), kn, c, r_c)
        for s in range(0, kn.size, 4096):
            kv = kvec[s:s + 4096]
            f = fk[s:s + 4096]
            ph = np.exp(1j * (pos @ kv.T))            # [N, K]
            vk = v @ kv.T                             # [N, K] v_i . k
            S = q[ch] @ ph
            T = (q[ch][:, None] * vk * ph).sum(axis=0)
            a = np.conj(ph) * T[None, :]              # e^{-ik r_j} T
            b = np.conj(S)[None, :] * ph              # conj(S) e^{ik r_j}
            dq[ch] += (2.0 / V) * ((a.imag + vk * b.imag) @ f)
            dr += (2.0 / V) * q[ch][:, None] * (((-a.real + vk * b.real) * f[None, :]) @ kv)
    return dq, dr


def evaluate(pos, q, box, ps, c, r_c, forces=True, potential=True, virial=True):
    """All channels.  q is [C, N], ps the exponents [C].

    Returns per-channel E_k, E_0, E_self (the energy vector the library
    returns), total potentials phi[C, N] = d(E_k + E_0)/dq, forces F[N, 3]
    and virial W[3, 3] of E_k + E_0.
    """
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    C, n = q.shape
    Ek = np.zeros(C)
    E0 = np.zeros(C)
    Es = np.zeros(C)
    phi = np.zeros((C, n))
    F = np.zeros((n, 3))
    W = np.zeros((3, 3))
    for ch in range(C):
        p = int(ps[ch])
        r = reciprocal_channel(pos, q[ch], box, p, c, r_c, forces, potential, virial)
        a = kernels.zero_mode_coefficient(p, c, r_c, V)
        qn = float(np.sum(q[ch]))
        Ek[ch] = r["E"]
        E0[ch] = a * qn * qn
        Es[ch] = kernels.self_coefficient(p, c, r_c) * float(np.sum(q[ch] ** 2))
        phi[ch] = r["phi"] + 2.0 * a * qn
        F += r["F"]
        W += r["W"] + E0[ch] * np.eye(3)
    return {"Ek": Ek, "E0": E0, "Eself": Es, "phi": phi, "F": F, "W": W}
