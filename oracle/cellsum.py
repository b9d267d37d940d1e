"""Truncated Fourier sum for a general (triclinic) cell, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The same quantities as oracle.reciprocal (Eq. Fourier with the truncation
0 < |k| <= k_c = c / r_c, per-channel latent structure factors), for a cell
whose lattice vectors are the rows of a 3x3 matrix H (the cell tensor of the
Fig. 1 caption; an orthorhombic box is H = diag(L)):

  s_j = r_j H^-1                       fractional coordinates
  k(m) = 2 pi m H^-T                   reciprocal-lattice vectors, m integer
  S(m) = sum_j q_j exp(2 pi i m . s_j) = sum_j q_j exp(i k . r_j)
  E_k  = (1 / 2V) sum_{0<|k|<=k_c} Phi_p(|k|) |S|^2,   V = |det H|

S is formed for every m of the bounding box |m_a| <= k_c |a_a| / 2 pi
(|m_a| = |k . a_a| / 2 pi) in the half space m_z > 0, or m_z = 0 and
m_y > 0, or m_z = m_y = 0 and m_x > 0, from separable phase tables
e^(2 pi i m_a s_ja): for each m_x the product over y and z is a matrix
product over atoms (the library primitive).  Potentials and forces are
formed only for the atoms asked for (`sample`), the energy and virial
always from all atoms:

  phi_i = (1/V) sum_k Phi_p Re(conj(S) e^(i k.r_i)) + 2 a_p Q_net
  F_i   = (q_i / V) sum_k Phi_p k Im(conj(S) e^(i k.r_i))
  W_ab  = (1 / 2V) sum_k |S|^2 (Phi_p delta_ab + Phi_p'(k) k_a k_b / k)
          + E_0 delta_ab                (W = -dE/d strain_ab)

(all sums over the full ball; the half space is counted twice).  E_0 and
E_self are those of oracle.kernels.

Pins (tests/test_oracle_cellsum.py): equality with the plain direct sum of
oracle.reciprocal on orthorhombic boxes (a different evaluation of the same
definition); invariance of every output under a unimodular change of the
lattice basis (the same lattice described by other vectors); forces equal
to minus central finite differences of the energy in a triclinic cell; the
whole virial tensor, off-diagonal entries included, equal to minus central
finite differences of the energy under affine strain of the cell and the
positions; force_vjp (the double backward) against central differences of
L = sum v . F formed from the forces of evaluate.
"""
import numpy as np

from . import kernels


def half_space_modes(cell, k_cut):
    """Integer m in the half space with 0 < |k(m)| <= k_cut, k(m) = 2 pi m H^-T.

    Returns (m [K,3], k [K,3], |k| [K], mmax [3])."""
    H = np.asarray(cell, dtype=np.float64)
    lens = np.sqrt(np.sum(H * H, axis=1))
    mmax = np.floor(k_cut * lens / (2.0 * np.pi) + 1e-9).astype(int)
    ax = [np.arange(-mm, mm + 1) for mm in mmax]
    mx, my, mz = np.meshgrid(*ax, indexing="ij")
    m = np.stack([mx.ravel(), my.ravel(), mz.ravel()], axis=1)
    half = (m[:, 2] > 0) | ((m[:, 2] == 0) & (m[:, 1] > 0)) | (
        (m[:, 2] == 0) & (m[:, 1] == 0) & (m[:, 0] > 0))
    m = m[half]
    kvec = 2.0 * np.pi * m @ np.linalg.inv(H).T
    kn = np.sqrt(np.sum(kvec * kvec, axis=1))
    keep = kn <= k_cut
    return m[keep], kvec[keep], kn[keep], mmax


def structure_factors(frac, q, m, mmax):
    """S(m) = sum_j q_j exp(2 pi i m . s_j) for the listed m (m_z >= 0)."""
    frac = np.asarray(frac, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    n = frac.shape[0]
    mxr = np.arange(-mmax[0], mmax[0] + 1)
    myr = np.arange(-mmax[1], mmax[1] + 1)
    mzr = np.arange(0, mmax[2] + 1)
    ex = np.exp(2j * np.pi * frac[:, 0:1] * mxr[None, :])     # [N, nx]
    ey = np.exp(2j * np.pi * frac[:, 1:2] * myr[None, :])     # [N, ny]
    ez = np.exp(2j * np.pi * frac[:, 2:3] * mzr[None, :])     # [N, nz]
    S = np.zeros((mxr.size, myr.size, mzr.size), dtype=np.complex128)
    if n == 0:
        return np.zeros(m.shape[0], dtype=np.complex128)
    for ix in range(mxr.size):
        a = (q * ex[:, ix])[:, None] * ey                      # [N, ny]
        S[ix] = a.T @ ez                                       # sum over atoms
    return S[m[:, 0] + mmax[0], m[:, 1] + mmax[1], m[:, 2]]


def evaluate(pos, q, cell, ps, c, r_c, sample=None, virial=True, chunk=8192):
    """All channels of a general cell.  q is [C, N]; cell is H (rows are the
    lattice vectors); sample lists the atoms whose potentials and forces are
    wanted (None: all).

    Returns per-channel Ek, E0, Eself, phi [C, len(sample)], F [len(sample), 3]
    of sum_c (E_k + E_0), W [3, 3] and the sample indices."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    H = np.asarray(cell, dtype=np.float64)
    V = abs(float(np.linalg.det(H)))
    C, n = q.shape
    idx = np.arange(n) if sample is None else np.asarray(sample, dtype=np.int64)
    frac = pos @ np.linalg.inv(H)
    m, kvec, kn, mmax = half_space_modes(H, c / r_c)
    Ek = np.zeros(C)
    E0 = np.zeros(C)
    Es = np.zeros(C)
    phi = np.zeros((C, idx.size))
    F = np.zeros((idx.size, 3))
    W = np.zeros((3, 3))
    for ch in range(C):
        p = int(ps[ch])
        S = structure_factors(frac, q[ch], m, mmax)
        S2 = (S * np.conj(S)).real
        fk = kernels.phi_hat(p, kn, c, r_c)
        Ek[ch] = np.sum(fk * S2) / V                           # (1/2V) x 2 half spaces
        a = kernels.zero_mode_coefficient(p, c, r_c, V)
        qn = float(np.sum(q[ch]))
        E0[ch] = a * qn * qn
        Es[ch] = kernels.self_coefficient(p, c, r_c) * float(np.sum(q[ch] ** 2))
        if virial:
            dk = kernels.phi_hat_deriv(p, kn, c, r_c)
            W += np.einsum("k,ka,kb->ab", S2 * dk / kn, kvec, kvec) / V
            W += np.eye(3) * (Ek[ch] + E0[ch])
        for s in range(0, kn.size, chunk):
            kv = kvec[s:s + chunk]
            ph = np.exp(1j * (pos[idx] @ kv.T))                # [n_sample, K]
            t = np.conj(S[s:s + chunk])[None, :] * ph
            f = fk[s:s + chunk]
            phi[ch] += (2.0 / V) * (t.real @ f)
            F += (2.0 / V) * q[ch][idx][:, None] * ((t.imag * f[None, :]) @ kv)
        phi[ch] += 2.0 * a * qn
    return {"Ek": Ek, "E0": E0, "Eself": Es, "phi": phi, "F": F, "W": W, "sample": idx}


def force_vjp(pos, q, cell, ps, c, r_c, v):
    """Derivatives of L = sum_i v_i . F_i (F the forces of sum_c E_k + E_0)
    in the charges and positions, for a general cell: the same sums as
    oracle.reciprocal.force_vjp over k = 2 pi m H^-T, V = |det H|.  With
    T(k) = sum_i q_i (v_i . k) e^{i k.r_i} and S the structure factor,

      dL/dq_j = (1/V) sum_k Phi_p Im(e^{-i k.r_j} T + conj(S) (v_j . k) e^{i k.r_j})
      dL/dr_j = (q_j/V) sum_k Phi_p k [-Re(e^{-i k.r_j} T) + (v_j . k) Re(conj(S) e^{i k.r_j})]

    over the whole ball (the half space counted twice).  Returns dq [C, N]
    and dr [N, 3] (summed over channels)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    v = np.asarray(v, dtype=np.float64)
    H = np.asarray(cell, dtype=np.float64)
    V = abs(float(np.linalg.det(H)))
    C, n = q.shape
    _, kvec, kn, _ = half_space_modes(H, c / r_c)
    dq = np.zeros((C, n))
    dr = np.zeros((n, 3))
    for ch in range(C):
        fk = kernels.phi_hat(int(ps[ch]), kn, c, r_c)
        for s in range(0, kn.size, 4096):
            kv = kvec[s:s + 4096]
            f = fk[s:s + 4096]
            ph = np.exp(1j * (pos @ kv.T))            # [N, K]
            vk = v @ kv.T                             # v_i . k
            S = q[ch] @ ph
            T = (q[ch][:, None] * vk * ph).sum(axis=0)
            a = np.conj(ph) * T[None, :]
            b = np.conj(S)[None, :] * ph
            dq[ch] += (2.0 / V) * ((a.imag + vk * b.imag) @ f)
            dr += (2.0 / V) * q[ch][:, None] * (((-a.real + vk * b.real) * f[None, :]) @ kv)
    return dq, dr
