"""Real-space complement (1 - G_p(r)) / r^p summed over periodic images, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Methods, "Implementation details": the Fourier sum of Eq. Fourier is paired
with the real-space term (1 - G_p)/r^p and the self-correction E_self for a
complete decomposition of Eq. realLR:

  E_total = E_real + E_k + E_0 - E_self,
  E_real  = 1/2 sum_n sum'_{i,j} q_i q_j (1 - G_p(|r_ij + n L|)) / |r_ij + n L|^p

with G_p from Eqs. G1, G6, G and the prime excluding i = j at n = 0.
1 - G_p vanishes for r >= r_c, so only images within r_c contribute.  The
cell may be general (lattice vectors as the rows of H, the cell tensor of
the Fig. 1 caption): image n is the lattice vector n H, and differences are
first reduced to the nearest image in fractional coordinates.

`evaluate` gives, per channel, E_real and the potentials
phi_i = dE_real/dq_i = sum_{j,n}' q_j K(r), and in total over channels the
forces F_i = sum_{j,n}' q_i q_j K'(r) d / r (d = r_j + n L - r_i) and the
virial W = -1/2 sum_i sum_{j,n}' q_i q_j K'(r) d d^T / r, with
K(r) = (1 - G_p(r)) / r^p and K'(r) = -G_p'(r) / r^p - p K(r) / r.

Pins: the total-energy pins (Madelung, splitting independence, brute force,
Ewald) of tests/test_oracle_invariants.py; evaluate's energy against
real_energy (an independent loop), its forces against central finite
differences of the energy, its virial against finite differences under
affine strain, its potentials against the quadratic form E = 1/2 sum q phi
and against finite differences in q (tests/test_oracle_realspace.py); in
general cells the rock-salt Madelung energy on the primitive cell,
splitting independence, invariance under a change of lattice basis and the
same derivative checks (tests/test_oracle_triclinic.py).
"""
import numpy as np

from . import cellsum, kernels, reciprocal


def _cell(box):
    """Lattice vectors as the rows of a 3x3 matrix (a length-3 box is the
    orthorhombic cell diag(box))."""
    b = np.asarray(box, dtype=np.float64)
    return np.diag(b) if b.ndim == 1 else b


def _image_range(H, r_c):
    """Image counts per axis that cover every vector of length < r_c once the
    fractional difference is reduced to [-1/2, 1/2]: along a_a the fractional
    component of any vector of length r is at most r / w_a, w_a the cell's
    width across the plane of the other two vectors."""
    V = abs(float(np.linalg.det(H)))
    w = np.array([V / np.linalg.norm(np.cross(H[(a + 1) % 3], H[(a + 2) % 3])) for a in range(3)])
    return np.ceil(r_c / w).astype(int) + 1


def real_energy(pos, q, box, p, c, r_c):
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    H = _cell(box)
    nimg = _image_range(H, r_c)
    n = pos.shape[0]
    E = 0.0
    frac = pos @ np.linalg.inv(H)
    df = frac[:, None, :] - frac[None, :, :]
    df -= np.round(df)                        # nearest image in the cell's basis
    qq = q[:, None] * q[None, :]
    for ix in range(-nimg[0], nimg[0] + 1):
        for iy in range(-nimg[1], nimg[1] + 1):
            for iz in range(-nimg[2], nimg[2] + 1):
                d = (df + np.array([ix, iy, iz], dtype=np.float64)) @ H
                r = np.sqrt(np.sum(d * d, axis=2))
                mask = r < r_c
                if ix == 0 and iy == 0 and iz == 0:
                    mask &= ~np.eye(n, dtype=bool)
                if not np.any(mask):
                    continue
                rr = r[mask]
                E += 0.5 * np.sum(qq[mask] * (1.0 - kernels.mollifier(p, rr, c, r_c)) / rr ** p)
    return E


def evaluate(pos, q, box, ps, c, r_c):
    """All channels of the real-space complement.  q is [C, N]; box is the
    three edges of an orthorhombic cell or a 3x3 matrix whose rows are the
    lattice vectors (the cell tensor of the Fig. 1 caption).

    Returns Ereal [C], phi [C, N], F [N, 3] and W [3, 3] (sums over channels)."""
    pos = np.asarray(pos, dtype=np.float64)
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    H = _cell(box)
    C, n = q.shape
    nimg = _image_range(H, r_c)
    frac = pos @ np.linalg.inv(H)
    df = frac[None, :, :] - frac[:, None, :]   # df[i, j]: fractional r_j - r_i
    df -= np.round(df)
    E = np.zeros(C)
    phi = np.zeros((C, n))
    F = np.zeros((n, 3))
    W = np.zeros((3, 3))
    for ix in range(-nimg[0], nimg[0] + 1):
        for iy in range(-nimg[1], nimg[1] + 1):
            for iz in range(-nimg[2], nimg[2] + 1):
                d = (df + np.array([ix, iy, iz], dtype=np.float64)) @ H
                r = np.sqrt(np.sum(d * d, axis=2))
                mask = (r < r_c) & (r > 0.0)
                if not np.any(mask):
                    continue
                ii, jj = np.nonzero(mask)
                rr = r[mask]
                dd = d[mask]
                for ch in range(C):
                    p = int(ps[ch])
                    K = (1.0 - kernels.mollifier(p, rr, c, r_c)) / rr ** p
                    Kd = -kernels.mollifier_deriv(p, rr, c, r_c) / rr ** p - p * K / rr
                    np.add.at(phi[ch], ii, q[ch, jj] * K)
                    s = q[ch, ii] * q[ch, jj] * Kd / rr
                    np.add.at(F, ii, s[:, None] * dd)
                    W -= 0.5 * np.einsum("k,ka,kb->ab", s, dd, dd)
    for ch in range(C):
        E[ch] = 0.5 * float(np.sum(q[ch] * phi[ch]))
    return {"Ereal": E, "phi": phi, "F": F, "W": W}


def total_energy(pos, q, box, p, c, r_c):
    """E_real + E_k + E_0 - E_self for one channel (Eq. realLR, split).  A
    3x3 cell takes the general-cell Fourier sum."""
    q = np.asarray(q, dtype=np.float64)
    if np.ndim(box) == 2:
        r = cellsum.evaluate(pos, q[None, :], box, [p], c, r_c, sample=[], virial=False)
        ek, e0, es = r["Ek"][0], r["E0"][0], r["Eself"][0]
    else:
        V = float(np.prod(box))
        ek = reciprocal.reciprocal_channel(pos, q, box, p, c, r_c, forces=False,
                                           potential=False, virial=False)["E"]
        e0 = kernels.zero_mode_coefficient(p, c, r_c, V) * float(np.sum(q)) ** 2
        es = kernels.self_coefficient(p, c, r_c) * float(np.sum(q * q))
    return real_energy(pos, q, box, p, c, r_c) + ek + e0 - es
