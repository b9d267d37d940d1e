"""Textbook Ewald summation for p = 1, FP64 (independent cross-check only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The Gaussian screening of Eq. screening with p = 1, G_1^Ewald = erfc(alpha r):
  E = 1/2 sum_n sum'_{ij} q_i q_j erfc(alpha r)/r
      + (2 pi / V) sum_{k != 0} exp(-k^2 / 4 alpha^2) / k^2 |S(k)|^2
      - (alpha / sqrt(pi)) sum_i q_i^2 - pi Q^2 / (2 V alpha^2).
Shares nothing with the PSWF kernels; it pins the PSWF p = 1 total.
"""
import numpy as np
from scipy.special import erfc


def ewald_energy(pos, q, box, alpha, r_cut, k_cut):
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    n = pos.shape[0]
    d0 = pos[:, None, :] - pos[None, :, :]
    d0 -= box * np.round(d0 / box)
    qq = q[:, None] * q[None, :]
    nimg = np.ceil(r_cut / box).astype(int) + 1
    er = 0.0
    for ix in range(-nimg[0], nimg[0] + 1):
        for iy in range(-nimg[1], nimg[1] + 1):
            for iz in range(-nimg[2], nimg[2] + 1):
                d = d0 + np.array([ix, iy, iz]) * box
                r = np.sqrt(np.sum(d * d, axis=2))
                mask = r < r_cut
                if ix == 0 and iy == 0 and iz == 0:
                    mask &= ~np.eye(n, dtype=bool)
                er += 0.5 * np.sum(qq[mask] * erfc(alpha * r[mask]) / r[mask])
    mmax = np.floor(k_cut * box / (2 * np.pi)).astype(int)
    ek = 0.0
    for mx in range(-mmax[0], mmax[0] + 1):
        kx = 2 * np.pi * mx / box[0]
        my, mz = np.meshgrid(np.arange(-mmax[1], mmax[1] + 1),
                             np.arange(-mmax[2], mmax[2] + 1), indexing="ij")
        ky = 2 * np.pi * my.ravel() / box[1]
        kz = 2 * np.pi * mz.ravel() / box[2]
        k2 = kx * kx + ky * ky + kz * kz
        keep = (k2 > 0) & (k2 <= k_cut * k_cut)
        kv = np.stack([np.full(keep.sum(), kx), ky[keep], kz[keep]], axis=1)
        S = q @ np.exp(1j * (pos @ kv.T))
        ek += (2 * np.pi / V) * np.sum(np.exp(-k2[keep] / (4 * alpha ** 2)) / k2[keep]
                                       * np.abs(S) ** 2)
    es = alpha / np.sqrt(np.pi) * np.sum(q * q)
    Q = np.sum(q)
    return er + ek - es - np.pi * Q * Q / (2 * V * alpha ** 2)
