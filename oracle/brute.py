"""Brute-force periodic image sums of 1/r^p for p > 3, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Eq. realLR with G_p = 1 summed directly over all image pairs with
|r_ij + n L| <= R, plus the continuum tail of the uniform average density
beyond R:  (2 pi Q^2 / V) R^(3 - p) / (p - 3).  Absolutely convergent for
p > 3; the sharp spherical cut leaves a lattice-count error ~ R^(1.5 - p),
so this is used for p = 4, 5, 6 on tiny cells only.
"""
import numpy as np


def image_sum(pos, q, box, p, R):
    pos = np.asarray(pos, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    box = np.asarray(box, dtype=np.float64)
    V = float(np.prod(box))
    n = pos.shape[0]
    d0 = pos[:, None, :] - pos[None, :, :]
    qq = (q[:, None] * q[None, :]).ravel()
    nim = np.ceil(R / box).astype(int) + 1
    E = 0.0
    ix = np.arange(-nim[0], nim[0] + 1)
    iy = np.arange(-nim[1], nim[1] + 1)
    for a in ix:
        gy, gz = np.meshgrid(iy, np.arange(-nim[2], nim[2] + 1), indexing="ij")
        sh = np.stack([np.full(gy.size, a), gy.ravel(), gz.ravel()], axis=1) * box
        d = d0.reshape(1, n * n, 3) + sh[:, None, :]
        r = np.sqrt(np.sum(d * d, axis=2))
        mask = (r <= R) & (r > 0.0)
        E += 0.5 * np.sum((qq[None, :] / np.where(mask, r, 1.0) ** p) * mask)
    Q = np.sum(q)
    return E + 2.0 * np.pi * Q * Q / V * R ** (3 - p) / (p - 3)
