"""Seeded synthetic workloads (positions, per-channel charges, boxes).

This module holds input generation only -- no part of the method's
arithmetic -- so that the HIP path and the FP64 oracle receive the same
bits.  Every generator works in FP64 from numpy's PCG64 with a fixed seed
and rounds positions and charges to FP32 at the end; consumers convert the
FP32 values exactly to FP64 where they need it.

Workloads (stand-ins for the paper's runtime benchmark systems, which are
not available: a rock-salt crystal, a water model and an electrolyte, all
at fixed number density and replicated to large sizes):

  nacl_512       rock-salt NaCl, 4x4x4 conventional cells, a = 5.64 A,
                 charges +-1, Gaussian jitter 0.1 A; channel p = 1; grid 32^3,
                 window support P = 6.
  water_3000     1000 rigid 3-site molecules (O -0.8476 e, H +0.4238 e,
                 O-H 1.0 A, HOH 109.47 deg) at uniform random positions and
                 Haar-random orientations in a 31 A cube; channels p = 1
                 (charges) and p = 6 (sqrt of a per-species C6 coefficient,
                 geometric mixing: 5.0 for O, sqrt(2) for H); grid 48^3.
  ionic_1m       N = 1e6 atoms uniform in a cube at 0.1 atoms/A^3
                 (L = 215.44 A); 4 latent charge sets x p in {1, 3, 6}
                 = 12 channels, q ~ N(0, 0.5) mean-subtracted per channel;
                 grid 256^3, P = 8.
  diff_batch     64 structures, N ~ U{200..4000}, density 0.1, p in {1, 6}
                 neutralised N(0, 0.5) charges; grid = smallest 2^a 3^b
                 >= L / 0.535 A clamped to [24, 64].
  serving_stream Poisson arrivals, N log-uniform in [100, 50000], density
                 0.1, p in {1, 6} neutralised N(0, 0.5).
  nacl_primitive rock salt on its face-centred primitive (triclinic) cell.
  triclinic_box  uniform random positions in a skewed cell.
"""
import math

import numpy as np

DENSITY = 0.1


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _finish(pos, q, box, ps, grid, support, name):
    box = np.asarray(box, dtype=np.float64)
    pos = np.mod(np.asarray(pos, dtype=np.float64), box)
    pos32 = pos.astype(np.float32)
    # rounding can land exactly on L; keep the stored bits inside [0, L)
    pos32 = np.where(pos32.astype(np.float64) >= box, np.float32(0.0), pos32)
    return {
        "name": name,
        "pos": np.ascontiguousarray(pos32),
        "q": np.ascontiguousarray(np.atleast_2d(np.asarray(q, dtype=np.float32))),
        "box": box,
        "ps": list(int(p) for p in ps),
        "grid": tuple(int(g) for g in grid) if grid is not None else None,
        "support": support,
    }


def nacl(ncell=4, a=5.64, jitter=0.1, seed=1):
    """Rock-salt NaCl.  jitter = 0 gives the perfect lattice (Madelung case)."""
    rng = _rng(seed)
    fcc = np.array([[0, 0, 0], [0, .5, .5], [.5, 0, .5], [.5, .5, 0]], dtype=np.float64)
    cells = np.array([[i, j, k] for i in range(ncell) for j in range(ncell)
                      for k in range(ncell)], dtype=np.float64)
    na = (cells[:, None, :] + fcc[None, :, :]).reshape(-1, 3) * a
    cl = na + np.array([a / 2, 0.0, 0.0])
    pos = np.empty((2 * na.shape[0], 3))
    pos[0::2] = na
    pos[1::2] = cl
    q = np.empty(pos.shape[0])
    q[0::2] = 1.0
    q[1::2] = -1.0
    if jitter > 0:
        pos = pos + rng.normal(0.0, jitter, pos.shape)
    L = ncell * a
    return _finish(pos, q[None, :], [L, L, L], [1], (32, 32, 32), 6,
                   "nacl_%d" % pos.shape[0])


def _finish_cell(pos, q, cell, ps, grid, support, name):
    """As _finish for a general cell (lattice vectors as the rows of `cell`):
    positions are wrapped into the parallelepiped through their fractional
    coordinates; "box" holds the 3x3 cell."""
    cell = np.asarray(cell, dtype=np.float64)
    frac = np.asarray(pos, dtype=np.float64) @ np.linalg.inv(cell)
    frac -= np.floor(frac)
    frac = np.where(frac >= 1.0, 0.0, frac)
    out = _finish(frac @ cell, q, [np.inf] * 3, ps, grid, support, name)
    out["box"] = cell
    return out


def nacl_primitive(ncell=4, a=5.64, jitter=0.0, seed=7):
    """Rock salt on its face-centred primitive cell (a triclinic description
    of the same crystal): lattice vectors a/2 (0,1,1), a/2 (1,0,1),
    a/2 (1,1,0), one Na+ at each lattice point and one Cl- displaced by
    (a/2, 0, 0); ncell^3 primitive cells (2 ncell^3 ions)."""
    rng = _rng(seed)
    prim = 0.5 * a * np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    idx = np.array([[i, j, k] for i in range(ncell) for j in range(ncell)
                    for k in range(ncell)], dtype=np.float64)
    na = idx @ prim
    cl = na + np.array([a / 2, 0.0, 0.0])
    pos = np.empty((2 * na.shape[0], 3))
    pos[0::2] = na
    pos[1::2] = cl
    q = np.empty(pos.shape[0])
    q[0::2] = 1.0
    q[1::2] = -1.0
    if jitter > 0:
        pos = pos + rng.normal(0.0, jitter, pos.shape)
    return _finish_cell(pos, q[None, :], ncell * prim, [1], None, None, "nacl_prim_%d" % pos.shape[0])


# a skewed cell shape (rows: lattice vectors before scaling); every angle
# between lattice vectors differs from 90 degrees
TRICLINIC_SHAPE = ((1.0, 0.0, 0.0), (0.31, 0.95, 0.0), (-0.22, 0.27, 0.93))


def triclinic_box(n, ps=(1, 6), seed=8, density=DENSITY, shape=TRICLINIC_SHAPE, neutral=True):
    """Uniform random positions in a triclinic cell of the given shape scaled
    to the density; charges N(0, 0.5), neutralised per channel if asked."""
    rng = _rng(seed)
    shape = np.asarray(shape, dtype=np.float64)
    s = (n / density / abs(np.linalg.det(shape))) ** (1.0 / 3.0)
    cell = shape * s
    pos = rng.uniform(0.0, 1.0, size=(n, 3)) @ cell
    if neutral:
        q = _neutral_charges(rng, len(ps), n)
    else:
        q = rng.normal(0.0, 0.5, size=(len(ps), n))
    return _finish_cell(pos, q, cell, list(ps), None, None, "triclinic_%d" % n)


def _random_rotations(rng, n):
    qv = rng.normal(size=(n, 4))
    qv /= np.linalg.norm(qv, axis=1, keepdims=True)
    w, x, y, z = qv.T
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)], -1),
        np.stack([2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)], -1),
        np.stack([2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], -1),
    ], axis=1)


def water(nmol=1000, L=31.0, seed=2):
    rng = _rng(seed)
    ang = math.radians(109.47)
    local = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0],
                      [math.cos(ang), math.sin(ang), 0.0]])
    rot = _random_rotations(rng, nmol)
    centre = rng.uniform(0.0, L, size=(nmol, 3))
    pos = centre[:, None, :] + np.einsum("nij,sj->nsi", rot, local)
    pos = pos.reshape(-1, 3)
    qc = np.tile(np.array([-0.8476, 0.4238, 0.4238]), nmol)
    q6 = np.tile(np.array([5.0, math.sqrt(2.0), math.sqrt(2.0)]), nmol)
    return _finish(pos, np.stack([qc, q6]), [L, L, L], [1, 6], (48, 48, 48), 8,
                   "water_%d" % pos.shape[0])


def _neutral_charges(rng, nchan, n, sigma=0.5):
    q = rng.normal(0.0, sigma, size=(nchan, n))
    return q - q.mean(axis=1, keepdims=True) if n > 0 else q


def ionic(n=1_000_000, nlatent=4, ps=(1, 3, 6), grid=256, support=8, seed=3):
    rng = _rng(seed)
    L = (n / DENSITY) ** (1.0 / 3.0)
    pos = rng.uniform(0.0, L, size=(n, 3))
    q = _neutral_charges(rng, nlatent * len(ps), n)
    chan_p = [p for _ in range(nlatent) for p in ps]
    return _finish(pos, q, [L, L, L], chan_p, (grid, grid, grid), support,
                   "ionic_%d" % n)


def smooth_size(x, lo=None, hi=None, primes=(2, 3), even=True):
    """Smallest integer >= x whose prime factors are all in `primes` (and
    even if asked: the z axis of the real-to-complex transform needs it)."""
    m = max(1, int(math.ceil(x - 1e-9)))
    while True:
        r = m
        for pr in primes:
            while r % pr == 0:
                r //= pr
        if r == 1 and (m % 2 == 0 or not even):
            break
        m += 1
    if lo is not None:
        m = max(m, lo)
    if hi is not None:
        m = min(m, hi)
    return m


def diff_batch(nstruct=64, seed=4, nmin=200, nmax=4000):
    rng = _rng(seed)
    out = []
    for i in range(nstruct):
        n = int(rng.integers(nmin, nmax + 1))
        L = (n / DENSITY) ** (1.0 / 3.0)
        pos = rng.uniform(0.0, L, size=(n, 3))
        q = _neutral_charges(rng, 2, n)
        m = smooth_size(L / 0.535, lo=24, hi=64)
        out.append(_finish(pos, q, [L, L, L], [1, 6], (m, m, m), None,
                           "batch%02d_%d" % (i, n)))
    return out


def random_box(n, ps=(1, 6), seed=5, density=DENSITY, aspect=(1.0, 1.0, 1.0),
               neutral=True):
    """One uniform random structure at the given density (serving requests,
    parity cases).  Charges N(0, 0.5), neutralised per channel if asked."""
    rng = _rng(seed)
    vol = n / density
    s = (vol / float(np.prod(aspect))) ** (1.0 / 3.0)
    box = np.array(aspect, dtype=np.float64) * s
    pos = rng.uniform(0.0, 1.0, size=(n, 3)) * box
    if neutral:
        q = _neutral_charges(rng, len(ps), n)
    else:
        q = rng.normal(0.0, 0.5, size=(len(ps), n))
    return _finish(pos, q, box, list(ps), None, None, "random_%d" % n)


def serving_stream(nreq=2000, rate=1.0, seed=6, nmin=100, nmax=50_000):
    """Poisson arrival times (s) and request sizes; structures are built lazily
    with random_box(n, seed=request seed)."""
    rng = _rng(seed)
    gaps = rng.exponential(1.0 / rate, size=nreq)
    t = np.cumsum(gaps)
    sizes = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=nreq))).astype(int)
    seeds = rng.integers(1, 2 ** 31 - 1, size=nreq)
    return [{"t": float(t[i]), "n": int(sizes[i]), "seed": int(seeds[i])} for i in range(nreq)]
