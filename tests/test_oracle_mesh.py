"""Pins for oracle.mesh (the paper's four-step mesh algorithm in plain form).

The mesh energy and forces converge spectrally to the plain Fourier sum of
oracle.reciprocal as the window support P grows; the mesh forces are the
exact negative gradient of the mesh energy; the spread grid's transform
reproduces What(k) conj(S(k)) / h^3 at low k (Poisson summation)."""
import numpy as np
import pytest

from oracle import mesh, reciprocal
from paper_2606_06617_amd import workloads as wl

C, RC = 12.024, 5.0


def _errs(res, ref):
    eE = abs(res["Ek"].sum() - ref["Ek"].sum()) / abs(ref["Ek"].sum())
    eF = np.sqrt(np.mean(np.sum((res["F"] - ref["F"]) ** 2, 1))) / np.sqrt(
        np.mean(np.sum(ref["F"] ** 2, 1)))
    return eE, eF


def test_spectral_convergence_in_support():
    w = wl.nacl()
    pos = w["pos"].astype(np.float64)
    q = w["q"].astype(np.float64)
    ref = reciprocal.evaluate(pos, q, w["box"], w["ps"], C, RC)
    e6 = _errs(mesh.evaluate(pos, q, w["box"], w["ps"], C, RC, (32,) * 3, 6, 16.4), ref)
    e8 = _errs(mesh.evaluate(pos, q, w["box"], w["ps"], C, RC, (32,) * 3, 8, 21.0), ref)
    assert e6[0] < 1e-5 and e6[1] < 1e-4
    assert e8[0] < 1e-7 and e8[1] < 2e-6
    assert e8[1] < e6[1] / 20


def test_mesh_two_channel_water_small_grid():
    w = wl.water(nmol=60, L=12.0)
    pos = w["pos"].astype(np.float64)
    q = w["q"].astype(np.float64)
    ref = reciprocal.evaluate(pos, q, w["box"], w["ps"], C, RC)
    res = mesh.evaluate(pos, q, w["box"], w["ps"], C, RC, (20, 20, 20), 8, 21.0)
    eE, eF = _errs(res, ref)
    assert eE < 1e-6 and eF < 1e-5
    assert np.allclose(res["E0"], ref["E0"]) and np.allclose(res["Eself"], ref["Eself"])
    wr = np.abs(res["W"] - ref["W"]).max() / np.abs(ref["W"]).max()
    assert wr < 1e-5
    pr = np.abs(res["phi"] - ref["phi"]).max() / np.abs(ref["phi"]).max()
    assert pr < 1e-5


def test_mesh_forces_are_exact_gradient_of_mesh_energy():
    w = wl.random_box(40, ps=(1,), seed=11)
    pos = w["pos"].astype(np.float64)
    q = w["q"].astype(np.float64)
    M, P, cs = (16, 16, 16), 6, 16.4
    res = mesh.evaluate(pos, q, w["box"], w["ps"], C, RC, M, P, cs)
    h = 1e-6

    def e(pp):
        return mesh.evaluate(pp, q, w["box"], w["ps"], C, RC, M, P, cs)["Ek"][0]
    for i in (0, 17):
        for a in range(3):
            pp = pos.copy()
            pm = pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            fd = -(e(pp) - e(pm)) / (2 * h)
            assert res["F"][i, a] == pytest.approx(fd, rel=1e-5, abs=1e-8)


def test_spread_grid_transform_poisson_summation():
    w = wl.random_box(30, ps=(1,), seed=12)
    pos = w["pos"].astype(np.float64)
    q = w["q"][0].astype(np.float64)
    box = w["box"]
    M, P, cs = (24, 24, 24), 8, 21.0
    g = mesh.spread(pos, q, box, M, P, cs)
    F = np.fft.fftn(g)
    h = box / np.array(M)
    ws = mesh.window_pswf(cs)
    for m in [(1, 0, 0), (0, 2, 1), (3, -2, 2), (-1, 1, 4)]:
        k = 2 * np.pi * np.array(m) / box
        S = np.sum(q * np.exp(1j * pos @ k))
        what = np.prod([0.5 * P * h[a] * ws.lam * ws(0.5 * P * h[a] * k[a] / cs) for a in range(3)])
        lhs = np.prod(h) * F[m[0] % M[0], m[1] % M[1], m[2] % M[2]]
        assert abs(lhs - what * np.conj(S)) < 1e-6 * abs(what) * np.sqrt(np.sum(q * q))
