"""The library's host-side FP64 math (Nystrom PSWF, closed-form kernels,
FKAD-style piecewise tables, window bandwidth choice), compiled from the
library's sources into a probe with g++, against the FP64 oracle (a
different method: Legendre series)."""
import os
import subprocess

import numpy as np
import pytest

from oracle import kernels as ok
from oracle.pswf import PSWF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_06617_amd", "csrc")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("probe") / "host_math_probe")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "host_math_probe.cpp"),
                    os.path.join(CSRC, "host_math.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe, "12.024"], check=True, capture_output=True, text=True).stdout
    rows = [ln.split() for ln in out.splitlines()]
    return rows


def _get(rows, tag):
    return [list(map(float, r[1:])) for r in rows if r[0] == tag]


def test_prolate_constants(probe):
    ps = PSWF(12.024)
    assert _get(probe, "lam")[0][0] == pytest.approx(ps.lam, rel=1e-13)
    assert _get(probe, "chi")[0][0] == pytest.approx(ps.chi, rel=1e-11)
    assert _get(probe, "C0")[0][0] == pytest.approx(ps.C0, rel=1e-13)
    assert _get(probe, "d4")[0][0] == pytest.approx(ps.deriv_at_zero(4), rel=1e-10)
    assert _get(probe, "d6")[0][0] == pytest.approx(ps.deriv_at_zero(6), rel=1e-9)
    for x, v, d in _get(probe, "psi"):
        assert v == pytest.approx(float(ps(x)), abs=1e-14)
        assert d == pytest.approx(float(ps.d1(x)), abs=1e-10)
    for kap, i0, j1, j3, t3 in _get(probe, "int"):
        assert i0 == pytest.approx(float(ps.I0(kap)), abs=1e-14)
        assert j1 == pytest.approx(float(ps.J1(kap)), abs=1e-14)
        assert j3 == pytest.approx(float(ps.J3(kap)), abs=1e-14)
        assert t3 == pytest.approx(float(ps.T3(kap)), abs=1e-12)


def test_kernels_and_device_tables(probe):
    c, rc = 12.024, 5.0
    for p, s, z, ferr, gerr in _get(probe, "coef"):
        p = int(p)
        assert s == pytest.approx(ok.self_coefficient(p, c, rc), rel=1e-10)
        assert z == pytest.approx(ok.zero_mode_coefficient(p, c, rc, 1.0), rel=1e-9)
        assert ferr < 1e-9 and gerr < 1e-9
    for p, k, phi, dphi, phi_dev, dph_dev in _get(probe, "phi"):
        p = int(p)
        ref = float(ok.phi_hat(p, np.array([k]), c, rc)[0])
        dref = float(ok.phi_hat_deriv(p, np.array([k]), c, rc)[0])
        assert phi == pytest.approx(ref, rel=1e-11, abs=1e-13)
        assert dphi == pytest.approx(dref, rel=1e-9, abs=1e-12)
        # the piecewise-polynomial representation the device evaluates
        assert phi_dev == pytest.approx(ref, rel=1e-8, abs=1e-10)
        assert dph_dev == pytest.approx(dref / k, rel=1e-7, abs=1e-9)


def test_window_table_and_transform(probe):
    w = PSWF(20.0)
    for t, poly, exact in _get(probe, "win"):
        assert exact == pytest.approx(float(w(t)), abs=1e-14)
        assert poly == pytest.approx(float(w(t)), abs=1e-10)
    # transform of the compact window equals lambda psi(s/c) inside the band
    for s, ft, band in _get(probe, "wft"):
        assert ft == pytest.approx(band, rel=1e-12, abs=1e-14)


def test_window_bandwidth_choice_tracks_measured_optimum(probe):
    # measured with the oracle's mesh algorithm on the rock-salt workload:
    # the RMS force error is minimal near c_s = 16.2-16.4 (P = 6) and
    # 20.5-21.0 (P = 8) at eta = 0.54
    assert 15.8 <= _get(probe, "cs6")[0][0] <= 16.8
    assert 20.3 <= _get(probe, "cs8")[0][0] <= 21.5


def test_support_choice_bound_is_conservative_and_tight(probe):
    # the cached bound used to choose P is the estimate at the next grid
    # point of eta (step 1/40): never below the estimate at eta itself, and
    # close to it (the estimate varies smoothly with eta)
    rows = _get(probe, "ebound")
    assert len(rows) == 12
    for P, eta, est, bound in rows:
        assert bound >= est * (1 - 1e-12), (P, eta, est, bound)
        assert bound <= 3.0 * est, (P, eta, est, bound)
    for P in (5, 7, 8):
        b = [r[3] for r in rows if r[0] == P]
        assert all(x < y for x, y in zip(b, b[1:])), (P, b)
