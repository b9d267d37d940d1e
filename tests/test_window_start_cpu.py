"""The binning kernel's window start (FP32 double-word grid coordinate),
compiled for the host with g++ from the library's header, against exact
rational arithmetic: n0 = ceil(u - P/2) mod M and delta = n0 - (u - P/2)
with u = x M / L in an orthorhombic cell, or u = sum_b T_b r_b (T a row of
diag(M) H^-T) in a triclinic one, for positions inside the cell, just
outside it, several cells away and at the edges (x = 0, x just below L)."""
import math
import os
import subprocess
from fractions import Fraction

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_06617_amd", "csrc")


def _cases():
    rng = np.random.default_rng(7)
    out = []
    for L, M, P in [(215.4435, 256, 8), (31.0, 48, 6), (22.56, 32, 6), (10.7, 16, 2), (79.37, 120, 7),
                    (18.0, 36, 8), (5.0, 1024, 5)]:
        xs = list(rng.uniform(0.0, L, 400)) + list(rng.uniform(-3 * L, 4 * L, 200))
        xs += [0.0, L * (1 - 1e-7), -1e-6, L + 1e-5, -L, 2 * L, 1e-30, -1e-30]
        xs += [k * L / M for k in range(0, M, max(1, M // 16))]       # on grid nodes
        xs += [(k + 0.5 * (P % 2)) * L / M for k in range(3)]         # window edge ties
        for x in xs:
            out.append(("O", float(np.float32(x)), L, M, P))
    return out


def _cases_general():
    rng = np.random.default_rng(8)
    out = []
    for H, M, P in [(((215.4435, 0, 0), (40.0, 210.0, 0), (-30.0, 25.0, 205.0)), (256, 256, 256), 8),
                    (((12.0, 0, 0), (3.0, 11.0, 0), (-2.0, 2.5, 10.0)), (24, 24, 24), 6),
                    (((0.0, 11.28, 11.28), (11.28, 0.0, 11.28), (11.28, 11.28, 0.0)), (30, 30, 30), 7)]:
        H = np.array(H, dtype=np.float64)
        T = np.array(M, dtype=np.float64)[:, None] * np.linalg.inv(H).T
        fr = list(rng.uniform(0.0, 1.0, (300, 3))) + list(rng.uniform(-3.0, 4.0, (100, 3)))
        fr += [np.zeros(3), np.full(3, 1 - 1e-7), np.array([0.5, 0.25, 0.75])]
        for f in fr:
            r = (np.asarray(f) @ H).astype(np.float32).astype(np.float64)
            for a in range(3):
                out.append(("G", r, T[a], M[a], P))
    return out


def _run(exe, lines):
    inp = "".join(lines)
    return subprocess.run([exe], input=inp, check=True, capture_output=True, text=True).stdout.split("\n")


def _check(n0, d, s, M, info):
    ne = math.ceil(s)
    de = float(ne - s)
    assert 0 <= n0 < M and 0.0 <= d < 1.0
    if n0 == ne % M:
        err = abs(d - de)
    else:  # the offset sits on a node: either neighbour is the same window to rounding
        assert min(de, 1.0 - de) < 1e-6, (info, n0, d, ne, de)
        err = min(abs(d - (de + 1.0)), abs(d - (de - 1.0)))
    assert err <= 2.4e-7, (info, n0, d, ne, de)
    return err


def _probe(tmp_path):
    exe = str(tmp_path / "window_probe")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "window_probe.cpp"), "-o", exe], check=True)
    return exe


def test_window_start_matches_exact_arithmetic(tmp_path):
    exe = _probe(tmp_path)
    cases = _cases()
    out = _run(exe, ["O %.17g %.17g %d %d\n" % c[1:] for c in cases])
    worst = 0.0
    for (_, x, L, M, P), line in zip(cases, out):
        n0, d = line.split()
        s = Fraction(x) * M / Fraction(L) - Fraction(P, 2)
        worst = max(worst, _check(int(n0), float(d), s, M, (x, L, M, P)))
    assert worst > 0.0 or len(cases) < 10


def test_general_cell_grid_coordinate_matches_exact_arithmetic(tmp_path):
    exe = _probe(tmp_path)
    cases = _cases_general()
    lines = ["G %.17g %.17g %.17g %.17g %.17g %.17g %d %d\n" % (*r, *T, M, P) for _, r, T, M, P in cases]
    out = _run(exe, lines)
    for (_, r, T, M, P), line in zip(cases, out):
        n0, d = line.split()
        # u = T . r with the float-rounded position and the FP64 row of T
        s = sum(Fraction(float(r[b])) * Fraction(float(T[b])) for b in range(3)) - Fraction(P, 2)
        _check(int(n0), float(d), s, M, (tuple(r), tuple(T), M, P))
