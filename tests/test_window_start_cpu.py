"""The binning kernel's window start (FP32 double-word grid coordinate),
compiled for the host with g++ from the library's header, against exact
rational arithmetic: n0 = ceil(x M / L - P/2) mod M and
delta = n0 - (x M / L - P/2), for positions inside the cell, just outside
it, several cells away and at the edges (x = 0, x just below L)."""
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
            out.append((float(np.float32(x)), L, M, P))
    return out


def test_window_start_matches_exact_arithmetic(tmp_path):
    exe = str(tmp_path / "window_probe")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC,
                    os.path.join(ROOT, "tests", "native", "window_probe.cpp"), "-o", exe], check=True)
    cases = _cases()
    inp = "".join("%.17g %.17g %d %d\n" % c for c in cases)
    out = subprocess.run([exe], input=inp, check=True, capture_output=True, text=True).stdout.split("\n")
    worst = 0.0
    for (x, L, M, P), line in zip(cases, out):
        n0, d = line.split()
        n0, d = int(n0), float(d)
        s = Fraction(x) * M / Fraction(L) - Fraction(P, 2)
        ne = math.ceil(s)
        de = float(ne - s)
        assert 0 <= n0 < M and 0.0 <= d < 1.0
        if n0 == ne % M:
            err = abs(d - de)
        else:  # the offset sits on a node: either neighbour is the same window to rounding
            assert min(de, 1.0 - de) < 1e-6, (x, L, M, P, n0, d, ne, de)
            err = min(abs(d - (de + 1.0)), abs(d - (de - 1.0)))
        worst = max(worst, err)
        assert err <= 2.4e-7, (x, L, M, P, n0, d, ne, de)
    assert worst > 0.0 or len(cases) < 10
