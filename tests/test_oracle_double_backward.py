"""Pins of oracle.reciprocal.force_vjp (the derivatives of a force-matching
loss L = sum_i v_i . F_i): central finite differences of L computed from
the oracle's forces (an independent formula), in charges and positions, on
a charged box with two exponents."""
import numpy as np
import pytest

from oracle import reciprocal

C, RC = 12.024, 5.0


def _system():
    rng = np.random.default_rng(17)
    box = np.array([9.0, 10.0, 8.0])
    n = 20
    pos = rng.uniform(0.0, 1.0, (n, 3)) * box
    q = rng.normal(0.0, 0.5, (2, n))
    v = rng.normal(0.0, 1.0, (n, 3))
    return pos, q, box, (1, 6), v


def _loss(pos, q, box, ps, v):
    F = reciprocal.evaluate(pos, q, box, ps, C, RC, potential=False, virial=False)["F"]
    return float(np.sum(v * F))


def test_charge_derivative():
    pos, q, box, ps, v = _system()
    dq, _ = reciprocal.force_vjp(pos, q, box, ps, C, RC, v)
    h = 1e-6
    for ch, j in ((0, 3), (1, 7), (0, 19)):
        qp, qm = q.copy(), q.copy()
        qp[ch, j] += h
        qm[ch, j] -= h
        fd = (_loss(pos, qp, box, ps, v) - _loss(pos, qm, box, ps, v)) / (2 * h)
        assert dq[ch, j] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_position_derivative():
    pos, q, box, ps, v = _system()
    _, dr = reciprocal.force_vjp(pos, q, box, ps, C, RC, v)
    h = 1e-6
    for j in (0, 11):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[j, a] += h
            pm[j, a] -= h
            fd = (_loss(pp, q, box, ps, v) - _loss(pm, q, box, ps, v)) / (2 * h)
            assert dr[j, a] == pytest.approx(fd, rel=1e-5, abs=1e-8)
