"""Pins for the oracle's sixth-order staggered flux difference, Section 2.2,
Eq. (2), on the CPU.

* The printed weights (golden fixture) have the moment sums of a staggered
  first derivative exact to degree 6: sum c_m (2m-1) = 1, sum c_m (2m-1)^3 = 0,
  sum c_m (2m-1)^5 = 0 (exact rationals), and sum c_m (2m-1)^7 = 225.
* The operator differentiates polynomials up to degree 6 exactly (to
  rounding), along each axis, for any grid size and origin.
* On xi^7 the error at xi = 0 is the closed form 2 h^6 / 2^7 * 225 = 225/64 h^6.
* On a sine the error falls as h^6.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import highorder as ho

HERE = os.path.dirname(os.path.abspath(__file__))


def _weights():
    out = {}
    for line in open(os.path.join(HERE, "golden", "wcns_e5_weights.txt")):
        line = line.strip()
        if line and not line.startswith("#"):
            k, a, b = line.split()
            out[k] = Fraction(int(a), int(b))
    return [out["c1"], out["c2"], out["c3"]]


def test_printed_weights_moments():
    c = _weights()
    mom = [sum(cm * (2 * m + 1) ** p for m, cm in enumerate(c)) for p in (1, 3, 5, 7)]
    assert mom == [1, 0, 0, 225]
    assert [float(x) for x in c] == [ho.C1, ho.C2, ho.C3]


def _faces_along(d, n, other, x0, h, fn, nvar=2):
    """Face field of fn(xi) along axis d (faces at x0 + (i - 1/2) h, i = -2 .. n+2)."""
    xf = x0 + (np.arange(-2, n + 3) - 0.5) * h
    shape = [nvar, other[2], other[1], other[0]]
    shape[3 - d] = n + 5
    vals = fn(xf)
    sh = [1, 1, 1, 1]
    sh[3 - d] = n + 5
    base = np.broadcast_to(vals.reshape(sh), shape)
    scale = np.arange(1, nvar + 1, dtype=float).reshape(nvar, 1, 1, 1)
    return np.ascontiguousarray(base * scale), scale


@pytest.mark.parametrize("d", [0, 1, 2])
@pytest.mark.parametrize("p", [0, 1, 2, 3, 4, 5, 6])
def test_exact_on_polynomials(d, p):
    rng = np.random.default_rng(10 * d + p)
    h = float(rng.uniform(0.05, 0.3))
    x0 = float(rng.uniform(-1, 1))
    n = 11
    f, scale = _faces_along(d, n, (4, 3, 2), x0, h, lambda x: x ** p)
    got = ho.staggered_diff6(f, d, h)
    xc = x0 + np.arange(n) * h
    want = p * xc ** (p - 1) if p > 0 else 0.0 * xc
    sh = [1, 1, 1, 1]
    sh[3 - d] = n
    want = want.reshape(sh) * scale
    tol = 1e-11 * max(1.0, np.max(np.abs(xc)) ** max(p - 1, 0) * p)
    assert np.max(np.abs(got - want)) <= tol


def test_degree_seven_error_closed_form():
    for h in (0.1, 0.25, 0.5):
        f, _ = _faces_along(0, 1, (1, 1, 1), 0.0, h, lambda x: x ** 7, nvar=1)
        got = ho.staggered_diff6(f, 0, h)[0, 0, 0, 0]
        assert got == pytest.approx(225.0 / 64.0 * h ** 6, rel=1e-12)


def test_sixth_order_convergence():
    errs = []
    for n in (16, 32, 64):
        h = 2 * np.pi / n
        f, _ = _faces_along(2, n, (1, 1, 1), 0.3, h, np.sin, nvar=1)
        got = ho.staggered_diff6(f, 2, h)[0, :, 0, 0]
        errs.append(np.max(np.abs(got - np.cos(0.3 + np.arange(n) * h))))
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 5.8
