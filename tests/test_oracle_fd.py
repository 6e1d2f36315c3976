"""Pins for the oracle's finite-difference weights (Section 2.1: Laplacian stencil of order n0)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.fd import second_derivative_weights

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd_weights.txt")


def _golden():
    rows = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            rows[int(parts[0])] = [Fraction(p) for p in parts[1:]]
    return rows


def _vandermonde_weights(r):
    """Solve the moment conditions of a symmetric stencil exactly in rationals.

    sum_{p=-r..r} w_|p| p^(2k) = 2 * delta_{k,1} for k = 0..r  (exact on x^0..x^(2r+1)).
    Independent of the closed form used by the oracle.
    """
    n = r + 1
    a = [[Fraction(0)] * n for _ in range(n)]
    b = [Fraction(0)] * n
    for k in range(n):
        for p in range(n):
            if p == 0:
                a[k][p] = Fraction(1) if k == 0 else Fraction(0)
            else:
                a[k][p] = Fraction(2 * p ** (2 * k))
        b[k] = Fraction(2) if k == 1 else Fraction(0)
    # Gaussian elimination in rationals
    for col in range(n):
        piv = next(i for i in range(col, n) if a[i][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        b[col], b[piv] = b[piv], b[col]
        for i in range(n):
            if i != col and a[i][col] != 0:
                f = a[i][col] / a[col][col]
                a[i] = [x - f * y for x, y in zip(a[i], a[col])]
                b[i] -= f * b[col]
    return [b[i] / a[i][i] for i in range(n)]


def test_matches_textbook_table():
    for order, ref in _golden().items():
        w = second_derivative_weights(order)
        np.testing.assert_allclose(w, [float(x) for x in ref], rtol=1e-15, atol=1e-16)


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6])
def test_matches_rational_moment_solve(r):
    w = second_derivative_weights(2 * r)
    exact = _vandermonde_weights(r)
    np.testing.assert_allclose(w, [float(x) for x in exact], rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("r", [1, 2, 3, 4, 5, 6])
def test_exact_on_polynomials(r):
    """The 2r+1 point stencil differentiates x^q exactly for q <= 2r+1 (at x0 = 0.37, h = 0.21)."""
    w = second_derivative_weights(2 * r)
    x0, h = Fraction(37, 100), Fraction(21, 100)
    wf = [Fraction(v) for v in w]  # exact values of the float weights
    for q in range(0, 2 * r + 2):
        approx = wf[0] * x0 ** q
        for p in range(1, r + 1):
            approx += wf[p] * ((x0 + p * h) ** q + (x0 - p * h) ** q)
        approx /= h * h
        exact = Fraction(q * (q - 1)) * x0 ** (q - 2) if q >= 2 else Fraction(0)
        assert abs(float(approx - exact)) < 1e-9 * max(1.0, abs(float(exact)))


def test_identities_r6():
    w = second_derivative_weights(12)
    r = 6
    assert abs(w[0] + 2 * w[1:].sum()) < 1e-14                       # constants annihilated
    assert abs(2 * sum(p * p * w[p] for p in range(1, r + 1)) - 2.0) < 1e-13  # x^2 -> 2
    # symbol s(theta) = -w0 - 2 sum w_p cos(p theta) approximates theta^2 near 0
    th = 1e-2
    s = -w[0] - 2 * sum(w[p] * np.cos(p * th) for p in range(1, r + 1))
    assert abs(s - th * th) < 1e-12
    # absolute sum used by the Gershgorin bound (value quoted in the design notes)
    assert abs(np.abs(w).sum() + np.abs(w[1:]).sum() - 7.0729) < 1e-4


def test_rejects_odd_order():
    with pytest.raises(ValueError):
        second_derivative_weights(3)
    with pytest.raises(ValueError):
        second_derivative_weights(0)
