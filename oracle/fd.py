"""Central finite-difference weights for the second derivative (oracle; test infrastructure only).

The paper discretises the Laplacian with a finite-difference stencil of order
n0 (Section 2.1, first bullet: 3*n0 + 1 operations per output point of the 3-D
stencil).  For an even order n0 = 2r the standard central approximation is

    f''(x) ~ (1/h^2) * sum_{p=-r..r} w_|p| f(x + p h)

with the closed-form weights (the limit of Lagrange interpolation on 2r+1
equispaced nodes)

    w_0 = -2 * sum_{p=1..r} 1/p^2
    w_p = 2 (-1)^(p+1) (r!)^2 / (p^2 (r-p)! (r+p)!)      p = 1..r.
"""
from __future__ import annotations

import math

import numpy as np


def second_derivative_weights(order: int) -> np.ndarray:
    """Return w_0..w_r (float64) for the central second-derivative stencil of even ``order`` = 2r."""
    if order < 2 or order % 2:
        raise ValueError("finite-difference order must be even and >= 2")
    r = order // 2
    w = np.zeros(r + 1)
    w[0] = -2.0 * sum(1.0 / (p * p) for p in range(1, r + 1))
    for p in range(1, r + 1):
        num = 2.0 * (-1.0) ** (p + 1) * math.factorial(r) ** 2
        den = p * p * math.factorial(r - p) * math.factorial(r + p)
        w[p] = num / den
    return w
