"""Closed forms used as pins.  Nothing here is imported from the oracle or
from the GPU library; every formula is derived independently of both."""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fd8_weights_from_moments() -> list:
    """Solve for c_0..c_4 so that (1/h^2) sum_m c_|m| f(x+mh) is exact for
    polynomials of degree <= 9: symmetric weights kill odd degrees, and the
    even moments must satisfy sum_m c_|m| m^(2j) = (2j)! [j == 1], j=0..4.
    Exact rational Gaussian elimination."""
    n = 5
    A = []
    for j in range(n):
        row = []
        for m in range(n):
            if j == 0:
                row.append(Fraction(1 if m == 0 else 2))
            else:
                row.append(Fraction(0 if m == 0 else 2 * m ** (2 * j)))
        A.append(row)
    b = [Fraction(0), Fraction(2), Fraction(0), Fraction(0), Fraction(0)]
    # Gaussian elimination
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        b[col], b[piv] = b[piv], b[col]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col] / A[col][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
                b[r] = b[r] - f * b[col]
    return [b[i] / A[i][i] for i in range(n)]


def fd8_weights_golden() -> list:
    w = {}
    with open(os.path.join(GOLDEN, "fd8_weights.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            m, num, den = (int(t) for t in line.split())
            w[m] = Fraction(num, den)
    return [w[m] for m in range(5)]


def positions(ijk: np.ndarray, dims, h: float) -> np.ndarray:
    """x_a = h (i_a - (n_a - 1)/2): the box is symmetric about the origin."""
    return h * (ijk.astype(np.float64) - 0.5 * (np.asarray(dims, dtype=np.float64) - 1.0))


def plane_wave_eigenvalue(k, h: float, kin: float = -0.5) -> float:
    """Symbol of kin * (8th-order star Laplacian) on exp(i k.r)."""
    c = [float(x) for x in fd8_weights_from_moments()]
    s = 0.0
    for ka in k:
        s += c[0] + 2.0 * sum(c[m] * math.cos(m * ka * h) for m in range(1, 5))
    return kin * s / (h * h)


def ho_rayleigh_closed_form(h: float) -> float:
    """Rayleigh quotient of the sampled Gaussian exp(-r^2/2) for
    H = -1/2 Lap_h + r^2/2 on an infinite grid (aliasing ~ exp(-pi^2/h^2)
    neglected).  Per axis, sum_x g(x) g(x+mh) / sum_x g(x)^2 =
    exp(-m^2 h^2 / 4), and sum_x x^2 g^2 / sum g^2 = 1/2, so
    E = 3/4 - (3 / (2 h^2)) [c0 + 2 sum_m c_m exp(-m^2 h^2 / 4)]."""
    c = [float(x) for x in fd8_weights_from_moments()]
    s = c[0] + 2.0 * sum(c[m] * math.exp(-m * m * h * h / 4.0) for m in range(1, 5))
    return 0.75 - 1.5 * s / (h * h)


def taylor4_scalar(z: complex | np.ndarray):
    """sum_{k=0}^{4} z^k / k! by the power series (Horner in z)."""
    return 1 + z * (1 + z / 2 * (1 + z / 3 * (1 + z / 4)))


def interior_mask(ijk: np.ndarray, dims, depth: int) -> np.ndarray:
    d = np.asarray(dims)
    return np.all((ijk >= depth) & (ijk < d - depth), axis=1)
