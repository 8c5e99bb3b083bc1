"""Exact rational arithmetic for tiny systems (test helper): Gaussian elimination over
Python Fractions, so the result is the exact solution of the stored double-precision system."""
from fractions import Fraction

import numpy as np


def exact_solve(A: np.ndarray, b: np.ndarray):
    """Exact solution of A x = b (A dense, nonsingular, small) as a list of Fractions."""
    n = len(b)
    M = [[Fraction(float(A[i, j])) for j in range(n)] + [Fraction(float(b[i]))] for i in range(n)]
    for k in range(n):
        piv = max(range(k, n), key=lambda i: abs(M[i][k]))
        if M[piv][k] == 0:
            raise ZeroDivisionError("singular")
        M[k], M[piv] = M[piv], M[k]
        for i in range(k + 1, n):
            if M[i][k] != 0:
                f = M[i][k] / M[k][k]
                for j in range(k, n + 1):
                    M[i][j] -= f * M[k][j]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n] - sum(M[i][j] * x[j] for j in range(i + 1, n))
        x[i] = s / M[i][i]
    return x


def exact_residual(rowptr, colidx, values, x, b):
    """rho = b - K x exactly, as Fractions."""
    out = []
    for i in range(len(b)):
        s = Fraction(float(b[i]))
        for p in range(rowptr[i], rowptr[i + 1]):
            s -= Fraction(float(values[p])) * Fraction(float(x[colidx[p]]))
        out.append(s)
    return out


def max_componentwise_error(x: np.ndarray, xe) -> float:
    """max_i |x_i - xe_i| / |xe_i| over the nonzero exact components."""
    return float(max(abs(Fraction(float(x[i])) - xe[i]) / abs(xe[i]) for i in range(len(xe)) if xe[i] != 0))
