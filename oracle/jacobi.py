"""Jacobi polynomials and Gauss-Jacobi rules, written out plainly (FP64).

Test infrastructure only (see the package header).

P_n^{(a,b)} is evaluated by the standard three-term recurrence; its
derivative uses d/dx P_n^{(a,b)} = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}.
Gauss-Jacobi nodes and weights for the weight (1-x)^a (1+x)^b on [-1,1]
come from the Golub-Welsch eigenvalue method on the monic recurrence.
The paper builds its shape functions from these polynomials
(Section 3.1, eq. phi2D, and Section 4.2.2).
"""
from __future__ import annotations

import math

import numpy as np


def jacobi(n: int, a: float, b: float, x):
    """P_n^{(a,b)}(x) for array x, by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    if n < 0:
        return np.zeros_like(x)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = 0.5 * ((a + b + 2.0) * x + (a - b))
    for m in range(2, n + 1):
        c = 2.0 * m + a + b
        a1 = 2.0 * m * (m + a + b) * (c - 2.0)
        a2 = (c - 1.0) * (a * a - b * b)
        a3 = (c - 2.0) * (c - 1.0) * c
        a4 = 2.0 * (m + a - 1.0) * (m + b - 1.0) * c
        p0, p1 = p1, ((a2 + a3 * x) * p1 - a4 * p0) / a1
    return p1


def djacobi(n: int, a: float, b: float, x):
    """d/dx P_n^{(a,b)}(x)."""
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return 0.5 * (n + a + b + 1.0) * jacobi(n - 1, a + 1.0, b + 1.0, x)


def gauss_jacobi(q: int, a: float, b: float):
    """q-point Gauss rule for int_{-1}^{1} (1-x)^a (1+x)^b f(x) dx (exact to degree 2q-1)."""
    alpha = np.empty(q)
    beta = np.empty(max(q - 1, 0))
    for k in range(q):
        c = 2.0 * k + a + b
        if k == 0:
            alpha[k] = (b - a) / (a + b + 2.0)
        else:
            alpha[k] = (b * b - a * a) / (c * (c + 2.0))
    for k in range(1, q):
        c = 2.0 * k + a + b
        num = 4.0 * k * (k + a) * (k + b) * (k + a + b)
        den = c * c * (c + 1.0) * (c - 1.0)
        beta[k - 1] = num / den
    T = np.diag(alpha) + np.diag(np.sqrt(beta), 1) + np.diag(np.sqrt(beta), -1)
    x, V = np.linalg.eigh(T)
    mu0 = 2.0 ** (a + b + 1.0) * math.gamma(a + 1.0) * math.gamma(b + 1.0) / math.gamma(a + b + 2.0)
    w = mu0 * V[0, :] ** 2
    return x, w
