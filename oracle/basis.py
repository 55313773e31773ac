"""The L2-orthonormal Dubiner basis on the reference tetrahedron (FP64).

Test infrastructure only (see the package header).

Reference tetrahedron: x, y, z >= 0, x + y + z <= 1 (Section 4.2.2).
Shape functions (Section 4.2.2, with the index roles i <-> z, j <-> y, k <-> x):

    phi_ijk = (1-x-y)^i (1-x)^j P_i(2z/(1-x-y) - 1)
              * P_j^{(2i+1,0)}(2y/(1-x) - 1) * P_k^{(2i+2j+2,0)}(2x - 1),

multiplied by sqrt((2i+1)(2i+2j+2)(2i+2j+2k+3)) so that the functions are
orthonormal; the paper uses orthonormality (Section 3.3.1) while printing
the unnormalised form.  Gradients follow from the chain rule in the
collapsed coordinates a = 2x-1, b = 2y/(1-x)-1, c = 2z/(1-x-y)-1 (all
quadrature points used here are interior, so no singular factor appears).
"""
from __future__ import annotations

import numpy as np

from .jacobi import djacobi, gauss_jacobi, jacobi


def mode_list(p: int):
    """All (i, j, k) with i + j + k <= p, in the oracle's own order (i, then j, then k)."""
    return [(i, j, k) for i in range(p + 1) for j in range(p + 1 - i) for k in range(p + 1 - i - j)]


def num_modes(p: int) -> int:
    return (p + 1) * (p + 2) * (p + 3) // 6


def norm_factor(i: int, j: int, k: int) -> float:
    return float(np.sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3)))


def tet_quadrature(q: int):
    """Collapsed Gauss rule on the reference tet: points (Q,3), weights (Q,), exact
    for polynomials of degree <= 2q-1 in each collapsed variable."""
    xa, wa = gauss_jacobi(q, 2.0, 0.0)
    xb, wb = gauss_jacobi(q, 1.0, 0.0)
    xc, wc = gauss_jacobi(q, 0.0, 0.0)
    A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
    W = wa[:, None, None] * wb[None, :, None] * wc[None, None, :] / 64.0
    x = (1 + A) / 2
    y = (1 + B) * (1 - A) / 4
    z = (1 + C) * (1 - A) * (1 - B) / 8
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1), W.ravel()


def triangle_quadrature(q: int):
    """Collapsed Gauss rule on the unit triangle {s,t >= 0, s+t <= 1}: points (Q,2),
    weights (Q,) summing to 1/2."""
    xa, wa = gauss_jacobi(q, 1.0, 0.0)
    xb, wb = gauss_jacobi(q, 0.0, 0.0)
    A, B = np.meshgrid(xa, xb, indexing="ij")
    W = wa[:, None] * wb[None, :] / 8.0
    s = (1 + A) / 2
    t = (1 + B) * (1 - A) / 4
    return np.stack([s.ravel(), t.ravel()], axis=1), W.ravel()


def eval_basis(p: int, pts, grad: bool = False):
    """Values V[m, q] (and reference gradients G[m, q, 3]) of all modes at points pts[Q,3].

    Points must lie in the interior of the tetrahedron or on it away from the
    collapse singularities x = 1 and x + y = 1 when grad is requested.
    """
    pts = np.asarray(pts, dtype=np.float64)
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    one_x = 1.0 - x
    w = 1.0 - x - y
    a = 2.0 * x - 1.0
    with np.errstate(divide="ignore", invalid="ignore"):
        b = np.where(one_x > 0, 2.0 * y / np.where(one_x > 0, one_x, 1.0) - 1.0, -1.0)
        c = np.where(w > 0, 2.0 * z / np.where(w > 0, w, 1.0) - 1.0, -1.0)
    modes = mode_list(p)
    V = np.empty((len(modes), len(x)))
    G = np.empty((len(modes), len(x), 3)) if grad else None
    for m, (i, j, k) in enumerate(modes):
        nf = norm_factor(i, j, k)
        # factors: f1 = w^i P_i(c), f2 = (1-x)^j P_j^{(2i+1,0)}(b), f3 = P_k^{(2i+2j+2,0)}(a)
        Pi, Pj, Pk = jacobi(i, 0, 0, c), jacobi(j, 2 * i + 1, 0, b), jacobi(k, 2 * i + 2 * j + 2, 0, a)
        wi = w ** i
        oxj = one_x ** j
        V[m] = nf * wi * Pi * oxj * Pj * Pk
        if grad:
            dPi, dPj, dPk = djacobi(i, 0, 0, c), djacobi(j, 2 * i + 1, 0, b), djacobi(k, 2 * i + 2 * j + 2, 0, a)
            with np.errstate(divide="ignore", invalid="ignore"):
                # f1 = w^i P_i(c) with c = 2z/w - 1:  d f1/dz = 2 w^{i-1} P_i'(c),
                # d f1/dx = d f1/dy = -i w^{i-1} P_i(c) + w^i P_i'(c) * 2z/w^2
                wim1 = w ** (i - 1) if i > 0 else np.zeros_like(w)
                df1_dz = 2.0 * wim1 * dPi if i > 0 else np.zeros_like(w)
                df1_dw = (i * wim1 * Pi if i > 0 else np.zeros_like(w)) - wi * dPi * (1.0 + c) / np.where(w > 0, w, 1.0)
                # f2 = (1-x)^j P_j(b) with b = 2y/(1-x) - 1
                oxjm1 = one_x ** (j - 1) if j > 0 else np.zeros_like(x)
                df2_dy = 2.0 * oxjm1 * dPj if j > 0 else np.zeros_like(x)
                df2_dox = (j * oxjm1 * Pj if j > 0 else np.zeros_like(x)) - oxj * dPj * (1.0 + b) / np.where(one_x > 0, one_x, 1.0)
            f1 = wi * Pi
            f2 = oxj * Pj
            f3 = Pk
            df3_dx = 2.0 * dPk
            # w = 1-x-y:  dw/dx = dw/dy = -1;  (1-x): d/dx = -1
            gx = (-df1_dw) * f2 * f3 + f1 * (-df2_dox) * f3 + f1 * f2 * df3_dx
            gy = (-df1_dw) * f2 * f3 + f1 * df2_dy * f3
            gz = df1_dz * f2 * f3
            G[m, :, 0] = nf * gx
            G[m, :, 1] = nf * gy
            G[m, :, 2] = nf * gz
    return (V, G) if grad else V
