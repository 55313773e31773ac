"""Orthonormal Dubiner basis, face basis and collapsed quadrature (host, FP64).

Used at build time by the table generator and at set-up time by the
projection helper.  Definitions follow Section 3.1 (eq. phi2D) for the face
basis and Section 4.2.2 for the volume basis, each scaled to unit L2 norm.

Volume modes are stored degree-major: total degree n = i+j+k ascending, then
i, then j (k = n-i-j).  The modes of degree < p therefore come first, which
is where every derivative lands.  Index roles: i <-> z (innermost collapse),
j <-> y, k <-> x.

Face basis on the unit triangle {s,t >= 0, s+t <= 1}:
    psi_ab(s,t) = P_a(2t/(1-s) - 1) (1-s)^a P_b^{(2a+1,0)}(2s-1) sqrt((2a+1)(2a+2b+2)),
ordered by n = a+b, then a.
"""
from __future__ import annotations

import numpy as np
from scipy.special import eval_jacobi, roots_jacobi


def volume_modes(p: int):
    out = []
    for n in range(p + 1):
        for i in range(n + 1):
            for j in range(n - i + 1):
                out.append((i, j, n - i - j))
    return out


def face_modes(p: int):
    out = []
    for n in range(p + 1):
        for a in range(n + 1):
            out.append((a, n - a))
    return out


def collapsed_rule_tet(q: int):
    xa, wa = roots_jacobi(q, 2, 0)
    xb, wb = roots_jacobi(q, 1, 0)
    xc, wc = roots_jacobi(q, 0, 0)
    a, b, c = np.meshgrid(xa, xb, xc, indexing="ij")
    w = (wa[:, None, None] * wb[None, :, None] * wc[None, None, :]).ravel() / 64.0
    x = (1 + a) / 2
    y = (1 + b) * (1 - a) / 4
    z = (1 + c) * (1 - a) * (1 - b) / 8
    return np.stack([x.ravel(), y.ravel(), z.ravel()], 1), w


def collapsed_rule_tri(q: int):
    xa, wa = roots_jacobi(q, 1, 0)
    xb, wb = roots_jacobi(q, 0, 0)
    a, b = np.meshgrid(xa, xb, indexing="ij")
    w = (wa[:, None] * wb[None, :]).ravel() / 8.0
    s = (1 + a) / 2
    t = (1 + b) * (1 - a) / 4
    return np.stack([s.ravel(), t.ravel()], 1), w


def _collapsed(pts):
    x, y, z = pts[:, 0], pts[:, 1], pts[:, 2]
    ox = 1.0 - x
    w = 1.0 - x - y
    with np.errstate(divide="ignore", invalid="ignore"):
        b = np.where(ox > 1e-300, 2 * y / np.where(ox > 1e-300, ox, 1) - 1, -1.0)
        c = np.where(w > 1e-300, 2 * z / np.where(w > 1e-300, w, 1) - 1, -1.0)
    return x, y, z, ox, w, 2 * x - 1, b, c


def volume_values(p: int, pts):
    """V[m, q] = phi_m(pts[q]) for the degree-major mode order."""
    x, y, z, ox, w, a, b, c = _collapsed(np.asarray(pts, float))
    modes = volume_modes(p)
    V = np.empty((len(modes), len(x)))
    for r, (i, j, k) in enumerate(modes):
        s = np.sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
        V[r] = s * w ** i * ox ** j * eval_jacobi(i, 0, 0, c) * eval_jacobi(j, 2 * i + 1, 0, b) * eval_jacobi(k, 2 * i + 2 * j + 2, 0, a)
    return V


def volume_gradients(p: int, pts):
    """Reference gradients G[m, q, 3] of the degree-major modes at interior points.

    Chain rule through the collapsed coordinates, with the Jacobi derivative
    d/dx P_n^{(a,b)} = (n+a+b+1)/2 P_{n-1}^{(a+1,b+1)}.  Write
    phi = s * u(z; w) * v(y; ox) * P_k(a), u = w^i P_i(2z/w-1), v = ox^j P_j(2y/ox-1),
    w = 1-x-y, ox = 1-x.
    """
    x, y, z, ox, w, a, b, c = _collapsed(np.asarray(pts, float))

    def dj(n, al, x_):
        return 0.0 * x_ if n == 0 else 0.5 * (n + al + 1) * eval_jacobi(n - 1, al + 1, 1, x_)

    modes = volume_modes(p)
    G = np.empty((len(modes), len(x), 3))
    for r, (i, j, k) in enumerate(modes):
        s = np.sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
        Pi, dPi = eval_jacobi(i, 0, 0, c), dj(i, 0, c)
        Pj, dPj = eval_jacobi(j, 2 * i + 1, 0, b), dj(j, 2 * i + 1, b)
        Pk, dPk = eval_jacobi(k, 2 * i + 2 * j + 2, 0, a), dj(k, 2 * i + 2 * j + 2, a)
        u = w ** i * Pi
        # partial derivatives of u in (z, w) and of v in (y, ox)
        u_z = 2.0 * w ** (i - 1) * dPi if i > 0 else 0.0 * x
        u_w = (i * w ** (i - 1) * Pi - w ** (i - 1) * dPi * (1 + c)) if i > 0 else 0.0 * x
        v = ox ** j * Pj
        v_y = 2.0 * ox ** (j - 1) * dPj if j > 0 else 0.0 * x
        v_o = (j * ox ** (j - 1) * Pj - ox ** (j - 1) * dPj * (1 + b)) if j > 0 else 0.0 * x
        # dw/dx = dw/dy = -1, d ox/dx = -1, da/dx = 2
        G[r, :, 0] = s * (-u_w * v * Pk - u * v_o * Pk + u * v * 2.0 * dPk)
        G[r, :, 1] = s * (-u_w * v * Pk + u * v_y * Pk)
        G[r, :, 2] = s * (u_z * v * Pk)
    return G


def face_values(p: int, st):
    st = np.asarray(st, float)
    s, t = st[:, 0], st[:, 1]
    os_ = 1.0 - s
    with np.errstate(divide="ignore", invalid="ignore"):
        eta = np.where(os_ > 1e-300, 2 * t / np.where(os_ > 1e-300, os_, 1) - 1, -1.0)
    modes = face_modes(p)
    V = np.empty((len(modes), len(s)))
    for r, (a, b) in enumerate(modes):
        V[r] = np.sqrt((2 * a + 1) * (2 * a + 2 * b + 2)) * eval_jacobi(a, 0, 0, eta) * os_ ** a * eval_jacobi(b, 2 * a + 1, 0, 2 * s - 1)
    return V
