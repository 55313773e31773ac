"""Reference-element operator tables for the DG curl (host, FP64, build time).

For polynomial order p this computes, on the reference tetrahedron with the
orthonormal degree-major Dubiner basis (gen/basis.py):

* sparse directional-derivative operators  D_d[b, a] = int phi_b (d . grad) phi_a
  for the three edge directions  d1 = (0,0,1), d2 = (1,-1,0), d3 = (0,2,-1).
  Section 3.2.2 computes derivatives modally through recurrences that follow
  the collapsed tensor-product structure; the same structure makes these
  operators sparse, and along these three directions (the collapse direction
  of the innermost Legendre factor, the edge v1->v2 that leaves that factor
  untouched, and a third one) they are sparsest: 686 + 504 + 868 nonzeros at
  p = 6 against 1680 + 1554 + 686 for x, y, z.  The curl is then assembled in
  that frame (see ``frame``).
* trace operators  T_f[m, a] = int_{unit triangle} psi_m(s,t) phi_a(xhat_f(s,t)) ds dt
  for the four faces in the sorted-vertex parametrisation
  xhat_f(s,t) = w0 + s (w1 - w0) + t (w2 - w0), (w0, w1, w2) the face's vertices
  in increasing local index (Section 3.2.3 evaluates traces modally through the
  tensor-product structure; T_0 is a signed sum over k, the others are sparse
  tables).  T_f^T is the lift used by the face flux.
* the face frames: reference edge tangents t1 = w1 - w0, t2 = w2 - w0, the
  scaled outer normals n_f (unit-triangle measure) and the 3x2 map L_f with
  n_f x a = L_f (a.t1, a.t2)  for any vector a.

Exact zeros are found from a gap of more than six decades between the
largest rounding residue (< 1e-12) and the smallest true entry (> 1e-6 for
p <= 10); ``build`` asserts the gap.
"""
from __future__ import annotations

import functools

import numpy as np

from . import basis as B

DIRS = np.array([[0.0, 0.0, 1.0], [1.0, -1.0, 0.0], [0.0, 2.0, -1.0]])
REF_VERTS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
FACE_VERTS = [tuple(v for v in range(4) if v != f) for f in range(4)]
ZERO_TOL = 1e-9
P_MAX = 8


class Tables:
    def __init__(self, p):
        self.p = p
        self.modes = B.volume_modes(p)
        self.fmodes = B.face_modes(p)
        self.N = len(self.modes)
        self.NF = len(self.fmodes)


def _clean(M, what):
    a = np.abs(M)
    small = a[a < ZERO_TOL]
    big = a[a >= ZERO_TOL]
    if small.size and small.max() > 1e-11:
        raise AssertionError(f"{what}: rounding residue {small.max()} too large")
    if big.size and big.min() < 1e-7:
        raise AssertionError(f"{what}: smallest entry {big.min()} too close to zero")
    out = M.copy()
    out[a < ZERO_TOL] = 0.0
    return out


@functools.lru_cache(maxsize=None)
def build(p: int) -> Tables:
    t = Tables(p)
    q = p + 2
    x, w = B.collapsed_rule_tet(q)
    V = B.volume_values(p, x)
    G = B.volume_gradients(p, x)
    mass = (V * w) @ V.T
    if np.abs(mass - np.eye(t.N)).max() > 1e-12:
        raise AssertionError("basis is not orthonormal")
    t.D = []
    for d in DIRS:
        t.D.append(_clean((V * w) @ (G @ d).T, f"D{d}"))
    st, wt = B.collapsed_rule_tri(q)
    Vf = B.face_values(p, st)
    fmass = (Vf * wt) @ Vf.T
    if np.abs(fmass - np.eye(t.NF)).max() > 1e-12:
        raise AssertionError("face basis is not orthonormal")
    t.T = []
    t.tang = []
    t.normal = []
    t.L = []
    for f in range(4):
        w0, w1, w2 = (REF_VERTS[v] for v in FACE_VERTS[f])
        pts = w0[None, :] + st[:, :1] * (w1 - w0)[None, :] + st[:, 1:] * (w2 - w0)[None, :]
        t.T.append(_clean((Vf * wt) @ B.volume_values(p, pts).T, f"T{f}"))
        t1, t2 = w1 - w0, w2 - w0
        n = np.cross(t1, t2)
        opp = REF_VERTS[f]
        if np.dot(n, opp - w0) > 0:
            n = -n
        Gm = np.array([[t1 @ t1, t1 @ t2], [t2 @ t1, t2 @ t2]])
        L = np.stack([np.cross(n, t1), np.cross(n, t2)], axis=1) @ np.linalg.inv(Gm)
        t.tang.append((t1, t2))
        t.normal.append(n)
        t.L.append(L)
    t.frame = frame()
    return t


@functools.lru_cache(maxsize=None)
def frame():
    """Constants of the derivative frame A (rows d1, d2, d3).

    For a covariant field u with w = A u, c_k = d_i(w_j) - d_j(w_i) over the cyclic
    (i,j,k) gives curl u = A^T c / det A.  State is kept in the frame
    S = det A * A^{-T} K^{-1} u (K the per-element mass-inverse factor), in which the
    update of component k is c_k plus the lifted face terms mapped by det A * A^{-T}.
    """
    A = DIRS.copy()
    detA = float(np.linalg.det(A))
    Ainv = np.linalg.inv(A)
    AinvT = Ainv.T
    return dict(A=A, detA=detA, Ainv=Ainv, AinvT=AinvT)


def face_weights(t: Tables):
    """g[f][k] (3-vectors): tangential component k of face f is  g . w  with w = A u;
    Lp[f] (3x2): stored-frame face term  1/2 det A A^{-T} L_f  applied to the jump of
    the two tangential traces."""
    fr = t.frame
    g = []
    Lp = []
    for f in range(4):
        t1, t2 = t.tang[f]
        g.append((fr["AinvT"] @ t1, fr["AinvT"] @ t2))
        Lp.append(0.5 * fr["detA"] * fr["AinvT"] @ t.L[f])
    return g, Lp


def op_counts(p: int):
    t = build(p)
    nD = [int((D != 0).sum()) for D in t.D]
    nT = [int((T != 0).sum()) for T in t.T]
    return dict(p=p, N=t.N, NF=t.NF, nnz_D=nD, nnz_T=nT)
