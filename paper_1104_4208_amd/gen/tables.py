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
  in increasing local index.  T_f^T is the lift used by the face flux.
  Densities at p = 6: 1572 (slanted face 0), 84 (x = 0, a signed sum over the
  x index k), 336 (y = 0) and 1320 (z = 0) of 2352 entries.
* the collapsed tensor-product factorisation of the two dense traces
  (Section 3.2.3: traces in O(N) through the tensor-product structure), see
  ``factors``: T_3 = B A_3 and T_0 = C B A_0 with A block-diagonal over
  (m, k) = (i + j, k) (a Legendre transform in the inner collapsed
  coordinate), B block-diagonal over the face index a (a Jacobi re-expansion
  in the outer one) and C block-diagonal over the face degree (the change
  between the two orthonormal face bases collapsed at different vertices):
  666 and 804 multiply-adds per scalar at p = 6 instead of 1320 and 1572;
  the y = 0 trace is B itself up to a column scaling (336).
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
        self.NV = self.N  # rows of the updated field (differs only in a mixed-order coupling)


class Coupling:
    """Operators of a phase between fields of different orders (Section 2: E of degree
    p + 1, H of degree p).  U (the differentiated field) has order pU, V (the updated one)
    order pV.  Because the mode orders are hierarchical (degree-major), every operator is
    a block of the higher order's exact table: the curl maps the N_U modes of U into the
    N_V rows of V (D[:N_V, :N_U]), the lift maps U's NF_U face modes into V's rows
    (T[:NF_U, :N_V]^T; a degree-pU trace has no component on higher face modes), and the
    collapsed factors are sliced the same way.  Attributes mirror Tables: N = N_U (the
    staged field's modes), NV = N_V, NF = NF_U, modes / p of V (its (m, k) blocks),
    fmodes of U."""

    def __init__(self, pU, pV):
        t = build(max(pU, pV))
        u, v = build(pU), build(pV)
        self.p, self.pU = pV, pU
        self.modes, self.fmodes = v.modes, u.fmodes
        self.N, self.NV, self.NF = u.N, v.N, u.NF
        self.D = [D[:v.N, :u.N] for D in t.D]
        self.T = [T[:u.NF, :v.N] for T in t.T]
        fac = t.fac
        self.fac = dict(X=fac["X"], A3=fac["A3"][:, :v.N], A0=fac["A0"][:, :v.N], B=fac["B"][:u.NF],
                        C=fac["C"][:u.NF, :u.NF])
        self.tang, self.normal, self.L, self.frame = t.tang, t.normal, t.L, t.frame
        self.mixed = pU != pV


@functools.lru_cache(maxsize=None)
def coupling(pU: int, pV: int):
    """Tables of the phase differentiating order pU and updating order pV (the order's own
    Tables when they are equal)."""
    return build(pU) if pU == pV else Coupling(pU, pV)


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
    t.fac = factors(t)
    for f, prod in ((3, t.fac["B"] @ t.fac["A3"]), (0, t.fac["C"] @ t.fac["B"] @ t.fac["A0"])):
        if np.abs(prod - t.T[f]).max() > 1e-12:
            raise AssertionError(f"trace factors of face {f} do not reproduce T{f}")
    return t


def factors(t: Tables):
    """Collapsed tensor-product factors of the face-0 and face-3 traces.

    On z = 0 (face 3, points (s, t, 0)) and, after the barycentric relabelling
    (s, t) -> (1 - s - t, s), on the slanted face 0 (points (1 - s - t, s, t)) the
    restriction of phi_ijk separates as
        sqrt((2i+1)(2m+2)) sigma_i ((1-eta)/2)^i P_j^{(2i+1,0)}(eta)
          * (1-s)^m P_k^{(2m+2,0)}(2s-1) sqrt(2m+2k+3),      m = i + j,
    with sigma_i = (-1)^i on z = 0 (the innermost factor at c = -1) and 1 on
    the slanted face (c = +1).  Expanding the eta factor in orthonormal Legendre
    polynomials gives the intermediate coefficients X[(a,m,k)] = A[(a,m,k), (i,j,k)]
    u[(i,j,k)] (a <= m); each intermediate function
        Lambda_amk = Phat_a(eta) (1-s)^m P_k^{(2m+2,0)}(2s-1) sqrt(2m+2k+3)
    projects onto the face modes (a, b) of the same a only (B).  On face 0 the
    result is in the face basis collapsed towards the face's first vertex,
    chi_ab(s, t) = psi_ab(1 - s - t, s); C maps it to psi and mixes only modes of
    equal degree a + b.  Returns dict(X = [(a, m, k)], A3, A0, B, C) with exact
    zeros; ``build`` checks B A3 = T_3 and C B A0 = T_0 to 1e-12.
    """
    from scipy.special import eval_jacobi, roots_legendre

    p = t.p
    idx = {m: r for r, m in enumerate(t.modes)}
    X = [(a, m, k) for m in range(p + 1) for k in range(p - m + 1) for a in range(m + 1)]
    xidx = {v: r for r, v in enumerate(X)}
    xe, we = roots_legendre(p + 2)
    phat = lambda a, x: np.sqrt((2 * a + 1) / 2.0) * eval_jacobi(a, 0, 0, x)
    A3 = np.zeros((len(X), t.N))
    A0 = np.zeros((len(X), t.N))
    for (i, j, k) in t.modes:
        m = i + j
        f = np.sqrt((2 * i + 1) * (2 * m + 2)) * ((1 - xe) / 2) ** i * eval_jacobi(j, 2 * i + 1, 0, xe)
        for a in range(m + 1):
            v = float(np.sum(we * phat(a, xe) * f))
            A0[xidx[(a, m, k)], idx[(i, j, k)]] = v
            A3[xidx[(a, m, k)], idx[(i, j, k)]] = v * (-1) ** i
    st, wt = B.collapsed_rule_tri(p + 2)
    s, tt = st[:, 0], st[:, 1]
    os_ = 1.0 - s
    eta = np.where(os_ > 1e-300, 2 * tt / np.where(os_ > 1e-300, os_, 1) - 1, -1.0)
    lam = np.empty((len(X), len(s)))
    for r, (a, m, k) in enumerate(X):
        lam[r] = phat(a, eta) * os_ ** m * eval_jacobi(k, 2 * m + 2, 0, 2 * s - 1) * np.sqrt(2 * m + 2 * k + 3)
    Vf = B.face_values(p, st)
    Bm = (Vf * wt) @ lam.T
    C = (Vf * wt) @ B.face_values(p, np.stack([1.0 - s - tt, s], 1)).T
    return dict(X=X, A3=_clean(A3, "A3"), A0=_clean(A0, "A0"), B=_clean(Bm, "B"), C=_clean(C, "C"))


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


@functools.lru_cache(maxsize=None)
def mass_factors(p: int):
    """Sum-factorisation tables of the approximate mass inverse (Section 3.3.2) on the
    collapsed Gauss rule with q = p + 1 points per direction (exact on products of two
    basis functions).  At the point (a, b, c) of the collapsed coordinates
        phi_ijk = s_ijk ((1-a)/2)^(i+j) P_k^{(2i+2j+2,0)}(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b) P_i(c)
    so phi = C1[r, qa] * Fb[i, j, qb] * Fc[i, qc] with C1 the s- and a-factor of mode r.
    Returns dict(q, C1 (N, q), Fb (p+1, p+1, q), Fc (p+1, q), W (q, q, q) the weights,
    lam (q, q, q, 4) the barycentric coordinates of the points); build checks the product
    against the basis values."""
    from scipy.special import eval_jacobi, roots_jacobi

    t = build(p)
    q = p + 1
    xa, _ = roots_jacobi(q, 2, 0)
    xb, _ = roots_jacobi(q, 1, 0)
    xc, _ = roots_jacobi(q, 0, 0)
    C1 = np.zeros((t.N, q))
    for r, (i, j, k) in enumerate(t.modes):
        s = np.sqrt((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
        C1[r] = s * ((1 - xa) / 2) ** (i + j) * eval_jacobi(k, 2 * i + 2 * j + 2, 0, xa)
    Fb = np.zeros((p + 1, p + 1, q))
    Fc = np.zeros((p + 1, q))
    for i in range(p + 1):
        Fc[i] = eval_jacobi(i, 0, 0, xc)
        for j in range(p + 1 - i):
            Fb[i, j] = ((1 - xb) / 2) ** i * eval_jacobi(j, 2 * i + 1, 0, xb)
    pts, w = B.collapsed_rule_tet(q)
    V = B.volume_values(p, pts).reshape(t.N, q, q, q)
    for r, (i, j, k) in enumerate(t.modes):
        prod = C1[r][:, None, None] * Fb[i, j][None, :, None] * Fc[i][None, None, :]
        if np.abs(prod - V[r]).max() > 1e-11 * max(1.0, np.abs(V[r]).max()):
            raise AssertionError("mass factors do not reproduce the basis")
    lam = np.stack([1 - pts.sum(1), pts[:, 0], pts[:, 1], pts[:, 2]], axis=1).reshape(q, q, q, 4)
    return dict(q=q, C1=C1, Fb=Fb, Fc=Fc, W=w.reshape(q, q, q), lam=lam)
