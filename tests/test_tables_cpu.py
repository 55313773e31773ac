"""The product's reference operator tables against the oracle's own quadrature.

gen/tables.py builds the derivative operators D_d and the face-trace operators
T_f with its own basis code and quadrature; here every entry is recomputed at
p = 1..8 from the oracle's basis (its own Jacobi recurrence and Golub-Welsch
rules) and from the orthonormal triangle basis written out from the printed
two-dimensional formula (Section 3.1, eq. phi2D, scaled to unit norm), and the
collapsed tensor-product factors of the two dense traces (Section 3.2.3) are
checked to multiply back to T_3 and T_0.  Entries agree to 1e-13 of the largest
entry (1e-12 absolute for the traces, whose entries are O(1)).
"""
import numpy as np
import pytest

from oracle.basis import eval_basis, mode_list, tet_quadrature, triangle_quadrature
from oracle.jacobi import jacobi
from paper_1104_4208_amd.gen import tables as TB

REF = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])


def psi(p, st):
    """Orthonormal triangle basis (a, b) ordered by a + b, then a:
    P_a(2t/(1-s) - 1) (1-s)^a P_b^{(2a+1,0)}(2s-1) sqrt((2a+1)(2a+2b+2))."""
    s, t = st[:, 0], st[:, 1]
    os_ = 1.0 - s
    eta = np.where(os_ > 1e-300, 2 * t / np.where(os_ > 1e-300, os_, 1.0) - 1.0, -1.0)
    rows = []
    for n in range(p + 1):
        for a in range(n + 1):
            b = n - a
            rows.append(np.sqrt((2 * a + 1) * (2 * a + 2 * b + 2)) * jacobi(a, 0, 0, eta) * os_ ** a
                        * jacobi(b, 2 * a + 1, 0, 2 * s - 1))
    return np.array(rows)


def perm(p):
    """Oracle rows of the product's modes."""
    om = {m: r for r, m in enumerate(mode_list(p))}
    return np.array([om[m] for m in TB.build(p).modes])


@pytest.mark.parametrize("p", range(1, TB.P_MAX + 1))
def test_derivative_operators_match_oracle_quadrature(p):
    t = TB.build(p)
    x, w = tet_quadrature(p + 2)
    V, G = eval_basis(p, x, grad=True)
    pm = perm(p)
    V, G = V[pm], G[pm]
    for d, D in zip(TB.DIRS, t.D):
        ref = (V * w) @ (G @ d).T
        assert np.abs(ref - D).max() < 1e-13 * max(1.0, np.abs(D).max())


@pytest.mark.parametrize("p", range(1, TB.P_MAX + 1))
def test_trace_operators_match_oracle_quadrature(p):
    t = TB.build(p)
    st, wt = triangle_quadrature(p + 2)
    Pf = psi(p, st)
    assert np.abs((Pf * wt) @ Pf.T - np.eye(t.NF)).max() < 1e-12  # orthonormal
    pm = perm(p)
    for f in range(4):
        w0, w1, w2 = (REF[v] for v in range(4) if v != f)
        pts = w0 + st[:, :1] * (w1 - w0) + st[:, 1:] * (w2 - w0)
        ref = (Pf * wt) @ eval_basis(p, pts)[pm].T
        assert np.abs(ref - t.T[f]).max() < 1e-12
    # the factored forms used by the kernels
    fac = t.fac
    assert np.abs(fac["B"] @ fac["A3"] - t.T[3]).max() < 1e-12
    assert np.abs(fac["C"] @ fac["B"] @ fac["A0"] - t.T[0]).max() < 1e-12
    # C is the change between two orthonormal bases: orthogonal, block-diagonal by degree
    assert np.abs(fac["C"] @ fac["C"].T - np.eye(t.NF)).max() < 1e-12
    deg = np.array([a + b for a, b in t.fmodes])
    assert np.all(fac["C"][deg[:, None] != deg[None, :]] == 0.0)
    # x = 0 is a signed sum over the x index: one entry per volume mode
    assert np.count_nonzero(t.T[1]) == t.N


def test_factored_traces_are_cheaper():
    """Multiply-adds per scalar of the two dense traces, direct vs factored (p = 6, 8)."""
    for p, direct, fac in ((6, (1572, 1320), (804, 666)), (8, (4883, 4075), (1923, 1640))):
        t = TB.build(p)
        f = t.fac
        nz = lambda M: int(np.count_nonzero(M))
        assert (nz(t.T[0]), nz(t.T[3])) == direct
        assert (nz(f["C"]) + nz(f["B"]) + nz(f["A0"]), nz(f["B"]) + nz(f["A3"])) == fac
