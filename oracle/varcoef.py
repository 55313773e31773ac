"""Variable material inside the elements through the approximate mass inverse
(Section 3.3.2), plain FP64.

Test infrastructure only (see the package header).

eps and mu vary linearly on each element, given by their values at the element's four
vertices (in the element's vertex order).  The exact mass matrix of element T,
    (M_eps)_{(a,l),(b,m)} = int_T eps phi_a phi_b dx (delta_lm in physical components),
is no longer diagonal.  Section 3.3.2 replaces its inverse by an approximate one that is
again cheap: for a functional f (the right-hand side, given by its moments
f_a = int_T f phi_a dx), "reverse numerical integration" gives point values f_i at the
quadrature points x_i with  f(v) = sum_i |det F| w_i f_i v(x_i)  for every v of the space
(f_i = sum_a f_a phi_a(x_i) / |det F| for the orthonormal basis and a rule exact on
products of two basis functions), the point values are divided by eps(x_i), and
numerical integration maps them back to coefficients:
    (M~^{-1} f)_a = sum_i w_i phi_a(x_i) f_i / eps(x_i).
With constant eps this is the exact inverse; in general it is symmetric positive definite.
The rule is the collapsed Gauss rule with p + 1 points per direction.  This solver uses the
central flux of dg.Solver for the right-hand sides and M~^{-1} in place of M^{-1}; the
scheme is skew in the inner product of M~ = (M~^{-1})^{-1}, so the leapfrog invariant with
M~ is conserved exactly.
"""
from __future__ import annotations

import numpy as np

from .basis import eval_basis, tet_quadrature
from .dg import Solver


class VarMaterialSolver(Solver):
    def __init__(self, mesh, p, eps_v, mu_v, chunk: int = 2048):
        """eps_v, mu_v: (K, 4) values at each element's vertices (element vertex order)."""
        eps_v = np.asarray(eps_v, float)
        mu_v = np.asarray(mu_v, float)
        if np.any(eps_v <= 0) or np.any(mu_v <= 0):
            raise ValueError("material must be positive")
        # the central-flux right-hand sides with unit material: they return the moments
        # divided by |J| (the flat mass inverse with eps = mu = 1)
        super().__init__(mesh, p, None, None, chunk)
        self.eps_v, self.mu_v = eps_v, mu_v
        xq, wq = tet_quadrature(p + 1)
        self.mx, self.mw = xq, wq
        self.mV = eval_basis(p, xq)  # (N, Q)
        lam = np.stack([1 - xq.sum(1), xq[:, 0], xq[:, 1], xq[:, 2]], axis=1)  # barycentric (Q, 4)
        self.eps_q = eps_v @ lam.T  # (K, Q)
        self.mu_q = mu_v @ lam.T

    def approx_inverse(self, moments, which):
        """M~^{-1} applied to moments (K, N, 3) of a functional: reverse integration,
        division by the material at the points, integration."""
        m = self.eps_q if which == "E" else self.mu_q
        f = np.einsum("aq,kad->kqd", self.mV, moments) / self.absJ[:, None, None]  # point values
        f = f / m[:, :, None]
        return np.einsum("aq,q,kqd->kad", self.mV, self.mw, f)

    def exact_inverse(self, moments, which):
        """The exact mass inverse (dense per element), for comparison."""
        xq, wq = tet_quadrature(self.p + 2)
        V = eval_basis(self.p, xq)
        lam = np.stack([1 - xq.sum(1), xq[:, 0], xq[:, 1], xq[:, 2]], axis=1)
        mq = (self.eps_v if which == "E" else self.mu_v) @ lam.T
        out = np.empty_like(moments)
        for k in range(self.K):
            M = self.absJ[k] * np.einsum("aq,q,bq->ab", V, wq * mq[k], V)
            out[k] = np.linalg.solve(M, moments[k])
        return out

    def mass_approx(self, which):
        """M~ (K, N, N): the inverse of the scalar approximate inverse, per element."""
        m = self.eps_q if which == "E" else self.mu_q
        out = np.empty((self.K, self.N, self.N))
        for k in range(self.K):
            P = np.einsum("aq,q,bq->ab", self.mV, self.mw / m[k], self.mV) / self.absJ[k]
            out[k] = np.linalg.inv(P)
        return out

    def rhs_h(self, e_coef):
        return self.approx_inverse(super().rhs_h(e_coef) * self.absJ[:, None, None], "H")

    def rhs_e(self, h_coef):
        return self.approx_inverse(super().rhs_e(h_coef) * self.absJ[:, None, None], "E")

    def mass_dot(self, a, b, which):
        M = self.mass_approx(which)
        return float(np.einsum("kad,kab,kbd->", a, M, b))
