"""Stabilised central flux with face unknowns H^F (Section 2.1), plain FP64.

Test infrastructure only (see the package header).

Unknowns: E, H as in ``dg.Solver`` (physical Cartesian modal coefficients) plus,
on every face F of the mesh (interior and wall), a tangential vector field H^F
of degree p, stored as Cartesian coefficient vectors b[F, m] of an orthonormal
basis chi_m of P_p(F):  chi_m = psi_m(s, t) / sqrt(2|F|), where (s, t) are the
coordinates x = w0 + s (w1 - w0) + t (w2 - w0) of the face with its vertices w0,
w1, w2 in increasing global id and psi_m the orthonormal triangle basis (the
printed two-dimensional basis, Section 3.1, scaled to unit norm).

Equations (the consistent reading; see below):
    (eps dE/dt, e)_T = (H, curl e)_T + (nu x {H}, e)_dT + sum_{F in dT} (H^F x nu_T, e)_F * c_F
    (mu dH/dt, h)_T  = -(curl E, h)_T - 1/2 (nu x (E_nb - E), h)_dT
    (h_F / alpha)(dH^F/dt, h^F)_F = ([E] x nu, h^F)_F
with [E] = E_s - E_nb and nu = nu_s (outward from the face's first side s; the
product is the same from either side), alpha = alpha0 p^2, h_F = 3 min |T| / |F|
over the face's elements (the smaller height over F), and on perfect-conductor
walls the ghost convention E_nb = -E: [E] = 2 E_s and the test-function jump
[e] = 2 e_s, so c_F = 2 on walls and 1 inside.

Reading: the paper prints the face-unknown equation with alpha/h on the left.
That contradicts its own definition H^F = alpha [E] x nu / (i omega h) and its
frequency-domain penalty S(E, e) = (alpha/h)([E] x nu, [e] x nu)_F, which both
follow from a face mass of h/alpha; with alpha/h on the left the penalty would
scale like h/alpha, against the requirement that it grow with p^2.  The mass
h/alpha is used here.  Either choice keeps the system skew (energy conserving).

Energy W = 1/2 (eps E, E) + 1/2 (mu H, H) + 1/2 sum_F (h_F/alpha) |b_F|^2 and the
leapfrog invariant Q (H and H^F paired between consecutive steps) are conserved.
"""
from __future__ import annotations

import numpy as np

from .basis import eval_basis, triangle_quadrature
from .dg import _FACE_LOCAL, Solver
from .jacobi import jacobi


def triangle_basis(p: int, st):
    """Orthonormal basis psi_m(s, t) on the unit triangle, m ordered by a + b then a:
    P_a(2t/(1-s) - 1) (1-s)^a P_b^{(2a+1,0)}(2s - 1) sqrt((2a+1)(2a+2b+2))."""
    s, t = st[:, 0], st[:, 1]
    os_ = 1.0 - s
    with np.errstate(divide="ignore", invalid="ignore"):
        eta = np.where(os_ > 0, 2.0 * t / np.where(os_ > 0, os_, 1.0) - 1.0, -1.0)
    out = []
    for n in range(p + 1):
        for a in range(n + 1):
            b = n - a
            out.append(np.sqrt((2 * a + 1) * (2 * a + 2 * b + 2)) * jacobi(a, 0, 0, eta) * os_ ** a
                       * jacobi(b, 2 * a + 1, 0, 2 * s - 1))
    return np.array(out)


class StabilizedSolver(Solver):
    """Central flux plus the face-unknown stabilisation (Section 2.1)."""

    def __init__(self, mesh, p, eps=None, mu=None, alpha0: float = 1.0, chunk: int = 2048):
        super().__init__(mesh, p, eps, mu, chunk)
        m = mesh
        self.alpha = alpha0 * p * p
        st, w = triangle_quadrature(p + 2)
        self.fw = w
        self.psi = triangle_basis(p, st)  # (NF, Qf)
        self.NF = self.psi.shape[0]
        faces = {}
        for e in range(self.K):
            for f in range(4):
                key = tuple(sorted(int(m.tets[e, v]) for v in _FACE_LOCAL[f]))
                faces.setdefault(key, []).append((e, f))
        self.faces = sorted(faces)
        self.sides = [faces[k] for k in self.faces]
        nF = len(self.faces)
        self.nF = nF
        self.area = np.empty(nF)
        self.hF = np.empty(nF)
        self.nu = np.empty((nF, 3))
        self.face_x = []   # physical quadrature points per face (Qf,3)
        self.side_V = []   # per face, per side: element basis values at the points (N,Qf)
        vol = np.abs(m.J) / 6.0
        for i, (key, sd) in enumerate(zip(self.faces, self.sides)):
            w0, w1, w2 = (m.verts[v] for v in key)
            n = np.cross(w1 - w0, w2 - w0)
            self.area[i] = 0.5 * np.linalg.norm(n)
            e0, f0 = sd[0]
            self.nu[i] = m.normal[e0, f0]
            self.hF[i] = 3.0 * min(vol[e] for e, _ in sd) / self.area[i]
            x = w0 + st[:, :1] * (w1 - w0) + st[:, 1:] * (w2 - w0)
            self.face_x.append(x)
            vals = []
            for e, f in sd:
                xh = (x - m.verts[m.tets[e, 0]]) @ m.Finv[e].T  # reference coordinates in e
                vals.append(eval_basis(p, xh))
            self.side_V.append(vals)

    def zeros_faces(self):
        return np.zeros((self.nF, self.NF, 3))

    def _jump_cross_nu(self, e_coef, i):
        """([E] x nu)(x_q) on face i (Qf,3), [E] = E_s - E_nb (2 E_s on walls)."""
        sd, V = self.sides[i], self.side_V[i]
        Es = np.einsum("aq,ad->qd", V[0], e_coef[sd[0][0]])
        jump = Es - np.einsum("aq,ad->qd", V[1], e_coef[sd[1][0]]) if len(sd) == 2 else 2.0 * Es
        return np.cross(jump, self.nu[i][None, :])

    def rhs_faces(self, e_coef):
        """dH^F/dt from E: b'[F, m] = (alpha/h_F) int_F ([E] x nu) chi_m dA."""
        out = np.empty((self.nF, self.NF, 3))
        for i in range(self.nF):
            g = self._jump_cross_nu(e_coef, i)
            # int_F g chi_m dA = 2|F| sum_q w_q g psi_m / sqrt(2|F|)
            out[i] = np.sqrt(2.0 * self.area[i]) * np.einsum("q,mq,qd->md", self.fw, self.psi, g)
            out[i] *= self.alpha / self.hF[i]
        return out

    def rhs_e_stab(self, h_coef, b):
        """dE/dt from H and H^F: the central weak form plus (H^F x nu_T, e)_F c_F."""
        r = self.rhs_e(h_coef) * (self.absJ * self.eps)[:, None, None]
        m = self.m
        for i in range(self.nF):
            sd, V = self.sides[i], self.side_V[i]
            HF = np.einsum("mq,md->qd", self.psi, b[i]) / np.sqrt(2.0 * self.area[i])  # (Qf,3)
            cF = 1.0 if len(sd) == 2 else 2.0
            ds = 2.0 * self.area[i] * self.fw
            for (e, f), Ve in zip(sd, V):
                g = np.cross(HF, m.normal[e, f][None, :])
                r[e] += cF * np.einsum("aq,ql->al", Ve, ds[:, None] * g)
        return r / (self.absJ * self.eps)[:, None, None]

    def step_stab(self, E, H, b, dt, nsteps=1):
        """Symplectic Euler, H and H^F first (both from E^n), then E (Section 3)."""
        E, H, b = E.copy(), H.copy(), b.copy()
        for _ in range(nsteps):
            H = H + dt * self.rhs_h(E)
            b = b + dt * self.rhs_faces(E)
            E = E + dt * self.rhs_e_stab(H, b)
        return E, H, b

    def face_dot(self, a, c):
        return float(np.einsum("f,fmd,fmd->", self.hF / self.alpha, a, c))

    def energy_stab(self, E, H, b):
        return self.energy(E, H) + 0.5 * self.face_dot(b, b)

    def leapfrog_invariant_stab(self, E, H, b, dt):
        Hn1 = H + dt * self.rhs_h(E)
        bn1 = b + dt * self.rhs_faces(E)
        return (0.5 * self.mass_dot(E, E, "E") + 0.5 * self.mass_dot(H, Hn1, "H")
                + 0.5 * self.face_dot(b, bn1))

    def assemble_stab(self):
        """Dense blocks of the stabilised semi-discrete system on tiny meshes, in the
        flattened (K,N,3) and (nF,NF,3) orders: A_h (dH from E), A_f (dH^F from E),
        A_e (dE from H) and A_b (dE from H^F)."""
        n, nb = self.K * self.N * 3, self.nF * self.NF * 3
        Ah, Af = np.empty((n, n)), np.empty((nb, n))
        Ae, Ab = np.empty((n, n)), np.empty((n, nb))
        z = self.zeros_faces()
        for c in range(n):
            u = np.zeros(n)
            u[c] = 1.0
            U = u.reshape(self.K, self.N, 3)
            Ah[:, c] = self.rhs_h(U).ravel()
            Af[:, c] = self.rhs_faces(U).ravel()
            Ae[:, c] = self.rhs_e_stab(U, z).ravel()
        zh = np.zeros((self.K, self.N, 3))
        for c in range(nb):
            u = np.zeros(nb)
            u[c] = 1.0
            Ab[:, c] = self.rhs_e_stab(zh, u.reshape(self.nF, self.NF, 3)).ravel()
        return Ah, Af, Ae, Ab

    def spectral_radius_stab(self, iters: int, start):
        """Power iteration on E -> -dE(dH(E), dH^F(E)) (the second-order operator whose
        largest eigenvalue bounds the leapfrog step); Rayleigh estimate in the eps mass."""
        x = np.asarray(start, float).reshape(self.K, self.N, 3)
        lam = 0.0
        for _ in range(iters):
            y = -self.rhs_e_stab(self.rhs_h(x), self.rhs_faces(x))
            lam = self.mass_dot(x, y, "E") / self.mass_dot(x, x, "E")
            x = y / np.sqrt(self.mass_dot(y, y, "E"))
        return lam
