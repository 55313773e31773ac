"""Mixed orders: E of degree pE, H of degree pH (Section 2 uses pE = pH + 1), plain FP64.

Test infrastructure only (see the package header).

Section 2 shifts every derivative onto E and its test functions (the E equation in
the weak form), which is why it approximates E one degree higher than H.  The
equations are those of ``dg.Solver`` (central flux, consistent signs, PEC ghosts
E_nb = -E, H_nb = H), with E expanded in the degree-pE modes and tested against
them, H in the degree-pH modes:
    (mu dH/dt, h)_T  = -(curl E, h)_T - 1/2 (nu x (E_nb - E), h)_dT,     h in P_pH
    (eps dE/dt, e)_T = (H, curl e)_T + (nu x {H}, e)_dT,                  e in P_pE
Every integral uses one Gauss rule exact for the products of both orders; the
neighbour's field is evaluated through its own inverse map, as in ``dg``.
"""
from __future__ import annotations

import numpy as np

from .basis import eval_basis, num_modes, tet_quadrature, triangle_quadrature
from .dg import _FACE_LOCAL, _REF_VERTS


class MixedSolver:
    def __init__(self, mesh, pE: int, pH: int, eps=None, mu=None):
        self.m = mesh
        self.pE, self.pH = pE, pH
        self.NE, self.NH = num_modes(pE), num_modes(pH)
        K = mesh.J.shape[0]
        self.K = K
        self.eps = np.ones(K) if eps is None else np.asarray(eps, float)
        self.mu = np.ones(K) if mu is None else np.asarray(mu, float)
        if np.any(self.eps <= 0) or np.any(self.mu <= 0):
            raise ValueError("material must be positive")
        self.absJ = np.abs(mesh.J)
        q = max(pE, pH) + 2
        self.xq, self.wq = tet_quadrature(q)
        self.VE, self.GE = eval_basis(pE, self.xq, grad=True)
        self.VH, self.GH = eval_basis(pH, self.xq, grad=True)
        st, self.wf = triangle_quadrature(q)
        lam = np.stack([1 - st[:, 0] - st[:, 1], st[:, 0], st[:, 1]], axis=1)
        self.lam = lam
        self.VfE, self.VfH = [], []
        for f in range(4):
            pts = lam @ _REF_VERTS[list(_FACE_LOCAL[f])]
            self.VfE.append(eval_basis(pE, pts))
            self.VfH.append(eval_basis(pH, pts))
        # neighbour values at the same physical points, through the neighbour's inverse map
        self._nb = []
        tets = mesh.tets
        for f in range(4):
            groups = {}
            own = tets[:, list(_FACE_LOCAL[f])]
            for e in np.nonzero(mesh.nbr[:, f] >= 0)[0]:
                e2, f2 = mesh.nbr[e, f], mesh.nbr_face[e, f]
                loc2 = _FACE_LOCAL[f2]
                ids2 = [int(tets[e2, v]) for v in loc2]
                corr = tuple(loc2[ids2.index(int(g))] for g in own[e])
                groups.setdefault(corr, []).append(e)
            ev = []
            for corr, es in groups.items():
                pts = lam @ _REF_VERTS[list(corr)]
                ev.append((np.asarray(es), eval_basis(pE, pts), eval_basis(pH, pts)))
            self._nb.append(ev)

    def _faces(self, coef, f, which):
        Vf = self.VfE[f] if which == "E" else self.VfH[f]
        own = np.einsum("aq,kad->kqd", Vf, coef)
        nb = np.full_like(own, np.nan)
        for es, VnE, VnH in self._nb[f]:
            Vn = VnE if which == "E" else VnH
            nb[es] = np.einsum("aq,kad->kqd", Vn, coef[self.m.nbr[es, f]])
        return own, nb

    def rhs_h(self, e_coef):
        """dH/dt (degree pH) from E (degree pE), strong form."""
        m = self.m
        gref = np.einsum("aqj,kal->kqjl", self.GE, e_coef, optimize=True)
        gphys = np.einsum("kjm,kqjl->kqml", m.Finv, gref, optimize=True)
        curl = np.stack([gphys[..., 1, 2] - gphys[..., 2, 1], gphys[..., 2, 0] - gphys[..., 0, 2],
                         gphys[..., 0, 1] - gphys[..., 1, 0]], axis=-1)
        wgt = self.absJ[:, None] * self.wq[None, :]
        r = -np.einsum("aq,kql->kal", self.VH, wgt[:, :, None] * curl, optimize=True)
        for f in range(4):
            own, nb = self._faces(e_coef, f, "E")
            wall = m.nbr[:, f] < 0
            nb[wall] = -own[wall]
            cross = np.cross(m.normal[:, f][:, None, :], nb - own)
            ds = 2.0 * m.area[:, f][:, None] * self.wf[None, :]
            r -= 0.5 * np.einsum("aq,kql->kal", self.VfH[f], ds[:, :, None] * cross, optimize=True)
        return r / (self.absJ * self.mu)[:, None, None]

    def rhs_e(self, h_coef):
        """dE/dt (degree pE) from H (degree pH), weak form."""
        m = self.m
        H = np.einsum("aq,kad->kqd", self.VH, h_coef)
        wgt = self.absJ[:, None] * self.wq[None, :]
        Y = np.cross(H[:, :, None, :], m.Finv[:, None, :, :]) * wgt[:, :, None, None]
        r = np.einsum("aqj,kqjl->kal", self.GE, Y, optimize=True)
        for f in range(4):
            own, nb = self._faces(h_coef, f, "H")
            wall = m.nbr[:, f] < 0
            nb[wall] = own[wall]
            cross = np.cross(m.normal[:, f][:, None, :], 0.5 * (own + nb))
            ds = 2.0 * m.area[:, f][:, None] * self.wf[None, :]
            r += np.einsum("aq,kql->kal", self.VfE[f], ds[:, :, None] * cross, optimize=True)
        return r / (self.absJ * self.eps)[:, None, None]

    def project(self, fn, which):
        """L2 projection (K, N, 3) of a physical field onto the E or H space."""
        V = self.VE if which == "E" else self.VH
        x = self.m.verts[self.m.tets[:, 0]][:, None, :] + np.einsum("kij,qj->kqi", self.m.F, self.xq)
        return np.einsum("aq,kqd->kad", V * self.wq[None, :], fn(x))

    def step(self, E, H, dt, nsteps=1):
        E, H = E.copy(), H.copy()
        for _ in range(nsteps):
            H = H + dt * self.rhs_h(E)
            E = E + dt * self.rhs_e(H)
        return E, H

    def mass_dot(self, a, b, which):
        w = self.absJ * (self.eps if which == "E" else self.mu)
        return float(np.einsum("k,kad,kad->", w, a, b))

    def energy(self, E, H):
        return 0.5 * self.mass_dot(E, E, "E") + 0.5 * self.mass_dot(H, H, "H")

    def leapfrog_invariant(self, E, H, dt):
        Hn1 = H + dt * self.rhs_h(E)
        return 0.5 * self.mass_dot(E, E, "E") + 0.5 * self.mass_dot(H, Hn1, "H")

    def rel_error(self, E, H, Eref, Href):
        num = self.mass_dot(E - Eref, E - Eref, "E") + self.mass_dot(H - Href, H - Href, "H")
        den = self.mass_dot(Eref, Eref, "E") + self.mass_dot(Href, Href, "H")
        return float(np.sqrt(num / den))

    def assemble(self):
        """Dense A_h (dH from E, (K NH 3) x (K NE 3)) and A_e (dE from H)."""
        nE, nH = self.K * self.NE * 3, self.K * self.NH * 3
        Ah, Ae = np.empty((nH, nE)), np.empty((nE, nH))
        for c in range(nE):
            u = np.zeros(nE)
            u[c] = 1.0
            Ah[:, c] = self.rhs_h(u.reshape(self.K, self.NE, 3)).ravel()
        for c in range(nH):
            u = np.zeros(nH)
            u[c] = 1.0
            Ae[:, c] = self.rhs_e(u.reshape(self.K, self.NH, 3)).ravel()
        return Ah, Ae

    def spectral_radius(self, iters: int, start):
        """Power iteration on H -> -dH(dE(H)) (start: NH-sized vector)."""
        x = np.asarray(start, float).reshape(self.K, self.NH, 3)
        lam = 0.0
        for _ in range(iters):
            y = -self.rhs_h(self.rhs_e(x))
            lam = self.mass_dot(x, y, "H") / self.mass_dot(x, x, "H")
            x = y / np.sqrt(self.mass_dot(y, y, "H"))
        return lam
