"""Plain FP64 central-flux DG solver for the loss-free Maxwell equations.

Test infrastructure only (see the package header).

State: physical Cartesian modal coefficients.  On element T with affine map
x = v0 + F xhat,  E|_T(x) = sum_a e_a phi_a(x),  e_a in R^3,  phi_a = phihat_a o Phi^{-1}.
Because the reference basis is orthonormal, int_T phi_a phi_b = |det F| delta_ab,
so the element mass matrix is |det F| eps I per mode (Section 3.3.1).

Semi-discrete equations (Section 2, element-wise integration by parts and the
central flux of Section 2.1, with the outer-normal signs of the consistent
reading; the printed flux terms carry the opposite sign on both equations):
  H-equation, strong form:
     (mu dH/dt, h)_T = -(curl E, h)_T - 1/2 (nu x (E_nb - E), h)_dT
  E-equation, weak form:
     (eps dE/dt, e)_T = (H, curl e)_T + (nu x {H}, e)_dT,   {H} = (H + H_nb)/2
Perfect conductor walls use ghost states E_nb = -E, H_nb = H.
Time stepping is symplectic Euler, H first (Section 3):
     H^{n+1} = H^n + dt dH(E^n),   E^{n+1} = E^n + dt dE(H^{n+1}).

Every integral is evaluated by Gauss quadrature in physical space; face
quadrature points are mapped onto the physical face, and the neighbour field
is evaluated there through the neighbour's own reference coordinates of those
points.  Nothing here uses the recurrences, traces or reference-frame tricks
of Section 3.2: it is the plain definition those tricks reproduce.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .basis import eval_basis, mode_list, num_modes, tet_quadrature, triangle_quadrature

_REF_VERTS = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
# local face f is the face opposite local vertex f; its vertices in increasing local index
_FACE_LOCAL = [tuple(v for v in range(4) if v != f) for f in range(4)]


@dataclass
class Mesh:
    verts: np.ndarray  # (nv,3)
    tets: np.ndarray  # (K,4) global vertex ids, in the caller's order
    F: np.ndarray  # (K,3,3) columns v1-v0, v2-v0, v3-v0
    Finv: np.ndarray
    J: np.ndarray  # signed det F
    nbr: np.ndarray  # (K,4) neighbour element or -1 (wall)
    nbr_face: np.ndarray  # (K,4) neighbour's local face or -1
    normal: np.ndarray  # (K,4,3) outward unit normal
    area: np.ndarray  # (K,4)


def build_mesh(verts, tets, tol: float = 1e-12) -> Mesh:
    verts = np.asarray(verts, dtype=np.float64)
    tets = np.asarray(tets, dtype=np.int64)
    K = tets.shape[0]
    P = verts[tets]  # (K,4,3)
    F = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    J = np.linalg.det(F)
    scale = np.max(np.linalg.norm(F, axis=1), axis=1) ** 3
    if np.any(np.abs(J) <= tol * scale):
        raise ValueError("degenerate tetrahedron")
    Finv = np.linalg.inv(F)
    faces = {}
    for e in range(K):
        for f in range(4):
            key = tuple(sorted(int(tets[e, v]) for v in _FACE_LOCAL[f]))
            faces.setdefault(key, []).append((e, f))
    nbr = -np.ones((K, 4), dtype=np.int64)
    nbf = -np.ones((K, 4), dtype=np.int64)
    for key, lst in faces.items():
        if len(lst) > 2:
            raise ValueError("non-manifold face")
        if len(lst) == 2:
            (e1, f1), (e2, f2) = lst
            nbr[e1, f1], nbf[e1, f1] = e2, f2
            nbr[e2, f2], nbf[e2, f2] = e1, f1
    normal = np.empty((K, 4, 3))
    area = np.empty((K, 4))
    for f in range(4):
        a, b, c = _FACE_LOCAL[f]
        n = np.cross(P[:, b] - P[:, a], P[:, c] - P[:, a])
        nn = np.linalg.norm(n, axis=1)
        n = n / nn[:, None]
        inward = np.einsum("kd,kd->k", n, P[:, f] - P[:, a]) > 0
        n[inward] *= -1.0
        normal[:, f] = n
        area[:, f] = 0.5 * nn
    return Mesh(verts, tets, F, Finv, J, nbr, nbf, normal, area)


class Solver:
    """Central-flux DG operator of order p on a mesh with per-element eps, mu."""

    def __init__(self, mesh: Mesh, p: int, eps=None, mu=None, chunk: int = 2048):
        self.m = mesh
        self.p = p
        self.N = num_modes(p)
        K = mesh.J.shape[0]
        self.K = K
        self.eps = np.ones(K) if eps is None else np.asarray(eps, float)
        self.mu = np.ones(K) if mu is None else np.asarray(mu, float)
        if np.any(self.eps <= 0) or np.any(self.mu <= 0):
            raise ValueError("material must be positive")
        self.absJ = np.abs(mesh.J)
        self.chunk = chunk
        q = p + 2
        self.xq, self.wq = tet_quadrature(q)
        self.V, self.G = eval_basis(p, self.xq, grad=True)  # (N,Q), (N,Q,3)
        st, self.wf = triangle_quadrature(q)
        self.st = st
        lam = np.stack([1 - st[:, 0] - st[:, 1], st[:, 0], st[:, 1]], axis=1)  # barycentric (Qf,3)
        self.lam = lam
        # self traces: reference face points of face f
        self.Vf = []
        for f in range(4):
            pts = lam @ _REF_VERTS[list(_FACE_LOCAL[f])]
            self.Vf.append(eval_basis(p, pts))
        # neighbour evaluation: group faces by (neighbour face, vertex correspondence)
        self._nb_groups = {}
        tets = mesh.tets
        for f in range(4):
            own = tets[:, list(_FACE_LOCAL[f])]  # (K,3) global ids of T's face vertices in T's order
            has = mesh.nbr[:, f] >= 0
            for e in np.nonzero(has)[0]:
                e2, f2 = mesh.nbr[e, f], mesh.nbr_face[e, f]
                loc2 = _FACE_LOCAL[f2]
                ids2 = [int(tets[e2, v]) for v in loc2]
                corr = tuple(loc2[ids2.index(int(g))] for g in own[e])  # nb local vertex for each of T's face vertices
                self._nb_groups.setdefault((f, corr), []).append(e)
        self._nb_eval = {}
        for (f, corr), es in self._nb_groups.items():
            pts = self.lam @ _REF_VERTS[list(corr)]
            self._nb_eval[(f, corr)] = (np.asarray(es), eval_basis(p, pts))

    # -- helpers -------------------------------------------------------------
    def check_neighbour_points(self, atol: float = 1e-9):
        """Recompute the neighbour's reference coordinates of every face quadrature
        point by inverting its affine map, and compare with the grouped points."""
        m = self.m
        worst = 0.0
        for (f, corr), (es, _) in self._nb_eval.items():
            pts_ref = self.lam @ _REF_VERTS[list(corr)]
            own_ref = self.lam @ _REF_VERTS[list(_FACE_LOCAL[f])]
            for e in es:
                x = m.verts[m.tets[e, 0]] + own_ref @ m.F[e].T
                e2 = m.nbr[e, f]
                xh2 = (x - m.verts[m.tets[e2, 0]]) @ m.Finv[e2].T
                worst = max(worst, float(np.abs(xh2 - pts_ref).max()))
        if worst > atol:
            raise AssertionError(f"neighbour point mismatch {worst}")
        return worst

    def project(self, fn):
        """L2 projection of a physical field fn(x[...,3]) -> [...,3]: coefficients (K,N,3)."""
        m = self.m
        out = np.empty((self.K, self.N, 3))
        for s in range(0, self.K, self.chunk):
            sl = slice(s, min(s + self.chunk, self.K))
            x = m.verts[m.tets[sl, 0]][:, None, :] + np.einsum("kij,qj->kqi", m.F[sl], self.xq)
            vals = fn(x)  # (k,Q,3)
            # int_T f phi_a = |J| sum_q w_q f(x_q) phihat_a(xhat_q); divide by |J| (mass)
            out[sl] = np.einsum("aq,kqd->kad", self.V * self.wq[None, :], vals)
        return out

    def evaluate(self, coef, xhat_elem):
        """Evaluate the field of element e at reference point xhat: used by tests."""
        e, xh = xhat_elem
        V = eval_basis(self.p, np.atleast_2d(xh))
        return np.einsum("aq,ad->qd", V, coef[e])

    def _face_values(self, coef, f):
        """Self values (K,Qf,3) and neighbour values (K,Qf,3, NaN on walls) on face f."""
        own = np.einsum("aq,kad->kqd", self.Vf[f], coef)
        nb = np.full_like(own, np.nan)
        for (ff, corr), (es, Vn) in self._nb_eval.items():
            if ff != f:
                continue
            e2 = self.m.nbr[es, f]
            nb[es] = np.einsum("aq,kad->kqd", Vn, coef[e2])
        return own, nb

    # -- right-hand sides ----------------------------------------------------
    def rhs_h(self, e_coef):
        """dH/dt from E (strong form).  Returns (K,N,3)."""
        m = self.m
        r = np.zeros((self.K, self.N, 3))
        for s in range(0, self.K, self.chunk):
            sl = slice(s, min(s + self.chunk, self.K))
            # reference gradient of each physical component: gref[k,q,j,l] = d_j E_l
            gref = np.einsum("aqj,kal->kqjl", self.G, e_coef[sl], optimize=True)
            # physical gradient d_m E_l = sum_j Finv[j,m] d_j E_l
            gphys = np.einsum("kjm,kqjl->kqml", m.Finv[sl], gref, optimize=True)
            # (curl E)_l = eps_lmn d_m E_n
            curl = np.stack([gphys[..., 1, 2] - gphys[..., 2, 1],
                             gphys[..., 2, 0] - gphys[..., 0, 2],
                             gphys[..., 0, 1] - gphys[..., 1, 0]], axis=-1)
            wgt = self.absJ[sl][:, None] * self.wq[None, :]
            r[sl] -= np.einsum("aq,kql->kal", self.V, wgt[:, :, None] * curl, optimize=True)
        for f in range(4):
            own, nb = self._face_values(e_coef, f)
            wall = m.nbr[:, f] < 0
            nb[wall] = -own[wall]
            jump = nb - own
            nu = m.normal[:, f]
            cross = np.cross(nu[:, None, :], jump)  # (K,Qf,3)
            ds = 2.0 * m.area[:, f][:, None] * self.wf[None, :]
            r -= 0.5 * np.einsum("aq,kql->kal", self.Vf[f], ds[:, :, None] * cross, optimize=True)
        return r / (self.absJ * self.mu)[:, None, None]

    def rhs_e(self, h_coef):
        """dE/dt from H (weak form).  Returns (K,N,3)."""
        m = self.m
        r = np.zeros((self.K, self.N, 3))
        for s in range(0, self.K, self.chunk):
            sl = slice(s, min(s + self.chunk, self.K))
            H = np.einsum("aq,kad->kqd", self.V, h_coef[sl])  # (k,Q,3)
            wgt = self.absJ[sl][:, None] * self.wq[None, :]
            # (H x grad phi_a)_l = eps_lmn H_m (grad phi_a)_n,  grad phi_a = Finv^T ghat_a
            # Y[k,q,j,:] = w_q |J| (H x row_j(Finv))
            Y = np.cross(H[:, :, None, :], m.Finv[sl][:, None, :, :]) * wgt[:, :, None, None]
            r[sl] += np.einsum("aqj,kqjl->kal", self.G, Y, optimize=True)
        for f in range(4):
            own, nb = self._face_values(h_coef, f)
            wall = m.nbr[:, f] < 0
            nb[wall] = own[wall]
            avg = 0.5 * (own + nb)
            nu = m.normal[:, f]
            cross = np.cross(nu[:, None, :], avg)
            ds = 2.0 * m.area[:, f][:, None] * self.wf[None, :]
            r += np.einsum("aq,kql->kal", self.Vf[f], ds[:, :, None] * cross, optimize=True)
        return r / (self.absJ * self.eps)[:, None, None]

    # -- time stepping and energies -----------------------------------------
    def step(self, E, H, dt, nsteps=1):
        """Symplectic Euler, H first (Section 3).  Returns new (E, H)."""
        E = E.copy()
        H = H.copy()
        for _ in range(nsteps):
            H = H + dt * self.rhs_h(E)
            E = E + dt * self.rhs_e(H)
        return E, H

    def mass_dot(self, a, b, which):
        w = self.absJ * (self.eps if which == "E" else self.mu)
        return float(np.einsum("k,kad,kad->", w, a, b))

    def energy(self, E, H):
        """W = 1/2 (eps E, E) + 1/2 (mu H, H)  (Section 2.1)."""
        return 0.5 * self.mass_dot(E, E, "E") + 0.5 * self.mass_dot(H, H, "H")

    def leapfrog_invariant(self, E, H, dt):
        """Q^n = 1/2 (E^n, M_eps E^n) + 1/2 (H^n, M_mu H^{n+1}), conserved exactly by the
        H-first symplectic Euler step (expand one step: the dt^2 terms cancel)."""
        Hn1 = H + dt * self.rhs_h(E)
        return 0.5 * self.mass_dot(E, E, "E") + 0.5 * self.mass_dot(H, Hn1, "H")

    def rel_error(self, E, H, Eref, Href):
        """Relative error in the energy norm ||u - u_ref||_M / ||u_ref||_M."""
        num = self.mass_dot(E - Eref, E - Eref, "E") + self.mass_dot(H - Href, H - Href, "H")
        den = self.mass_dot(Eref, Eref, "E") + self.mass_dot(Href, Href, "H")
        return float(np.sqrt(num / den))

    # -- representation change ----------------------------------------------
    def to_covariant(self, coef):
        """Reference covariant coefficients: ehat_a = F^T e_a (the field is F^{-T} ehat)."""
        return np.einsum("kji,kaj->kai", self.m.F, coef)

    def from_covariant(self, chat):
        return np.einsum("kji,kaj->kai", self.m.Finv, chat)

    # -- dense operators on tiny meshes -------------------------------------
    def assemble(self):
        """Dense matrices A_h (dH/dt from E) and A_e (dE/dt from H), in the flattened
        (K,N,3) coefficient order."""
        n = self.K * self.N * 3
        Ah = np.empty((n, n))
        Ae = np.empty((n, n))
        for c in range(n):
            u = np.zeros(n)
            u[c] = 1.0
            U = u.reshape(self.K, self.N, 3)
            Ah[:, c] = self.rhs_h(U).ravel()
            Ae[:, c] = self.rhs_e(U).ravel()
        return Ah, Ae

    def spectral_radius(self, iters: int, start):
        """Power iteration (Section 3) on H -> -dH(dE(H)), whose spectrum is that of
        M_mu^{-1/2} C M_eps^{-1} C^T M_mu^{-1/2}; returns the Rayleigh estimate."""
        x = np.asarray(start, float).reshape(self.K, self.N, 3)
        lam = 0.0
        for _ in range(iters):
            y = -self.rhs_h(self.rhs_e(x))
            lam = self.mass_dot(x, y, "H") / self.mass_dot(x, x, "H")
            x = y / np.sqrt(self.mass_dot(y, y, "H"))
        return lam

    def modes(self):
        return mode_list(self.p)
