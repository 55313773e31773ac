"""CPU model (numpy, FP64) of the arithmetic the generated phase kernels perform.

Test helper only: it applies the product's tables (paper_1104_4208_amd.gen) the
way the kernels do -- derivative frame, stored frame, tangential-trace jumps,
lift -- so the formulation can be checked against the oracle on the CPU before
any GPU run.  It does not run on the product path.
"""
import numpy as np

from paper_1104_4208_amd.gen import tables as TB
from paper_1104_4208_amd.project import sorted_geometry

CYC = {0: (1, 2), 1: (2, 0), 2: (0, 1)}


def neighbours(tets_sorted):
    K = tets_sorted.shape[0]
    faces = {}
    for e in range(K):
        for f in range(4):
            key = tuple(int(tets_sorted[e, v]) for v in range(4) if v != f)
            faces.setdefault(key, []).append((e, f))
    code = -np.ones((4, K), dtype=np.int64)
    for lst in faces.values():
        if len(lst) == 2:
            (a, fa), (b, fb) = lst
            code[fa, a] = 4 * b + fb
            code[fb, b] = 4 * a + fa
    return code


class Model:
    def __init__(self, verts, tets, p, eps=None, mu=None):
        self.t = TB.build(p)
        self.g, self.Lp = TB.face_weights(self.t)
        fr = TB.frame()
        self.A, self.Ainv, self.detA = fr["A"], fr["Ainv"], fr["detA"]
        ts, _, F = sorted_geometry(verts, tets)
        self.K = F.shape[0]
        self.J = np.linalg.det(F)
        self.code = neighbours(ts)
        eps = np.ones(self.K) if eps is None else np.asarray(eps, float)
        mu = np.ones(self.K) if mu is None else np.asarray(mu, float)
        FtF = np.einsum("kqr,kqs->krs", F, F)
        self.M = []
        for c in (eps, mu):
            Kf = FtF / (c * self.J)[:, None, None]
            self.M.append(np.einsum("rq,kqs,ts->krt", self.A, Kf, self.A) / self.detA)

    def rate(self, U_cov, fld_u):
        """Covariant rate of the other field from covariant U (3,N,K): fld_u 0 = E -> dH."""
        t = self.t
        M = self.M[fld_u]
        w = np.einsum("rq,qnk->rnk", self.A, U_cov)  # w = A uhat (equals M S)
        tau = np.zeros((4, 2, t.NF, self.K))
        for f in range(4):
            for k in range(2):
                q = np.einsum("r,rnk->nk", self.g[f][k], w)
                tau[f, k] = t.T[f] @ q
        jump = np.zeros_like(tau)
        wall = -1.0 if fld_u == 0 else 1.0
        for f in range(4):
            for e in range(self.K):
                c = self.code[f, e]
                if c < 0:
                    jump[f, :, :, e] = (wall - 1.0) * tau[f, :, :, e]
                else:
                    jump[f, :, :, e] = tau[c & 3, :, :, c >> 2] - tau[f, :, :, e]
        rate = np.zeros((3, t.N, self.K))
        for k in range(3):
            i, j = CYC[k]
            rate[k] = t.D[i] @ w[j] - t.D[j] @ w[i]
            for f in range(4):
                gf = self.Lp[f][k][0] * jump[f, 0] + self.Lp[f][k][1] * jump[f, 1]
                rate[k] += t.T[f].T @ gf
        sgn = -1.0 if fld_u == 0 else 1.0
        Mo = self.M[1 - fld_u]
        # stored-frame rate -> covariant: uhat = A^{-1} M S
        return sgn * np.einsum("rq,kqs,snk->rnk", self.Ainv, Mo, rate)
