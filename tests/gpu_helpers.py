"""Shared helpers of the GPU parity tests: the oracle on the same (sorted-vertex)
elements, representation changes, and patch meshes for sampled checks."""
import numpy as np

import oracle
from paper_1104_4208_amd.gen.basis import volume_modes


def sort_tets(tets):
    return np.sort(np.asarray(tets, dtype=np.int64), axis=1)


def frames(verts, tets):
    ts = sort_tets(tets)
    P = np.asarray(verts, float)[ts]
    return np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)


def perm(p, solver):
    """Oracle mode rows in the library's order (matched by (i, j, k))."""
    idx = {m: r for r, m in enumerate(solver.modes())}
    return np.array([idx[m] for m in volume_modes(p)])


def inv_perm(pm):
    out = np.empty_like(pm)
    out[pm] = np.arange(len(pm))
    return out


class Pair:
    """The oracle on the library's elements plus conversions between the oracle's
    physical (K,N,3) coefficients and the library's covariant (3,N,K) layout."""

    def __init__(self, verts, tets, p, eps=None, mu=None):
        self.verts = np.asarray(verts, float)
        self.tets = np.asarray(tets, np.int64)
        self.s = oracle.Solver(oracle.build_mesh(self.verts, sort_tets(tets)), p, eps, mu)
        self.F = frames(verts, tets)
        self.pm = perm(p, self.s)
        self.ipm = inv_perm(self.pm)

    def to_cov(self, phys):
        return np.einsum("kji,kmj->imk", self.F, phys)[:, self.pm, :]

    def to_phys(self, cov):
        c = np.asarray(cov, float)[:, self.ipm, :]
        Finv = np.linalg.inv(self.F)
        return np.einsum("kji,jmk->kmi", Finv, c)


def rel_err(a, b):
    a = np.asarray(a, float)
    b = np.asarray(b, float)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def patch(tets, centers):
    """Sub-mesh made of the given elements and all their face neighbours.
    Returns (patch tets, index of each center in the patch)."""
    ts = sort_tets(tets)
    faces = {}
    for e in range(ts.shape[0]):
        for f in range(4):
            faces.setdefault(tuple(int(ts[e, v]) for v in range(4) if v != f), []).append(e)
    keep = []
    for c in centers:
        keep.append(int(c))
        for f in range(4):
            for e in faces[tuple(int(ts[c, v]) for v in range(4) if v != f)]:
                keep.append(e)
    keep = list(dict.fromkeys(keep))
    pos = {e: r for r, e in enumerate(keep)}
    return np.asarray(keep), ts[keep], [pos[int(c)] for c in centers]
