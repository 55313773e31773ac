"""Set-up helpers on the host (FP64): initial data in the library's layout.

The L2 projection of a physical field f onto the covariant space of element T
(Section 3.2.1: u = F^{-T} uhat o Phi^{-1}) has coefficients
    uhat_m = F^T int_That f(Phi(xhat)) phi_m(xhat) dxhat,
because the element mass matrix is |det F| F^{-1} F^{-T} (x) I (Section 3.3.1).
F is built from the element's vertices sorted by global id, as in the library.
"""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np

from .gen import basis as B


def sorted_geometry(verts, tets):
    """(tets sorted per row, v0 (K,3), F (K,3,3) with columns v1-v0, v2-v0, v3-v0)."""
    verts = np.asarray(verts, dtype=np.float64)
    ts = np.sort(np.asarray(tets, dtype=np.int64), axis=1)
    P = verts[ts]
    F = np.stack([P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]], axis=2)
    return ts, P[:, 0], F


def project_covariant(verts, tets, p: int, fn, chunk: int = 4096) -> np.ndarray:
    """Covariant coefficients (3, N, K) of the L2 projection of fn(x[...,3]) -> [...,3]."""
    _, v0, F = sorted_geometry(verts, tets)
    xq, wq = B.collapsed_rule_tet(p + 2)
    V = B.volume_values(p, xq)
    K = F.shape[0]
    out = np.empty((3, V.shape[0], K))
    W = np.ascontiguousarray((V * wq[None, :]).T)  # (Q, N) quadrature weights times basis values

    def part(s):
        sl = slice(s, min(s + chunk, K))
        x = v0[sl, None, :] + sum(xq[None, :, j, None] * F[sl, None, :, j] for j in range(3))
        f = fn(x)
        mom = np.matmul(f.transpose(0, 2, 1), W)  # (k, 3, N): int f phi_m over the reference tet
        out[:, :, sl] = np.matmul(F[sl].transpose(0, 2, 1), mom).transpose(1, 2, 0)  # F^T per mode

    starts = list(range(0, K, chunk))
    if len(starts) > 1:
        # numpy releases the GIL in its ufuncs and matrix products: chunks run in parallel
        with cf.ThreadPoolExecutor(max_workers=min(len(starts), os.cpu_count() or 1, 16)) as ex:
            list(ex.map(part, starts))
    else:
        part(0)
    return out


def covariant_from_physical(verts, tets, coef_phys) -> np.ndarray:
    """Physical Cartesian modal coefficients (K, N, 3) -> covariant (3, N, K): uhat = F^T u."""
    _, _, F = sorted_geometry(verts, tets)
    return np.einsum("kji,kmj->imk", F, np.asarray(coef_phys, dtype=np.float64))
