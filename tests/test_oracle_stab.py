"""Pins of the oracle's stabilised central flux with face unknowns (Section 2.1).

Each check is against something other than the oracle itself: an identity of the
continuous problem (skew-symmetry, exact conservation of the leapfrog invariant),
a closed-form count (the null space), the exact PEC cube eigenvalues, the central
flux it must reduce to, or a polynomial field whose tangential jumps vanish.
"""
import math

import numpy as np
import pytest
import scipy.special as sps

import oracle
import synth
from oracle.stab import StabilizedSolver, triangle_basis


def cube(p, n=1, jitter=0.0, seed=0, **kw):
    rng = np.random.default_rng(seed)
    verts, tets = synth.kuhn_mesh(n, jitter, rng if jitter else None)
    return StabilizedSolver(oracle.build_mesh(verts, np.sort(tets, axis=1)), p, **kw)


def test_triangle_basis_orthonormal_against_scipy_quadrature():
    """Orthonormal on the unit triangle, integrated with scipy's Gauss-Jacobi rule (not the
    oracle's), and equal to the printed two-dimensional formula at random points."""
    p = 5
    xa, wa = sps.roots_jacobi(p + 2, 1, 0)
    xb, wb = sps.roots_jacobi(p + 2, 0, 0)
    A, Bq = np.meshgrid(xa, xb, indexing="ij")
    st = np.stack([((1 + A) / 2).ravel(), ((1 + Bq) * (1 - A) / 4).ravel()], 1)
    w = (wa[:, None] * wb[None, :]).ravel() / 8
    P = triangle_basis(p, st)
    assert np.abs((P * w) @ P.T - np.eye(P.shape[0])).max() < 1e-12
    rng = np.random.default_rng(3)
    s = rng.uniform(0, 0.9, 20)
    t = rng.uniform(0, 1, 20) * (1 - s)
    Q = triangle_basis(p, np.stack([s, t], 1))
    r = 0
    for n in range(p + 1):
        for a in range(n + 1):
            b = n - a
            ref = (sps.eval_legendre(a, 2 * t / (1 - s) - 1) * (1 - s) ** a * sps.eval_jacobi(b, 2 * a + 1, 0, 2 * s - 1)
                   * math.sqrt((2 * a + 1) * (2 * a + 2 * b + 2)))
            assert np.allclose(Q[r], ref, rtol=1e-12, atol=1e-12)
            r += 1


def _full_operator(s):
    Ah, Af, Ae, Ab = s.assemble_stab()
    n, nb = Ah.shape[0], Af.shape[0]
    Z = np.zeros
    A = np.block([[Z((n, n)), Ae, Ab], [Ah, Z((n, n)), Z((n, nb))], [Af, Z((nb, n)), Z((nb, nb))]])
    M = np.concatenate([np.repeat(s.absJ * s.eps, 3 * s.N), np.repeat(s.absJ * s.mu, 3 * s.N),
                        np.repeat(s.hF / s.alpha, 3 * s.NF)])
    return A, M, (Ah, Af, Ae, Ab)


@pytest.mark.parametrize("jitter,seed", [(0.0, 0), (0.15, 4)])
def test_stabilised_system_is_skew(jitter, seed):
    """M A is antisymmetric: the energy with the face term is conserved (Section 2.1)."""
    rng = np.random.default_rng(seed)
    verts, tets = synth.kuhn_mesh(1, jitter, rng if jitter else None)
    K = tets.shape[0]
    s = StabilizedSolver(oracle.build_mesh(verts, np.sort(tets, axis=1)), 2, rng.uniform(1, 4, K), rng.uniform(1, 2, K))
    A, M, _ = _full_operator(s)
    S = M[:, None] * A
    assert np.abs(S + S.T).max() < 1e-13 * np.abs(S).max()


def _kernel_dim(p):
    """Continuous fields of degree q = p + 1 vanishing on the boundary of one Kuhn cell
    (1 interior edge, 6 interior faces, 6 tetrahedra): their gradients are exactly the
    static fields the stabilised operator keeps (no tangential jump anywhere)."""
    q = p + 1
    return (q - 1) + 6 * (q - 1) * (q - 2) // 2 + 6 * (q - 1) * (q - 2) * (q - 3) // 6


@pytest.mark.parametrize("p", [1, 2, 3])
def test_null_space_is_the_continuous_gradients(p):
    s = cube(p)
    _, _, (Ah, Af, Ae, Ab) = _full_operator(s)
    ev = np.linalg.eigvals(-(Ae @ Ah + Ab @ Af)).real
    scale = ev.max()
    assert np.sum(np.abs(ev) < 1e-9 * scale) == _kernel_dim(p)


@pytest.mark.parametrize("p", [3, 4])
def test_spurious_modes_removed_cavity_modes_kept(p):
    """Six-tet unit cube: the stabilised spectrum starts at the cavity eigenvalues
    2 pi^2 (x3) and 3 pi^2 (x2) with nothing below, while the central flux at the same
    order has eigenvalues below 1.9 pi^2 that belong to no cavity mode."""
    s = cube(p)
    _, _, (Ah, Af, Ae, Ab) = _full_operator(s)
    ev = np.sort(np.linalg.eigvals(-(Ae @ Ah + Ab @ Af)).real) / np.pi ** 2
    nz = ev[ev > 1e-6]
    tol2, tol3 = (0.05, 0.06) if p == 3 else (0.002, 0.015)
    assert nz[0] > 2 * (1 - tol2)
    assert np.all(np.abs(nz[:3] - 2) < 2 * tol2) and np.all(np.abs(nz[3:5] - 3) < 3 * tol3)
    evc = np.sort(np.linalg.eigvals(-(Ae @ Ah)).real) / np.pi ** 2
    assert np.any((evc > 1e-6) & (evc < 1.9))


def test_reduces_to_central_flux():
    """With H^F = 0 the E update is the central one; a continuous E with zero tangential
    trace on the walls has no tangential jump, so H^F does not move."""
    rng = np.random.default_rng(5)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    s = StabilizedSolver(oracle.build_mesh(verts, np.sort(tets, axis=1)), 4)
    H = rng.standard_normal((s.K, s.N, 3))
    assert np.abs(s.rhs_e_stab(H, s.zeros_faces()) - s.rhs_e(H)).max() < 1e-12 * np.abs(s.rhs_e(H)).max()
    E = s.project(lambda x: np.stack([0 * x[..., 0], x[..., 0] * (1 - x[..., 0]) * x[..., 2] * (1 - x[..., 2]),
                                      0 * x[..., 0]], -1))
    g = s.rhs_faces(E)
    assert np.abs(g).max() < 1e-11 * s.alpha / s.hF.min()
    # while a random field's jumps do move it
    assert np.abs(s.rhs_faces(rng.standard_normal(E.shape))).max() > 1.0


def test_leapfrog_invariant_with_face_unknowns_conserved():
    rng = np.random.default_rng(6)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    s = StabilizedSolver(oracle.build_mesh(verts, np.sort(tets, axis=1)), 2, rng.choice([1.0, 4.0], K), None)
    E = s.project(synth.te101().E)
    H = np.zeros_like(E)
    b = s.zeros_faces()
    rho = s.spectral_radius_stab(40, synth.splitmix64(6, E.size))
    dt = 1.0 / math.sqrt(rho)
    Q0 = s.leapfrog_invariant_stab(E, H, b, dt)
    W0 = s.energy_stab(E, H, b)
    worst, wmax = 0.0, 0.0
    for _ in range(10):
        E, H, b = s.step_stab(E, H, b, dt, 10)
        worst = max(worst, abs(s.leapfrog_invariant_stab(E, H, b, dt) - Q0) / Q0)
        wmax = max(wmax, abs(s.energy_stab(E, H, b) - W0) / W0)
    assert worst < 1e-13
    assert wmax < 0.5  # W oscillates at O(dt) around the conserved Q
    assert np.abs(b).max() > 0  # the face unknowns are excited


def test_te101_converges_with_stabilised_flux():
    """TE101 at T = 0.5: the error falls at least like h^p (p = 2) under refinement."""
    p, T = 2, 0.5
    errs = []
    for n in (2, 4):
        s = cube(p, n)
        mode = synth.te101()
        w = mode.omega
        rho = s.spectral_radius_stab(30, synth.splitmix64(7, 3 * s.N * s.K))
        steps = int(math.ceil(T / (0.25 / math.sqrt(rho))))
        dt = T / steps
        E = s.project(mode.E)
        H = s.project(lambda x: mode.H(x, -dt / 2))
        E, H, b = s.step_stab(E, H, s.zeros_faces(), dt, steps)
        Er, Hr = s.project(lambda x: mode.E(x, T)), s.project(lambda x: mode.H(x, T - dt / 2))
        errs.append(s.rel_error(E, H, Er, Hr))
    rate = math.log2(errs[0] / errs[1])
    assert rate > p - 0.3, (errs, rate)
