"""Pins of the oracle's approximate mass inverse for material varying inside the
elements (Section 3.3.2): exactness for constant material, symmetry and positivity,
second-order agreement with the exact inverse as elements shrink, and an exactly
conserved leapfrog invariant in the inner product the approximation defines."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.varcoef import VarMaterialSolver

V0 = np.array([[0.0, 0, 0], [1, 0.1, 0], [0.2, 1, 0], [0.1, 0.2, 1]])


def matrices(s, which="E"):
    """Approximate and exact inverses of one element as N x N matrices (one component)."""
    cols_a, cols_e = [], []
    for c in range(s.N):
        f = np.zeros((1, s.N, 3))
        f[0, c, :] = 1.0
        cols_a.append(s.approx_inverse(f, which)[0, :, 0])
        cols_e.append(s.exact_inverse(f, which)[0, :, 0])
    return np.stack(cols_a, 1), np.stack(cols_e, 1)


def test_constant_material_gives_the_flat_method():
    """Material constant on each element: the approximate inverse is the exact one, and
    both phases equal the flat central-flux solver's."""
    rng = np.random.default_rng(1)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    ts = np.sort(tets, axis=1)
    K = ts.shape[0]
    eps, mu = rng.uniform(1, 4, K), rng.uniform(1, 2, K)
    s = VarMaterialSolver(oracle.build_mesh(verts, ts), 3, np.repeat(eps[:, None], 4, 1), np.repeat(mu[:, None], 4, 1))
    flat = oracle.Solver(oracle.build_mesh(verts, ts), 3, eps, mu)
    E = rng.standard_normal((K, s.N, 3))
    assert np.abs(s.rhs_h(E) - flat.rhs_h(E)).max() < 1e-12 * np.abs(flat.rhs_h(E)).max()
    assert np.abs(s.rhs_e(E) - flat.rhs_e(E)).max() < 1e-12 * np.abs(flat.rhs_e(E)).max()


def test_approximate_inverse_is_spd_and_second_order():
    """For eps linear on a shrinking element, M~^{-1} M -> I at second order in the size;
    M~^{-1} is symmetric positive definite at every size."""
    g = np.array([0.7, -0.4, 0.5])
    errs = []
    for sc in (1.0, 0.5, 0.25):
        v = V0 * sc + np.array([0.3, 0.2, 0.1])
        eps_v = (1.0 + v @ g)[None, :]
        s = VarMaterialSolver(oracle.build_mesh(v, np.array([[0, 1, 2, 3]])), 3, eps_v, np.ones((1, 4)))
        A, Ex = matrices(s)
        assert np.abs(A - A.T).max() < 1e-12 * np.abs(A).max()
        assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() > 0
        errs.append(np.abs(A @ np.linalg.inv(Ex) - np.eye(s.N)).max())
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)


def _var_mesh(rng, n=2, p=2):
    verts, tets = synth.kuhn_mesh(n, 0.1, rng)
    ts = np.sort(tets, axis=1)
    epsf = lambda x: 1.5 + 0.5 * np.sin(2.0 * x[..., 0]) + 0.4 * x[..., 1]
    muf = lambda x: 1.0 + 0.3 * x[..., 2]
    return VarMaterialSolver(oracle.build_mesh(verts, ts), p, epsf(verts[ts]), muf(verts[ts])), verts, ts


def test_skew_in_the_approximate_mass_inner_product():
    rng = np.random.default_rng(3)
    s, _, _ = _var_mesh(rng, 1, 2)
    Ah, Ae = s.assemble()
    Mh, Me = s.mass_approx("H"), s.mass_approx("E")
    n = s.K * s.N * 3
    Mhf, Mef = np.zeros((n, n)), np.zeros((n, n))
    for k in range(s.K):
        for d in range(3):
            idx = k * s.N * 3 + np.arange(s.N) * 3 + d
            Mhf[np.ix_(idx, idx)] = Mh[k]
            Mef[np.ix_(idx, idx)] = Me[k]
    S = Mhf @ Ah
    assert np.abs(S + (Mef @ Ae).T).max() < 1e-12 * np.abs(S).max()


def test_leapfrog_invariant_conserved_with_variable_material():
    rng = np.random.default_rng(4)
    s, _, _ = _var_mesh(rng, 2, 2)
    E = s.project(synth.te101().E)
    H = np.zeros_like(E)
    dt = 1.0 / math.sqrt(s.spectral_radius(40, synth.splitmix64(4, E.size)))
    Q0 = s.leapfrog_invariant(E, H, dt)
    worst = 0.0
    for _ in range(5):
        E, H = s.step(E, H, dt, 10)
        worst = max(worst, abs(s.leapfrog_invariant(E, H, dt) - Q0) / Q0)
    assert worst < 1e-13
