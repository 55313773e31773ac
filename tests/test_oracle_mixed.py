"""Pins of the oracle's mixed-order solver (E of degree p+1, H of degree p; Section 2).

Checks against things other than the oracle: skew-symmetry of the semi-discrete system,
exact curl of global polynomials (both phases), exact conservation of the leapfrog
invariant, the exact PEC cube eigenvalues with no spurious mode below the first one (the
equal-order central flux has several there), and h-convergence to TE101.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle.mixed import MixedSolver


def mixed(pH, n=1, jitter=0.0, seed=0, eps=None, mu=None):
    rng = np.random.default_rng(seed)
    verts, tets = synth.kuhn_mesh(n, jitter, rng if jitter else None)
    return MixedSolver(oracle.build_mesh(verts, np.sort(tets, axis=1)), pH + 1, pH, eps, mu)


@pytest.mark.parametrize("pH,jitter", [(1, 0.0), (2, 0.15)])
def test_mixed_system_is_skew(pH, jitter):
    rng = np.random.default_rng(3)
    s = mixed(pH, 1, jitter, 4, rng.uniform(1, 4, 6), rng.uniform(1, 2, 6))
    Ah, Ae = s.assemble()
    wE = np.repeat(s.absJ * s.eps, 3 * s.NE)
    wH = np.repeat(s.absJ * s.mu, 3 * s.NH)
    S = wH[:, None] * Ah
    assert np.abs(S + (wE[:, None] * Ae).T).max() < 1e-13 * np.abs(S).max()


def test_polynomial_fields_give_exact_curls():
    """A global polynomial H of degree pH has no jumps: the E phase returns curl H.  The
    field E = (0, x(1-x) z(1-z), 0) (degree 4 = pE) is continuous with zero tangential
    trace on the walls: the H phase returns -curl E, which has degree 3 = pH."""
    rng = np.random.default_rng(8)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    s = MixedSolver(oracle.build_mesh(verts, np.sort(tets, axis=1)), 4, 3)
    c = rng.standard_normal((3, 4))

    def Hf(x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        mon = [X * Y * Z, X ** 2 * Y, Z ** 3, Y * Z]
        return np.stack([sum(c[d, q] * mon[q] for q in range(4)) for d in range(3)], -1)

    def curlHf(x):
        X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
        # d/dx, d/dy, d/dz of each monomial
        dm = [(Y * Z, X * Z, X * Y), (2 * X * Y, X ** 2, 0 * X), (0 * X, 0 * X, 3 * Z ** 2), (0 * X, Z, Y)]
        g = [[sum(c[d, q] * dm[q][j] for q in range(4)) for j in range(3)] for d in range(3)]  # g[d][j] = dH_d/dx_j
        return np.stack([g[2][1] - g[1][2], g[0][2] - g[2][0], g[1][0] - g[0][1]], -1)

    H = s.project(Hf, "H")
    ref = s.project(curlHf, "E") / s.eps[:, None, None]
    assert np.abs(s.rhs_e(H) - ref).max() < 1e-11 * np.abs(ref).max()
    E = s.project(lambda x: np.stack([0 * x[..., 0], x[..., 0] * (1 - x[..., 0]) * x[..., 2] * (1 - x[..., 2]),
                                      0 * x[..., 0]], -1), "E")

    def curlE(x):
        X, Z = x[..., 0], x[..., 2]
        Ey_z = X * (1 - X) * (1 - 2 * Z)
        Ey_x = (1 - 2 * X) * Z * (1 - Z)
        return np.stack([-Ey_z, 0 * X, Ey_x], -1)

    refh = -s.project(curlE, "H")
    assert np.abs(s.rhs_h(E) - refh).max() < 1e-11 * np.abs(refh).max()


def test_mixed_leapfrog_invariant_conserved():
    rng = np.random.default_rng(9)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    s = MixedSolver(oracle.build_mesh(verts, np.sort(tets, axis=1)), 3, 2, rng.choice([1.0, 4.0], K), None)
    E = s.project(synth.te101().E, "E")
    H = np.zeros((K, s.NH, 3))
    dt = 1.0 / math.sqrt(s.spectral_radius(40, synth.splitmix64(9, H.size)))
    Q0 = s.leapfrog_invariant(E, H, dt)
    worst = 0.0
    for _ in range(10):
        E, H = s.step(E, H, dt, 10)
        worst = max(worst, abs(s.leapfrog_invariant(E, H, dt) - Q0) / Q0)
    assert worst < 1e-13


@pytest.mark.parametrize("pH", [1, 2, 3])
def test_no_spurious_modes_below_the_first_cavity_mode(pH):
    """Six-tet unit cube: with E one degree higher the spectrum of the H-side operator
    has no eigenvalue between 0 and 2 pi^2; at pH = 3 it starts with the cavity
    eigenvalues 2 pi^2 (x3, within 1 %) and 3 pi^2 (x2, within 5 %).  The equal-order
    central flux at the same pH has eigenvalues below 1.9 pi^2."""
    s = mixed(pH)
    Ah, Ae = s.assemble()
    ev = np.sort(np.linalg.eigvals(-(Ah @ Ae)).real) / np.pi ** 2
    nz = ev[ev > 1e-6]
    assert nz[0] > 2.0
    if pH == 3:
        assert np.all(np.abs(nz[:3] - 2) < 0.02) and np.all(np.abs(nz[3:5] - 3) < 0.15)
    verts, tets = synth.kuhn_mesh(1)
    eq = oracle.Solver(oracle.build_mesh(verts, np.sort(tets, axis=1)), pH)
    Ah2, Ae2 = eq.assemble()
    ev2 = np.sort(np.linalg.eigvals(-(Ah2 @ Ae2)).real) / np.pi ** 2
    assert np.any((ev2 > 1e-6) & (ev2 < 1.9))


def test_te101_converges_with_mixed_orders():
    """TE101 at T = 0.5 with (pE, pH) = (3, 2): the energy-norm error falls at least like h^2."""
    pH, T = 2, 0.5
    errs = []
    for n in (2, 4):
        s = mixed(pH, n)
        mode = synth.te101()
        rho = s.spectral_radius(30, synth.splitmix64(7, 3 * s.NH * s.K))
        steps = int(math.ceil(T / (0.25 / math.sqrt(rho))))
        dt = T / steps
        E = s.project(mode.E, "E")
        H = s.project(lambda x: mode.H(x, -dt / 2), "H")
        E, H = s.step(E, H, dt, steps)
        errs.append(s.rel_error(E, H, s.project(lambda x: mode.E(x, T), "E"), s.project(lambda x: mode.H(x, T - dt / 2), "H")))
    rate = math.log2(errs[0] / errs[1])
    assert rate > pH - 0.3, (errs, rate)
