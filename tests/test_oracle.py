"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: every check is against a
closed form, a library routine, an identity (integration by parts,
skew-symmetry, exact energy conservation), a relation printed in the paper
(tests/golden), brute force, or the exact PEC cube eigenmodes.
"""
import math

import numpy as np
import pytest
import scipy.special as sps

import oracle
import synth
from oracle.basis import eval_basis, mode_list, norm_factor, tet_quadrature, triangle_quadrature
from oracle.jacobi import djacobi, gauss_jacobi, jacobi
from golden_io import legendre_relation, relations_2d, support_dx_3d


# ---------------------------------------------------------------- Jacobi / quadrature
@pytest.mark.parametrize("n,a,b", [(0, 0, 0), (3, 0, 0), (5, 1, 0), (7, 5, 0), (6, 12, 0), (4, 2.5, 1.0)])
def test_jacobi_matches_scipy(n, a, b):
    x = np.linspace(-1, 1, 41)
    assert np.allclose(jacobi(n, a, b, x), sps.eval_jacobi(n, a, b, x), rtol=1e-12, atol=1e-12)
    h = 1e-6
    fd = (sps.eval_jacobi(n, a, b, x + h) - sps.eval_jacobi(n, a, b, x - h)) / (2 * h)
    assert np.allclose(djacobi(n, a, b, x), fd, rtol=1e-6, atol=1e-5)


@pytest.mark.parametrize("a,b", [(0, 0), (1, 0), (2, 0), (3, 1)])
def test_gauss_jacobi_exact_on_beta_integrals(a, b):
    q = 6
    x, w = gauss_jacobi(q, a, b)
    # int (1-x)^(a+m) (1+x)^(b+l) dx = 2^(a+b+m+l+1) B(a+m+1, b+l+1), exact for m+l <= 2q-1
    for m in range(0, 6):
        for l in range(0, 2 * q - m):
            exact = 2.0 ** (a + b + m + l + 1) * sps.beta(a + m + 1, b + l + 1)
            got = np.sum(w * (1 - x) ** m * (1 + x) ** l)
            assert abs(got - exact) <= 1e-12 * max(1.0, abs(exact))


def test_quadrature_volumes():
    _, w = tet_quadrature(4)
    assert abs(w.sum() - 1 / 6) < 1e-15
    _, wt = triangle_quadrature(4)
    assert abs(wt.sum() - 0.5) < 1e-15


# ---------------------------------------------------------------- basis
@pytest.mark.parametrize("p", [1, 2, 4, 6, 8])
def test_orthonormal_basis(p):
    x, w = tet_quadrature(p + 2)
    V = eval_basis(p, x)
    assert V.shape[0] == (p + 1) * (p + 2) * (p + 3) // 6
    assert np.abs((V * w) @ V.T - np.eye(V.shape[0])).max() < 1e-13


def test_unnormalised_norms_closed_form():
    # int phi_ijk^2 over the tet = 1 / ((2i+1)(2i+2j+2)(2i+2j+2k+3))   (unnormalised phi)
    p = 5
    x, w = tet_quadrature(p + 3)
    V = eval_basis(p, x)
    for m, (i, j, k) in enumerate(mode_list(p)):
        raw = V[m] / norm_factor(i, j, k)
        got = np.sum(w * raw * raw)
        exact = 1.0 / ((2 * i + 1) * (2 * i + 2 * j + 2) * (2 * i + 2 * j + 2 * k + 3))
        assert abs(got - exact) < 1e-14 * 10 + 1e-12 * exact


def test_basis_definition_pointwise():
    # direct evaluation of the printed formula with scipy at a few points
    pts = np.array([[0.1, 0.2, 0.3], [0.25, 0.05, 0.6], [0.6, 0.3, 0.05]])
    V = eval_basis(4, pts)
    for m, (i, j, k) in enumerate(mode_list(4)):
        x, y, z = pts.T
        ref = ((1 - x - y) ** i * (1 - x) ** j * sps.eval_legendre(i, 2 * z / (1 - x - y) - 1)
               * sps.eval_jacobi(j, 2 * i + 1, 0, 2 * y / (1 - x) - 1) * sps.eval_jacobi(k, 2 * i + 2 * j + 2, 0, 2 * x - 1))
        assert np.allclose(V[m], norm_factor(i, j, k) * ref, rtol=1e-12, atol=1e-13)


def test_gradients_against_finite_differences():
    rng = np.random.default_rng(3)
    pts = rng.dirichlet([1, 1, 1, 1], size=12)[:, 1:]
    _, G = eval_basis(6, pts, grad=True)
    h = 1e-6
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (eval_basis(6, pts + e) - eval_basis(6, pts - e)) / (2 * h)
        assert np.abs(fd - G[:, :, d]).max() < 1e-6 * max(1.0, np.abs(G).max())


# ---------------------------------------------------------------- printed relations
def test_legendre_relation_and_sweep():
    x = np.linspace(-1, 1, 17)
    rel = legendre_relation()
    for n in range(0, 8):
        tot = np.zeros_like(x)
        for c, s, d in rel:
            f = djacobi(n + s, 0, 0, x) if d else jacobi(n + s, 0, 0, x)
            tot += c(n=n) * f
        assert np.abs(tot).max() < 1e-11
    # first step of the derivative sweep: w_{n-1} = (2n-1) v_n
    nodes, wts = gauss_jacobi(12, 0, 0)
    for n in range(1, 9):
        dP = djacobi(n, 0, 0, nodes)
        w_top = np.sum(wts * dP * jacobi(n - 1, 0, 0, nodes)) / (2.0 / (2 * (n - 1) + 1))
        assert abs(w_top - (2 * n - 1)) < 1e-12


def _phi2d(i, j, x, y):
    return jacobi(i, 0, 0, 2 * y / (1 - x) - 1) * (1 - x) ** i * jacobi(j, 2 * i + 1, 0, 2 * x - 1)


def test_printed_2d_relations_hold():
    rng = np.random.default_rng(5)
    pts = rng.dirichlet([1, 1, 1], size=20)[:, 1:]
    x, y = pts[:, 0], pts[:, 1]
    h = 1e-4
    cs = [(1, 4 / 5), (2, -1 / 5), (3, 4 / 105), (4, -1 / 280)]

    def d(fn, axis):
        ex = np.array([h, 0.0]) if axis == "x" else np.array([0.0, h])
        return sum(c * (fn(x + k * ex[0], y + k * ex[1]) - fn(x - k * ex[0], y - k * ex[1])) for k, c in cs) / h

    rels = relations_2d()
    for name in ("dx", "dy"):
        for i in range(0, 4):
            for j in range(0, 4):
                tot = np.zeros_like(x)
                scale = 0.0
                for c, (si, sj), der in rels[name]:
                    fn = (lambda a, b, ii=i + si, jj=j + sj: _phi2d(ii, jj, a, b))
                    term = c(i=i, j=j) * (fn(x, y) if der == "-" else d(fn, der))
                    tot += term
                    scale = max(scale, np.abs(term).max())
                assert np.abs(tot).max() < 1e-7 * scale, (name, i, j)


def test_printed_3d_dx_support_has_one_relation():
    """The 16-monomial d/dx support of Section 4.2.2 admits exactly one relation at generic
    (i,j,k): this pins the 3D basis definition and its index roles."""
    sup = support_dx_3d()
    rng = np.random.default_rng(11)
    pts = rng.dirichlet([1, 1, 1, 1], size=60)[:, 1:]
    pmax = 10
    V, G = eval_basis(pmax, pts, grad=True)
    index = {m: r for r, m in enumerate(mode_list(pmax))}
    for (i, j, k) in [(1, 0, 0), (1, 1, 1), (2, 0, 1)]:
        cols = []
        for (si, sj, sk), der in sup:
            m = (i + si, j + sj, k + sk)
            r = index[m]
            col = (G[r, :, 0] if der == "x" else V[r]) / norm_factor(*m)
            cols.append(col / np.linalg.norm(col))
        s = np.linalg.svd(np.array(cols).T, compute_uv=False)
        assert s[-1] < 1e-9 * s[0] and s[-2] > 1e-4 * s[0], (i, j, k, s[-3:])


# ---------------------------------------------------------------- mesh
@pytest.mark.parametrize("n", [1, 2, 3])
def test_kuhn_mesh_topology(n):
    v, t = synth.kuhn_mesh(n)
    m = oracle.build_mesh(v, t)
    nb = int((m.nbr < 0).sum())
    assert nb == 12 * n * n
    assert int((m.nbr >= 0).sum()) == 24 * n ** 3 - 12 * n * n
    assert np.allclose(np.abs(m.J).sum() / 6.0, 1.0)  # volumes add up to the unit cube
    # closed surface: sum of area-weighted outward normals vanishes per element
    assert np.abs(np.einsum("kf,kfd->kd", m.area, m.normal)).max() < 1e-13


def test_degenerate_and_nonmanifold_rejected():
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    with pytest.raises(ValueError):
        oracle.build_mesh(v, np.array([[0, 1, 2, 3]]))
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1]], float)
    with pytest.raises(ValueError):
        oracle.build_mesh(v, np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]]))


def test_integration_by_parts_on_a_physical_tet():
    """int_T d_x(phi_a) phi_b + phi_a d_x(phi_b) = int_dT phi_a phi_b nu_x: pins gradients,
    face quadrature, areas and outward normals together."""
    rng = np.random.default_rng(2)
    v = np.array([[0, 0, 0], [1, 0.1, 0], [0.2, 0.9, 0.1], [0.1, 0.3, 1.1]]) + rng.uniform(-0.1, 0.1, (4, 3))
    m = oracle.build_mesh(v, np.array([[0, 2, 1, 3]]))  # negative orientation on purpose
    s = oracle.Solver(m, 3)
    F, Finv = m.F[0], m.Finv[0]
    Gp = np.einsum("jm,aqj->aqm", Finv, s.G)
    vol = np.einsum("aqm,bq,q->abm", Gp, s.V, s.wq) * abs(m.J[0])
    lhs = vol + vol.transpose(1, 0, 2)
    rhs = np.zeros_like(lhs)
    for f in range(4):
        ds = 2.0 * m.area[0, f] * s.wf
        rhs += np.einsum("aq,bq,q,m->abm", s.Vf[f], s.Vf[f], ds, m.normal[0, f])
    assert np.abs(lhs - rhs).max() < 1e-12


# ---------------------------------------------------------------- operator
def _poly_H(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([Y * Y * Z, X * Z, X ** 3], -1)


def _curl_poly_H(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([-X, Y * Y - 3 * X * X, Z - 2 * Y * Z], -1)


def _pec_E(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([0 * X, X * (1 - X) * Z * (1 - Z), 0 * X], -1)


def _curl_pec_E(x):
    X, Y, Z = x[..., 0], x[..., 1], x[..., 2]
    return np.stack([-(X * (1 - X) * (1 - 2 * Z)), 0 * X, (1 - 2 * X) * Z * (1 - Z)], -1)


def _jittered(n=2, seed=1):
    rng = np.random.default_rng(seed)
    v, t = synth.kuhn_mesh(n, 0.1, rng)
    return oracle.build_mesh(v, t), rng


def test_polynomial_exactness_pins_flux_signs():
    m, rng = _jittered()
    eps = rng.choice([1.0, 4.0], size=m.J.shape[0])
    mu = rng.choice([1.0, 2.0], size=m.J.shape[0])
    s = oracle.Solver(m, 4, eps, mu)
    # E-phase: a global cubic H has no jumps, so dE/dt = curl H / eps exactly
    r = s.rhs_e(s.project(_poly_H))
    assert np.abs(r - s.project(_curl_poly_H) / eps[:, None, None]).max() < 1e-12
    # H-phase: a global quartic E with zero tangential trace on the walls
    r = s.rhs_h(s.project(_pec_E))
    assert np.abs(r + s.project(_curl_pec_E) / mu[:, None, None]).max() < 1e-12


def test_printed_flux_orientation_fails_exactness():
    """Planted mistake: the flux terms with the inner normal (the printed signs) break
    the consistency the corrected reading satisfies."""
    m, _ = _jittered()
    m.normal = -m.normal
    s = oracle.Solver(m, 4)
    r = s.rhs_e(s.project(_poly_H))
    assert np.abs(r - s.project(_curl_poly_H)).max() > 1e-2


@pytest.mark.parametrize("mesh", ["two", "cube1"])
def test_semidiscrete_system_is_skew(mesh):
    rng = np.random.default_rng(4)
    if mesh == "two":
        v, t = synth.two_tets(rng)
    else:
        v, t = synth.kuhn_mesh(1, 0.0)
    m = oracle.build_mesh(v, t)
    K = m.J.shape[0]
    eps, mu = rng.uniform(1, 3, K), rng.uniform(1, 3, K)
    s = oracle.Solver(m, 2, eps, mu)
    Ah, Ae = s.assemble()
    we = np.repeat(s.absJ * eps, s.N * 3)
    wm = np.repeat(s.absJ * mu, s.N * 3)
    # M_eps A_e = -(M_mu A_h)^T  (Section 2.1, eq. semidiscrete)
    assert np.abs(we[:, None] * Ae + (wm[:, None] * Ah).T).max() < 1e-12 * np.abs(we[:, None] * Ae).max()


def test_leapfrog_invariant_conserved_and_energy_bounded():
    m, rng = _jittered()
    s = oracle.Solver(m, 3, rng.choice([1.0, 4.0], size=m.J.shape[0]))
    E = s.project(synth.te101().E)
    H = np.zeros_like(E)
    rho = s.spectral_radius(30, synth.splitmix64(7, E.size))
    dt = 1.0 / math.sqrt(rho)
    Q0 = s.leapfrog_invariant(E, H, dt)
    W0 = s.energy(E, H)
    E2, H2 = s.step(E, H, dt, 60)
    assert abs(s.leapfrog_invariant(E2, H2, dt) - Q0) < 1e-13 * Q0
    assert abs(s.energy(E2, H2) - W0) < 0.5 * W0  # W oscillates at O(dt), never grows


def test_stability_threshold():
    """Leapfrog is stable iff dt <= 2/sqrt(rho) (the scalar amplification matrix has
    trace 2 - dt^2 w^2 and determinant 1); the printed bound lacks the root."""
    v, t = synth.kuhn_mesh(1)
    s = oracle.Solver(oracle.build_mesh(v, t), 2)
    Ah, Ae = s.assemble()
    lam = np.linalg.eigvals(-Ah @ Ae).real
    rho = lam.max()
    rng = np.random.default_rng(0)
    E0 = rng.standard_normal((s.K, s.N, 3))
    for fac, grows in [(0.98, False), (1.03, True)]:
        dt = fac * 2 / math.sqrt(rho)
        E, H = s.step(E0, np.zeros_like(E0), dt, 400)
        W = s.energy(E, H)
        assert (W > 1e3 * s.energy(E0, 0 * E0)) == grows
    # power iteration approaches the spectral radius from below (hence the CFL margin)
    est = s.spectral_radius(300, synth.splitmix64(1, E0.size))
    assert 0.999 * rho < est <= rho * (1 + 1e-12)


@pytest.mark.slow
def test_te101_h_convergence():
    errs = []
    p, T = 2, 0.25
    for n in (2, 4):
        v, t = synth.kuhn_mesh(n)
        s = oracle.Solver(oracle.build_mesh(v, t), p)
        mode = synth.te101()
        nst = 5 * n
        dt = T / nst
        E = s.project(mode.E)
        H = s.project(lambda x: mode.H(x, -dt / 2))  # leapfrog reading: H staggered by dt/2
        E2, H2 = s.step(E, H, dt, nst)
        Ee = s.project(lambda x: mode.E(x, T))
        He = s.project(lambda x: mode.H(x, T - dt / 2))
        errs.append(s.rel_error(E2, H2, Ee, He))
    rate = math.log2(errs[0] / errs[1])
    assert rate > 1.8, errs


def test_neighbour_points_by_inverse_map():
    m, _ = _jittered(2, 9)
    assert oracle.Solver(m, 3).check_neighbour_points() < 1e-12
    rng = np.random.default_rng(3)
    v, t = synth.two_tets(rng)
    assert oracle.Solver(oracle.build_mesh(v, t), 2).check_neighbour_points() < 1e-12


def test_tiny_mesh_spectrum_contains_cavity_modes():
    """Discrete resonances (omega^2 = eigenvalues of -A_h A_e) of the six-tet unit cube at
    p = 4: the PEC cube's two lowest exact eigenvalues, 2 pi^2 (three modes: TE101, TE011,
    TE110) and 3 pi^2 (two polarisations of the (1,1,1) mode), each appear with exactly that
    multiplicity to 0.5 %; the spectrum is real and non-negative (the operator is similar to
    a symmetric positive semi-definite one), and the null space of discrete gradients is
    separated from the rest.  The unstabilised central flux adds spurious non-zero modes
    in between (Section 2 points this out), which the counts above do not include."""
    v, t = synth.kuhn_mesh(1)
    s = oracle.Solver(oracle.build_mesh(v, t), 4)
    Ah, Ae = s.assemble()
    lam = np.linalg.eigvals(-Ah @ Ae)
    top = np.abs(lam.real).max()
    assert np.abs(lam.imag).max() < 1e-12 * top
    w2 = np.sort(lam.real)
    assert w2.min() > -1e-12 * top
    small = np.abs(w2) < 1e-12 * top
    assert small.sum() > 0 and np.all(w2[~small] > 1e-3 * top)
    r = w2 / np.pi ** 2
    assert np.sum(np.abs(r - 2) < 0.005 * 2) == 3
    assert np.sum(np.abs(r - 3) < 0.005 * 3) == 2
    assert np.sum(np.abs(r - 2) < 0.1) > 3  # spurious central-flux modes near the true ones
