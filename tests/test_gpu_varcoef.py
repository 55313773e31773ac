"""Material linear inside the elements through the approximate mass inverse (Section
3.3.2): the HIP path (dgm_set_material_linear and the generated dgm_mass_p{p} kernels)
against the oracle's VarMaterialSolver, element by element, through the C-ABI.

The approximate inverse depends on the reference map its quadrature rule is laid on;
the library uses the map with vertices sorted by global id, so the oracle is given the
sorted elements with the vertex values permuted alike.  Tolerances as for the constant
material: FP64 1e-10, FP32 1e-5 relative to the largest value; runs in the energy norm;
the leapfrog invariant in the inner product of M~ = P^{-1} (exactly conserved by the
scheme, Section 3)."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import frames, patch, rel_err, sort_tets
from oracle.mixed import MixedSolver
from oracle.varcoef import VarMaterialSolver
from paper_1104_4208_amd.gen.basis import volume_modes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1104_4208_amd as P  # noqa: E402
from paper_1104_4208_amd.gen.emit import F64_MAX_ORDER as F64_MAX  # noqa: E402
from paper_1104_4208_amd.gen.tables import P_MAX  # noqa: E402

# every order in FP32, the orders instantiated in FP64
ORDERS_DTYPES = [(p, "f32") for p in range(1, P_MAX + 1)] + [(p, "f64") for p in range(1, F64_MAX + 1)]


def sorted_values(tets, vals):
    """(K,4) vertex values in the caller's order -> in sorted-vertex order."""
    order = np.argsort(np.asarray(tets), axis=1)
    return np.take_along_axis(np.asarray(vals, float), order, axis=1)


def mode_perm(p):
    idx = {m: r for r, m in enumerate(oracle.mode_list(p))}
    pm = np.array([idx[m] for m in volume_modes(p)])
    ipm = np.empty_like(pm)
    ipm[pm] = np.arange(len(pm))
    return pm, ipm


class VarPair:
    """The oracle's variable-material solver on the library's (sorted) elements."""

    def __init__(self, verts, tets, p, eps_v, mu_v):
        ts = sort_tets(tets)
        self.s = VarMaterialSolver(oracle.build_mesh(np.asarray(verts, float), ts), p,
                                   sorted_values(tets, eps_v), sorted_values(tets, mu_v))
        self.F = frames(verts, tets)
        self.pm, self.ipm = mode_perm(p)

    def to_cov(self, phys):
        return np.einsum("kji,kmj->imk", self.F, phys)[:, self.pm, :]

    def to_phys(self, cov):
        c = np.asarray(cov, float)[:, self.ipm, :]
        return np.einsum("kji,jmk->kmi", np.linalg.inv(self.F), c)

    def invariant(self, E, H, dt):
        Hn = H + dt * self.s.rhs_h(E)
        return 0.5 * self.s.mass_dot(E, E, "E") + 0.5 * self.s.mass_dot(H, Hn, "H")


def dev(a, dtype):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


MESHES = {
    "one": lambda rng: synth.single_tet(np.array([[0.1, 0, 0], [1, 0.2, 0], [0, 1.1, 0.1], [0.2, 0.1, 0.9]])),
    "two_unsorted": lambda rng: synth.two_tets(rng),
    "cube1": lambda rng: synth.kuhn_mesh(1),
    "jit2": lambda rng: synth.kuhn_mesh(2, 0.1, rng),
    "jit3_ragged": lambda rng: synth.kuhn_mesh(3, 0.1, rng),
}


def smooth_material(verts, tets):
    """Continuous material fields sampled at the vertices (caller's order)."""
    x = np.asarray(verts, float)[np.asarray(tets)]
    eps = 1.5 + 0.5 * np.sin(2.0 * x[..., 0]) + 0.4 * x[..., 1]
    mu = 1.0 + 0.3 * x[..., 2]
    return eps, mu


@pytest.mark.parametrize("p,dtype", ORDERS_DTYPES)
@pytest.mark.parametrize("mesh", list(MESHES))
def test_var_apply_curl_parity(mesh, p, dtype):
    rng = np.random.default_rng(700 + p)
    verts, tets = MESHES[mesh](rng)
    K = tets.shape[0]
    eps_v, mu_v = rng.uniform(1, 4, (K, 4)), rng.uniform(1, 2, (K, 4))  # jumps between elements too
    pr = VarPair(verts, tets, p, eps_v, mu_v)
    E = rng.standard_normal((K, pr.s.N, 3))
    H = rng.standard_normal((K, pr.s.N, 3))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tol = 1e-10 if dtype == "f64" else 1e-5
    m = P.Mesh(verts, tets).set_order(p).set_material_linear(eps_v, mu_v)
    dE, dH = m.apply_curl(dev(pr.to_cov(E), tdt), dev(pr.to_cov(H), tdt))
    ee = rel_err(host(dE), pr.to_cov(pr.s.rhs_e(H)))
    eh = rel_err(host(dH), pr.to_cov(pr.s.rhs_h(E)))
    print(f"var p={p} {mesh} {dtype}: dE {ee:.2e} dH {eh:.2e}")
    assert ee < tol and eh < tol


@pytest.mark.parametrize("p,dtype", ORDERS_DTYPES)
def test_mass_inverse_alone(p, dtype):
    """dgm_apply_mass_inverse: Y[c] = P X[c] for both fields against the oracle's approximate
    inverse (which takes moments, so it is given X |det F|), on the ragged 162-tet mesh with
    vertex values jumping between elements."""
    rng = np.random.default_rng(800 + p)
    verts, tets = synth.kuhn_mesh(3, 0.1, rng)
    K = tets.shape[0]
    eps_v, mu_v = rng.uniform(1, 4, (K, 4)), rng.uniform(0.5, 2, (K, 4))
    pr = VarPair(verts, tets, p, eps_v, mu_v)
    N = pr.s.N
    X = rng.standard_normal((3, N, K))
    Xo = np.transpose(X, (2, 1, 0))[:, pr.ipm, :]  # (K, N, 3) in the oracle's mode order
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tol = 1e-12 if dtype == "f64" else 1e-6
    m = P.Mesh(verts, tets).set_order(p).set_material_linear(eps_v, mu_v)
    for field in ("E", "H"):
        Y = host(m.apply_mass_inverse(dev(X, tdt), field))
        Yo = pr.s.approx_inverse(Xo * pr.s.absJ[:, None, None], field)
        ref = np.transpose(Yo[:, pr.pm, :], (2, 1, 0))
        err = rel_err(Y, ref)
        print(f"mass inverse p={p} {dtype} {field}: {err:.2e}")
        assert err < tol


@pytest.mark.parametrize("p", [2, 5])
def test_var_constant_values_equal_the_flat_method(p):
    """Vertex values equal on each element: the same rates as dgm_set_material (the
    approximate inverse is then exact), and dgm_set_material switches back."""
    rng = np.random.default_rng(71)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    eps, mu = rng.uniform(1, 4, K), rng.uniform(1, 2, K)
    E = dev(rng.standard_normal((3, P.num_modes(p), K)), torch.float64)
    H = dev(rng.standard_normal((3, P.num_modes(p), K)), torch.float64)
    m = P.Mesh(verts, tets).set_order(p).set_material(eps, mu)
    dE0, dH0 = m.apply_curl(E, H)
    m.set_material_linear(np.repeat(eps[:, None], 4, 1), np.repeat(mu[:, None], 4, 1))
    dE1, dH1 = m.apply_curl(E, H)
    assert rel_err(host(dE1), host(dE0)) < 1e-12 and rel_err(host(dH1), host(dH0)) < 1e-12
    m.set_material(eps, mu)
    dE2, dH2 = m.apply_curl(E, H)
    assert torch.equal(dE2, dE0) and torch.equal(dH2, dH0)


@pytest.mark.parametrize("dtype,tol,qtol", [(torch.float64, 1e-10, 1e-12), (torch.float32, 1e-5, 1e-6)])
def test_var_run_against_oracle(dtype, tol, qtol):
    """TE101 on the jittered 48-tet cube at p = 3 with smooth eps and mu: 80 leapfrog
    steps against the oracle's, energies against the oracle's M~ products, and the
    invariant Q conserved."""
    rng = np.random.default_rng(73)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    eps_v, mu_v = smooth_material(verts, tets)
    pr = VarPair(verts, tets, 3, eps_v, mu_v)
    s = pr.s
    E = s.project(synth.te101().E)
    H = np.zeros_like(E)
    dt = 0.9 / math.sqrt(s.spectral_radius(40, synth.splitmix64(73, H.size)))
    m = P.Mesh(verts, tets).set_order(3).set_material_linear(eps_v, mu_v)
    Eg, Hg = dev(pr.to_cov(E), dtype), dev(pr.to_cov(H), dtype)
    W0, Q0 = m.energy(Eg, Hg, dt=dt)
    Q0o = pr.invariant(E, H, dt)
    assert abs(Q0 - Q0o) < (1e-10 if dtype == torch.float64 else 1e-6) * Q0o
    worst, drift = 0.0, 0.0
    for _ in range(8):
        m.step(Eg, Hg, dt, 10)
        E, H = s.step(E, H, dt, 10)
        worst = max(worst, s.rel_error(pr.to_phys(host(Eg)), pr.to_phys(host(Hg)), E, H))
        W, Q = m.energy(Eg, Hg, dt=dt)
        drift = max(drift, abs(Q - Q0) / Q0)
    Qo = pr.invariant(E, H, dt)
    print(f"var run {dtype}: worst energy-norm error {worst:.2e}, Q drift {drift:.2e}, "
          f"Q vs oracle {abs(Q - Qo) / Qo:.2e}")
    assert worst < tol
    assert drift < qtol
    assert abs(Q - Qo) < (1e-10 if dtype == torch.float64 else 1e-5) * Qo


def test_var_estimate_dt_and_spectrum():
    """The power iteration in the M~ inner product approaches the largest eigenvalue of
    the assembled operator from below (within 1e-3 after 200 iterations)."""
    rng = np.random.default_rng(75)
    verts, tets = synth.kuhn_mesh(1)
    eps_v, mu_v = rng.uniform(1, 4, (6, 4)), rng.uniform(1, 2, (6, 4))
    pr = VarPair(verts, tets, 2, eps_v, mu_v)
    Ah, Ae = pr.s.assemble()
    rho = float(np.linalg.eigvals(-(Ah @ Ae)).real.max())
    m = P.Mesh(verts, tets).set_order(2).set_material_linear(eps_v, mu_v)
    dt, est = m.estimate_dt(cfl=0.5, iters=200, seed=7)
    print(f"var rho: library {est:.8e}, assembled oracle {rho:.8e}")
    assert rho * (1 - 1e-3) < est < rho * (1 + 1e-10)


def test_var_mixed_orders():
    """Mixed orders (E of degree 3, H of degree 2) with the material linear on the
    elements: the oracle's unit-material mixed rates followed by its approximate
    inverses of the two orders."""
    rng = np.random.default_rng(77)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    eps_v, mu_v = rng.uniform(1, 4, (K, 4)), rng.uniform(1, 2, (K, 4))
    ts = sort_tets(tets)
    mesh = oracle.build_mesh(verts, ts)
    mix = MixedSolver(mesh, 3, 2, None, None)
    invE = VarMaterialSolver(mesh, 3, sorted_values(tets, eps_v), sorted_values(tets, mu_v))
    invH = VarMaterialSolver(mesh, 2, sorted_values(tets, eps_v), sorted_values(tets, mu_v))
    F = frames(verts, tets)
    pmE, ipmE = mode_perm(3)
    pmH, ipmH = mode_perm(2)
    cov = lambda phys, pm: np.einsum("kji,kmj->imk", F, phys)[:, pm, :]
    E = rng.standard_normal((K, mix.NE, 3))
    H = rng.standard_normal((K, mix.NH, 3))
    J = invE.absJ[:, None, None]
    refE = invE.approx_inverse(mix.rhs_e(H) * J, "E")
    refH = invH.approx_inverse(mix.rhs_h(E) * J, "H")
    m = P.Mesh(verts, tets).set_orders(3, 2).set_material_linear(eps_v, mu_v)
    for dtype, tol in ((torch.float64, 1e-10), (torch.float32, 1e-5)):
        dE, dH = m.apply_curl(dev(cov(E, pmE), dtype), dev(cov(H, pmH), dtype))
        ee, eh = rel_err(host(dE), cov(refE, pmE)), rel_err(host(dH), cov(refH, pmH))
        print(f"var mixed (3,2) {dtype}: dE {ee:.2e} dH {eh:.2e}")
        assert ee < tol and eh < tol


@pytest.mark.parametrize("pE,pH,qtol", [(3, 2, 1e-12), (8, 7, 1e-6)])
def test_var_mixed_orders_run_and_invariant(pE, pH, qtol):
    """Mixed orders with the material linear on the elements through the whole run path:
    30 leapfrog steps (FP64 where the orders have FP64 kernels, else FP32) from random
    fields; the invariant Q (energies by conjugate-gradient solves of the approximate mass
    matrices, FP64 at (3, 2), FP32 at (8, 7) where no FP64 kernels exist) stays constant, and
    at (3, 2) W and Q agree with the oracle's M~ products of the same state."""
    rng = np.random.default_rng(81)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    eps_v, mu_v = smooth_material(verts, tets)
    m = P.Mesh(verts, tets).set_orders(pE, pH).set_material_linear(eps_v, mu_v)
    f64 = pE <= P.max_order(P.DGM_F64)
    tdt = torch.float64 if f64 else torch.float32
    E = dev(rng.standard_normal((3, P.num_modes(pE), K)), tdt)
    H = dev(rng.standard_normal((3, P.num_modes(pH), K)), tdt)
    dt, _ = m.estimate_dt(cfl=0.5, iters=30, seed=5)
    W0, Q0 = m.energy(E, H, dt=dt)
    if f64:
        ts = sort_tets(tets)
        mesh = oracle.build_mesh(verts, ts)
        invE = VarMaterialSolver(mesh, pE, sorted_values(tets, eps_v), sorted_values(tets, mu_v))
        invH = VarMaterialSolver(mesh, pH, sorted_values(tets, eps_v), sorted_values(tets, mu_v))
        F = frames(verts, tets)
        Finv = np.linalg.inv(F)
        phys = lambda cov, p: np.einsum("kji,jmk->kmi", Finv, np.asarray(cov, float)[:, mode_perm(p)[1], :])
        Eo, Ho = phys(host(E), pE), phys(host(H), pH)
        Wo = 0.5 * invE.mass_dot(Eo, Eo, "E") + 0.5 * invH.mass_dot(Ho, Ho, "H")
        assert abs(W0 - Wo) < 1e-10 * Wo
    drift = 0.0
    for _ in range(3):
        m.step(E, H, dt, 10)
        _, Q = m.energy(E, H, dt=dt)
        drift = max(drift, abs(Q - Q0) / Q0)
    print(f"var mixed ({pE},{pH}) {tdt}: Q drift over 30 steps {drift:.2e}")
    assert drift < qtol


def test_var_nodal_material_is_the_linear_one_at_the_vertices():
    """set_material_nodal (values at the mesh vertices) gives the same rates, bitwise, as
    set_material_linear with each element's vertex values, on a mesh with unsorted elements."""
    rng = np.random.default_rng(85)
    verts, tets = synth.two_tets(rng)
    eps_n, mu_n = rng.uniform(1, 3, len(verts)), rng.uniform(1, 2, len(verts))
    N = P.num_modes(4)
    E = dev(rng.standard_normal((3, N, 2)), torch.float64)
    H = dev(rng.standard_normal((3, N, 2)), torch.float64)
    a = P.Mesh(verts, tets).set_order(4).set_material_nodal(eps_n, mu_n)
    b = P.Mesh(verts, tets).set_order(4).set_material_linear(eps_n[tets], mu_n[tets])
    dEa, dHa = a.apply_curl(E, H)
    dEb, dHb = b.apply_curl(E, H)
    torch.cuda.synchronize()
    assert torch.equal(dEa, dEb) and torch.equal(dHa, dHb)
    with pytest.raises(P.DGMError):
        a.set_material_nodal(eps_n[:-1])


def test_var_probed_run_equals_plain_run():
    """dgm_step_probe with the material linear on the elements leaves the same fields as
    dgm_step (bitwise), and a longer probed run repeats the shorter one's signal."""
    rng = np.random.default_rng(83)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    eps_v, mu_v = smooth_material(verts, tets)
    m = P.Mesh(verts, tets).set_order(3).set_material_linear(eps_v, mu_v)
    N = P.num_modes(3)
    E0 = dev(rng.standard_normal((3, N, K)), torch.float32)
    H0 = dev(rng.standard_normal((3, N, K)), torch.float32)
    w = dev(rng.standard_normal((3, N, K)), torch.float32)
    Ea, Ha, Eb, Hb, Ec, Hc = E0.clone(), H0.clone(), E0.clone(), H0.clone(), E0.clone(), H0.clone()
    m.step(Ea, Ha, 1e-3, 10)
    s10 = m.step_probe(Eb, Hb, 1e-3, 10, w)
    s20 = m.step_probe(Ec, Hc, 1e-3, 20, w)
    torch.cuda.synchronize()
    assert torch.equal(Ea, Eb) and torch.equal(Ha, Hb)
    assert np.array_equal(s10, s20[:10]) and np.all(np.isfinite(s20))


def test_var_run_against_oracle_golden():
    """The linear-material version of the p = 6 workload recipe (4^3 cells, jitter, eps in
    {1,4} times a smooth factor, mu linear, three cavity modes) for its full 500 steps in
    FP32 against the oracle's stored run (tests/golden/run_cfg3_var.npz, written by
    make_run_goldens.py from the oracle alone): sampled elements at every checkpoint and the
    whole final state within 1e-5 in the energy norm of the approximate mass matrices, and
    the invariant Q within 1e-6 of the oracle's at every checkpoint."""
    import importlib.util
    import os

    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "golden", "run_cfg3_var.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    spec = importlib.util.spec_from_file_location("make_run_goldens", os.path.join(here, "golden", "make_run_goldens.py"))
    MG = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(MG)
    with np.load(path, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    r, verts, tets, eps_v, mu_v, s, E, H = MG.setup("cfg3_var")
    assert np.array_equal(verts, g["verts"]) and np.array_equal(tets, g["tets"])
    assert np.array_equal(eps_v, g["eps"]) and np.array_equal(mu_v, g["mu"])
    assert abs(float(E.sum()) - float(g["init_checksum"])) <= 1e-12 * max(1.0, abs(float(g["init_checksum"])))
    pr = VarPair(verts, tets, r["p"], eps_v, mu_v)
    dt, every, C = float(g["dt"]), int(g["every"]), int(g["steps"]) // int(g["every"])
    m = P.Mesh(verts, tets).set_order(r["p"]).set_material_linear(eps_v, mu_v)
    Eg, Hg = dev(pr.to_cov(E), torch.float32), dev(pr.to_cov(H), torch.float32)
    smp = g["sample"]
    worst_s = worst_q = 0.0
    for c in range(C):
        m.step(Eg, Hg, dt, every)
        Ec, Hc = pr.to_phys(host(Eg)), pr.to_phys(host(Hg))
        num = np.abs(Ec[smp] - g["E_s"][c]).max() + np.abs(Hc[smp] - g["H_s"][c]).max()
        den = np.abs(g["E_s"][c]).max() + np.abs(g["H_s"][c]).max()
        worst_s = max(worst_s, num / den)
        _, Q = m.energy(Eg, Hg, dt=dt)
        worst_q = max(worst_q, abs(Q - float(g["Q"][c])) / float(g["Q"][c]))
    end = pr.s.rel_error(pr.to_phys(host(Eg)), pr.to_phys(host(Hg)), g["E_end"], g["H_end"])
    print(f"cfg3_var FP32 {int(g['steps'])} steps vs oracle: worst sampled {worst_s:.2e}, final energy-norm "
          f"{end:.2e}, Q vs oracle {worst_q:.2e}")
    assert worst_s < 1e-5 and end < 1e-5 and worst_q < 1e-6


def test_var_full_size_sampled():
    """The 32^3 x 6 jittered cube at p = 6 (196,608 tets), FP32, material linear on every
    element with eps jumping between 1 and 4 times a smooth factor: one application,
    sampled elements against the oracle on their patch meshes."""
    rng = np.random.default_rng(79)
    w = synth.WORKLOADS["cube32_p6_f32"]
    d = synth.build_workload(w)
    verts, tets = d["verts"], d["tets"]
    K = tets.shape[0]
    x = verts[tets]
    eps_v = d["eps"][:, None] * (1.0 + 0.25 * np.sin(3.0 * x[..., 0]) * np.cos(2.0 * x[..., 2]))
    mu_v = 1.0 + 0.2 * x[..., 1]
    m = P.Mesh(verts, tets).set_order(w.p).set_material_linear(eps_v, mu_v)
    N = P.num_modes(w.p)
    Ecov = rng.standard_normal((3, N, K)).astype(np.float32)
    Hcov = rng.standard_normal((3, N, K)).astype(np.float32)
    dE, dH = m.apply_curl(dev(Ecov, torch.float32), dev(Hcov, torch.float32))
    dE, dH = host(dE), host(dH)
    centers = np.unique(np.concatenate([rng.integers(0, K, 8), [0, K - 1]]))
    keep, ptets, pos = patch(tets, centers)
    pr = VarPair(verts, ptets, w.p, sorted_values(tets, eps_v)[keep], sorted_values(tets, mu_v)[keep])
    ref_dE = pr.to_cov(pr.s.rhs_e(pr.to_phys(Hcov[:, :, keep].astype(np.float64))))[:, :, pos]
    ref_dH = pr.to_cov(pr.s.rhs_h(pr.to_phys(Ecov[:, :, keep].astype(np.float64))))[:, :, pos]
    ee, eh = rel_err(dE[:, :, centers], ref_dE), rel_err(dH[:, :, centers], ref_dH)
    print(f"var 32^3 p6 sampled {len(centers)}: dE {ee:.2e} dH {eh:.2e}")
    assert ee < 1e-5 and eh < 1e-5


def test_var_rejected_where_unsupported():
    verts, tets = synth.kuhn_mesh(1)
    m = P.Mesh(verts, tets).set_order(2)
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        m.apply_mass_inverse(m.zeros(torch.float32))
    with pytest.raises(P.DGMError, match="DGM_ERR_MATERIAL"):
        m.set_material_linear(np.full((6, 4), -1.0))
    m.set_material_linear(np.full((6, 4), 2.0)).set_stab_alpha(1.0)
    E, H = m.zeros(torch.float32), m.zeros(torch.float32)
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        m.energy_stab(E, H, m.face_zeros(torch.float32))
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        m.apply_curl_dense(E, H)
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        m.step_noalloc(E, H, 1e-3, 1)
    b = P.Batch(chunk=2)
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        b.add(m, E, H, 1e-3, 2)
