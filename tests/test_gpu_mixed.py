"""Mixed orders (E of degree p+1, H of degree p; Section 2): the HIP path against the
oracle's MixedSolver, element by element, through the C-ABI.  Tolerances as for equal
orders: FP64 1e-10, FP32 1e-5 relative to the largest value, runs in the energy norm."""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import frames, patch, rel_err, sort_tets
from oracle.mixed import MixedSolver
from paper_1104_4208_amd.gen.basis import volume_modes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1104_4208_amd as P  # noqa: E402
from paper_1104_4208_amd.gen.emit import F64_MAX_ORDER as F64_MAX  # noqa: E402
from paper_1104_4208_amd.gen.tables import P_MAX  # noqa: E402

# every order in FP32, the orders instantiated in FP64
ORDERS_DTYPES = [(p, "f32") for p in range(1, P_MAX + 1)] + [(p, "f64") for p in range(1, F64_MAX + 1)]


class MixedPair:
    """The oracle's mixed solver on the library's elements, with the representation
    changes of both fields (physical (K,N,3) <-> covariant (3,N,K), mode orders)."""

    def __init__(self, verts, tets, pE, pH, eps=None, mu=None):
        self.s = MixedSolver(oracle.build_mesh(np.asarray(verts, float), sort_tets(tets)), pE, pH, eps, mu)
        self.F = frames(verts, tets)
        self.pm = {}
        for p in (pE, pH):
            idx = {m: r for r, m in enumerate(oracle.mode_list(p))}
            pm = np.array([idx[m] for m in volume_modes(p)])
            ipm = np.empty_like(pm)
            ipm[pm] = np.arange(len(pm))
            self.pm[p] = (pm, ipm)
        self.pE, self.pH = pE, pH

    def to_cov(self, phys, p):
        return np.einsum("kji,kmj->imk", self.F, phys)[:, self.pm[p][0], :]

    def to_phys(self, cov, p):
        c = np.asarray(cov, float)[:, self.pm[p][1], :]
        return np.einsum("kji,jmk->kmi", np.linalg.inv(self.F), c)


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


@pytest.mark.parametrize("pH,dtype", [(p, "f32") for p in range(1, P_MAX)] + [(p, "f64") for p in range(1, F64_MAX)])
@pytest.mark.parametrize("mesh", list(MESHES))
def test_mixed_apply_curl_parity(mesh, pH, dtype):
    pE = pH + 1
    rng = np.random.default_rng(500 + pH)
    verts, tets = MESHES[mesh](rng)
    K = tets.shape[0]
    eps, mu = rng.uniform(1, 4, K), rng.uniform(1, 2, K)
    pr = MixedPair(verts, tets, pE, pH, eps, mu)
    E = rng.standard_normal((K, pr.s.NE, 3))
    H = rng.standard_normal((K, pr.s.NH, 3))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    tol = 1e-10 if dtype == "f64" else 1e-5
    m = P.Mesh(verts, tets).set_orders(pE, pH).set_material(eps, mu)
    dE, dH = m.apply_curl(dev(pr.to_cov(E, pE), tdt), dev(pr.to_cov(H, pH), tdt))
    ee = rel_err(host(dE), pr.to_cov(pr.s.rhs_e(H), pE))
    eh = rel_err(host(dH), pr.to_cov(pr.s.rhs_h(E), pH))
    print(f"mixed ({pE},{pH}) {mesh} {dtype}: dE {ee:.2e} dH {eh:.2e}")
    assert ee < tol and eh < tol


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-10), (torch.float32, 1e-5)])
def test_mixed_run_against_oracle(dtype, tol):
    """TE101 on the jittered 48-tet cube with (pE, pH) = (3, 2), eps in {1, 4}: 80
    leapfrog steps against the oracle's, and the leapfrog invariant."""
    rng = np.random.default_rng(41)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    eps = rng.choice([1.0, 4.0], size=K)
    pr = MixedPair(verts, tets, 3, 2, eps, None)
    s = pr.s
    E = s.project(synth.te101().E, "E")
    H = np.zeros((K, s.NH, 3))
    dt = 1.0 / math.sqrt(s.spectral_radius(40, synth.splitmix64(41, H.size)))
    m = P.Mesh(verts, tets).set_orders(3, 2).set_material(eps, None)
    Eg, Hg = dev(pr.to_cov(E, 3), dtype), dev(pr.to_cov(H, 2), dtype)
    _, Q0 = m.energy(Eg, Hg, dt=dt)
    Q0o = s.leapfrog_invariant(E, H, dt)
    assert abs(Q0 - Q0o) < (1e-10 if dtype == torch.float64 else 1e-6) * Q0o
    worst, drift = 0.0, 0.0
    for _ in range(8):
        m.step(Eg, Hg, dt, 10)
        E, H = s.step(E, H, dt, 10)
        worst = max(worst, s.rel_error(pr.to_phys(host(Eg), 3), pr.to_phys(host(Hg), 2), E, H))
        _, Q = m.energy(Eg, Hg, dt=dt)
        drift = max(drift, abs(Q - Q0) / Q0)
    print(f"mixed run {dtype}: worst energy-norm error {worst:.2e}, Q drift {drift:.2e}")
    assert worst < tol
    assert drift < (1e-12 if dtype == torch.float64 else 1e-6)


def test_mixed_run_against_oracle_golden():
    """The p = 6 workload recipe (4^3 cells, jitter, eps in {1,4}, three cavity modes) with E
    of degree 7 and H of degree 6 for its full 500 steps in FP32 against the oracle's stored
    run (tests/golden/run_cfg3_mixed.npz, written by make_run_goldens.py from the oracle
    alone): sampled elements at every checkpoint and the final state within 1e-5 in the
    energy norm, the invariant within 1e-6 of the oracle's."""
    import importlib.util
    import os

    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "golden", "run_cfg3_mixed.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    spec = importlib.util.spec_from_file_location("make_run_goldens", os.path.join(here, "golden", "make_run_goldens.py"))
    MG = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(MG)
    with np.load(path, allow_pickle=False) as z:
        g = {k: z[k] for k in z.files}
    r, verts, tets, eps, mu, s, E, H = MG.setup("cfg3_mixed")
    assert np.array_equal(verts, g["verts"]) and np.array_equal(tets, g["tets"]) and np.array_equal(eps, g["eps"])
    assert abs(float(E.sum()) - float(g["init_checksum"])) <= 1e-12 * max(1.0, abs(float(g["init_checksum"])))
    pE, pH = r["pE"], r["p"]
    pr = MixedPair(verts, tets, pE, pH, eps, mu)
    m = P.Mesh(verts, tets).set_orders(pE, pH).set_material(eps, mu)
    dt, every, C = float(g["dt"]), int(g["every"]), int(g["steps"]) // int(g["every"])
    Eg, Hg = dev(pr.to_cov(E, pE), torch.float32), dev(pr.to_cov(H, pH), torch.float32)
    smp = g["sample"]
    worst_s = worst_q = 0.0
    for c in range(C):
        m.step(Eg, Hg, dt, every)
        Ec, Hc = pr.to_phys(host(Eg), pE), pr.to_phys(host(Hg), pH)
        num = np.abs(Ec[smp] - g["E_s"][c]).max() + np.abs(Hc[smp] - g["H_s"][c]).max()
        den = np.abs(g["E_s"][c]).max() + np.abs(g["H_s"][c]).max()
        worst_s = max(worst_s, num / den)
        _, Q = m.energy(Eg, Hg, dt=dt)
        worst_q = max(worst_q, abs(Q - float(g["Q"][c])) / float(g["Q"][c]))
    end = pr.s.rel_error(pr.to_phys(host(Eg), pE), pr.to_phys(host(Hg), pH), g["E_end"], g["H_end"])
    print(f"cfg3_mixed FP32 {int(g['steps'])} steps vs oracle: worst sampled {worst_s:.2e}, final energy-norm "
          f"{end:.2e}, Q vs oracle {worst_q:.2e}")
    assert worst_s < 1e-5 and end < 1e-5 and worst_q < 1e-6


def test_mixed_estimate_dt_and_spectrum():
    """The power iteration approaches the largest eigenvalue of the mixed operator from
    below (within 1e-3 of the oracle's assembled value after 200 iterations)."""
    verts, tets = synth.kuhn_mesh(1)
    pr = MixedPair(verts, tets, 3, 2)
    Ah, Ae = pr.s.assemble()
    rho = float(np.linalg.eigvals(-(Ah @ Ae)).real.max())
    m = P.Mesh(verts, tets).set_orders(3, 2)
    dt, est = m.estimate_dt(cfl=0.5, iters=200, seed=7)
    print(f"mixed rho: library {est:.8e}, assembled oracle {rho:.8e}")
    assert rho * (1 - 1e-3) < est < rho * (1 + 1e-12)


def test_mixed_full_size_sampled():
    """(pE, pH) = (5, 4) on the 16^3 x 6 jittered cube, FP32: one application, sampled
    elements against the oracle on their patch meshes; and a step through the
    allocation-free entry point equals dgm_step bitwise."""
    rng = np.random.default_rng(54)
    n, pE, pH = 16, 5, 4
    verts, tets = synth.kuhn_mesh(n, 0.1, rng)
    K = tets.shape[0]
    eps = rng.choice([1.0, 4.0], size=K)
    m = P.Mesh(verts, tets).set_orders(pE, pH).set_material(eps, None)
    Ecov = rng.standard_normal((3, P.num_modes(pE), K)).astype(np.float32)
    Hcov = rng.standard_normal((3, P.num_modes(pH), K)).astype(np.float32)
    dE, dH = m.apply_curl(dev(Ecov, torch.float32), dev(Hcov, torch.float32))
    dE, dH = host(dE), host(dH)
    centers = np.unique(np.concatenate([rng.integers(0, K, 8), [0, K - 1]]))
    keep, ptets, pos = patch(tets, centers)
    pr = MixedPair(verts, ptets, pE, pH, eps[keep], None)
    ref_dE = pr.to_cov(pr.s.rhs_e(pr.to_phys(Hcov[:, :, keep].astype(np.float64), pH)), pE)[:, :, pos]
    ref_dH = pr.to_cov(pr.s.rhs_h(pr.to_phys(Ecov[:, :, keep].astype(np.float64), pE)), pH)[:, :, pos]
    ee, eh = rel_err(dE[:, :, centers], ref_dE), rel_err(dH[:, :, centers], ref_dH)
    print(f"mixed 16^3 ({pE},{pH}) sampled {len(centers)}: dE {ee:.2e} dH {eh:.2e}")
    assert ee < 1e-5 and eh < 1e-5
    # allocation-free step on a small mixed mesh, bitwise against dgm_step
    v2, t2 = synth.kuhn_mesh(4, 0.1, rng)
    m2 = P.Mesh(v2, t2).set_orders(3, 2)
    E0 = dev(rng.standard_normal((3, P.num_modes(3), t2.shape[0])), torch.float32)
    H0 = dev(rng.standard_normal((3, P.num_modes(2), t2.shape[0])), torch.float32)
    Ea, Ha, Eb, Hb = E0.clone(), H0.clone(), E0.clone(), H0.clone()
    m2.step(Ea, Ha, 1e-3, 7)
    m2.step_noalloc(Eb, Hb, 1e-3, 7)
    torch.cuda.synchronize()
    assert torch.equal(Ea, Eb) and torch.equal(Ha, Hb)


def test_mixed_orders_rejected_where_unsupported():
    verts, tets = synth.kuhn_mesh(1)
    m = P.Mesh(verts, tets)
    with pytest.raises(P.DGMError, match="DGM_ERR_ARG"):
        m.set_orders(5, 3)
    m.set_orders(3, 2).set_stab_alpha(1.0)
    E = m.zeros(torch.float32, field="E")
    H = m.zeros(torch.float32)
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        m.energy_stab(E, H, m.face_zeros(torch.float32))
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        m.apply_curl_dense(E, H)
    b = P.Batch(chunk=2)
    with pytest.raises(P.DGMError, match="DGM_ERR_STATE"):
        b.add(m, E, H, 1e-3, 2)
    with pytest.raises(P.DGMError):
        m.step(H.clone(), H, 1e-3, 1)  # E with H's shape
