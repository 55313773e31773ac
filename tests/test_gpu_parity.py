"""HIP path against the FP64 oracle, element by element, through the C-ABI.

Tolerances: FP64 mode 1e-10 relative (the oracle's own rounding is ~1e-13);
FP32 mode 1e-5 relative to the largest coefficient for one operator
application and over whole runs (rounding of a non-dissipative scheme grows
at most linearly with the step count; measured margins are printed).
"""
import math

import numpy as np
import pytest

import synth
from gpu_helpers import Pair, patch, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1104_4208_amd as P  # noqa: E402
from paper_1104_4208_amd.gen.emit import F64_MAX_ORDER as F64_MAX  # noqa: E402
from paper_1104_4208_amd.gen.tables import P_MAX  # noqa: E402

# every order in FP32, the orders instantiated in FP64
ORDERS_DTYPES = [(p, "f32") for p in range(1, P_MAX + 1)] + [(p, "f64") for p in range(1, F64_MAX + 1)]


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
    "jit3_ragged": lambda rng: synth.kuhn_mesh(3, 0.1, rng),  # K = 162: two full tiles + 34
}


def _materials(rng, K):
    return rng.uniform(1.0, 4.0, K), rng.uniform(1.0, 2.0, K)


@pytest.mark.parametrize("p,dtype", ORDERS_DTYPES)
@pytest.mark.parametrize("mesh", list(MESHES))
def test_apply_curl_parity(mesh, p, dtype):
    rng = np.random.default_rng(100 + p)
    verts, tets = MESHES[mesh](rng)
    K = tets.shape[0]
    eps, mu = _materials(rng, K)
    pr = Pair(verts, tets, p, eps, mu)
    E = rng.standard_normal((K, pr.s.N, 3))
    H = rng.standard_normal((K, pr.s.N, 3))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    m = P.Mesh(verts, tets).set_order(p).set_material(eps, mu)
    dE, dH = m.apply_curl(dev(pr.to_cov(E), tdt), dev(pr.to_cov(H), tdt))
    ref_dh = pr.to_cov(pr.s.rhs_h(E))
    ref_de = pr.to_cov(pr.s.rhs_e(H))
    tol = 1e-10 if dtype == "f64" else 1e-5
    eh, ee = rel_err(host(dH), ref_dh), rel_err(host(dE), ref_de)
    print(f"{mesh} p={p} {dtype}: dH {eh:.2e} dE {ee:.2e}")
    assert eh < tol and ee < tol


def test_operator_brute_force_two_tets():
    """Assemble the library's operator column by column and compare every entry."""
    rng = np.random.default_rng(5)
    verts, tets = synth.two_tets(rng)
    p = 2
    eps, mu = _materials(rng, 2)
    pr = Pair(verts, tets, p, eps, mu)
    Ah, Ae = pr.s.assemble()
    m = P.Mesh(verts, tets).set_order(p).set_material(eps, mu)
    n = 2 * pr.s.N * 3
    for col in range(n):
        u = np.zeros(n)
        u[col] = 1.0
        U = u.reshape(2, pr.s.N, 3)
        Ucov = dev(pr.to_cov(U), torch.float64)
        dE, dH = m.apply_curl(Ucov, Ucov)
        assert rel_err(pr.to_phys(host(dH)).ravel(), Ah[:, col]) < 1e-10 or np.abs(Ah[:, col]).max() < 1e-14
        assert rel_err(pr.to_phys(host(dE)).ravel(), Ae[:, col]) < 1e-10 or np.abs(Ae[:, col]).max() < 1e-14


def _te101_setup(n, p, jitter=0.0, seed=1):
    rng = np.random.default_rng(seed)
    verts, tets = synth.kuhn_mesh(n, jitter, rng if jitter else None)
    pr = Pair(verts, tets, p)
    E = pr.s.project(synth.te101().E)
    H = np.zeros_like(E)
    rho = pr.s.spectral_radius(40, synth.splitmix64(seed, E.size))
    dt = 1.0 / math.sqrt(rho)  # CFL 0.5 of the bound 2 / sqrt(rho)
    return verts, tets, pr, E, H, dt


def test_step_parity_cube2_p2_fp64():
    """48 tets, p = 2, TE101, 100 steps: every 10th step within 1e-10; Q conserved."""
    verts, tets, pr, E, H, dt = _te101_setup(2, 2)
    m = P.Mesh(verts, tets).set_order(2)
    Eg, Hg = dev(pr.to_cov(E), torch.float64), dev(pr.to_cov(H), torch.float64)
    W0, Q0 = m.energy(Eg, Hg, dt=dt)
    assert abs(W0 - pr.s.energy(E, H)) < 1e-12 * W0
    assert abs(Q0 - pr.s.leapfrog_invariant(E, H, dt)) < 1e-12 * Q0
    worst = 0.0
    for blk in range(10):
        m.step(Eg, Hg, dt, 10)
        E, H = pr.s.step(E, H, dt, 10)
        err = pr.s.rel_error(pr.to_phys(host(Eg)), pr.to_phys(host(Hg)), E, H)
        worst = max(worst, err)
        assert err < 1e-10, (blk, err)
    W, Q = m.energy(Eg, Hg, dt=dt)
    print(f"cube2 p2 f64: worst rel err {worst:.2e}, Q drift {abs(Q - Q0) / Q0:.2e}")
    assert abs(Q - Q0) < 1e-12 * Q0


def test_step_parity_fp32_jittered_p4():
    """FP32 run against the FP64 oracle: 200 steps on a jittered 3^3 mesh with eps in {1,4}."""
    rng = np.random.default_rng(2)
    verts, tets = synth.kuhn_mesh(3, 0.1, rng)
    K = tets.shape[0]
    eps = rng.choice([1.0, 4.0], size=K)
    pr = Pair(verts, tets, 4, eps, None)
    fld = synth.three_mode_sum(rng)
    E = pr.s.project(fld.E)
    H = np.zeros_like(E)
    rho = pr.s.spectral_radius(40, synth.splitmix64(2, E.size))
    dt = 1.0 / math.sqrt(rho)
    m = P.Mesh(verts, tets).set_order(4).set_material(eps, None)
    Eg, Hg = dev(pr.to_cov(E), torch.float32), dev(pr.to_cov(H), torch.float32)
    _, Q0 = m.energy(Eg, Hg, dt=dt)
    worst = 0.0
    for blk in range(4):
        m.step(Eg, Hg, dt, 50)
        E, H = pr.s.step(E, H, dt, 50)
        err = pr.s.rel_error(pr.to_phys(host(Eg)), pr.to_phys(host(Hg)), E, H)
        worst = max(worst, err)
    _, Q = m.energy(Eg, Hg, dt=dt)
    print(f"jit3 p4 f32 200 steps: worst rel err {worst:.2e}, Q drift {abs(Q - Q0) / Q0:.2e}")
    assert worst < 1e-5
    assert abs(Q - Q0) < 1e-6 * Q0


def test_estimate_dt_matches_spectrum():
    verts, tets = synth.kuhn_mesh(1)
    pr = Pair(verts, tets, 2)
    Ah, Ae = pr.s.assemble()
    rho = float(np.max(np.linalg.eigvals(-Ah @ Ae).real))
    m = P.Mesh(verts, tets).set_order(2)
    dt, est = m.estimate_dt(cfl=0.5, iters=300, seed=3)
    assert 0.999 * rho < est <= rho * (1 + 1e-9)
    assert abs(dt - 0.5 * 2 / math.sqrt(est)) < 1e-15


def test_deterministic_and_ragged():
    rng = np.random.default_rng(9)
    verts, tets = synth.kuhn_mesh(3, 0.1, rng)
    m = P.Mesh(verts, tets).set_order(3)
    K, N = tets.shape[0], P.num_modes(3)
    E0 = dev(rng.standard_normal((3, N, K)), torch.float32)
    H0 = dev(rng.standard_normal((3, N, K)), torch.float32)
    outs = []
    for _ in range(2):
        E, H = E0.clone(), H0.clone()
        m.step(E, H, 1e-3, 7)
        outs.append((host(E), host(H)))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_zero_steps_and_errors():
    verts, tets = synth.kuhn_mesh(1)
    m = P.Mesh(verts, tets)
    E = torch.zeros((3, 10, 6), dtype=torch.float32, device="cuda")
    with pytest.raises(P.DGMError):
        P.load_library()
        from paper_1104_4208_amd.dgmax import _check, _ptr, _stream
        _check(P.load_library().dgm_step(m.handle, 0, _ptr(E), _ptr(E.clone()), 0.1, 1, _stream()))
    m.set_order(2)
    H = E.clone()
    m.step(E, H, 0.1, 0)
    with pytest.raises(P.DGMError):
        m.set_material(np.full(6, -1.0), None)


@pytest.mark.parametrize("n,p", [(32, 6), (16, 4), (24, 8)])
def test_full_size_sampled_apply_curl(n, p):
    """At the benchmark sizes and launch configuration: apply_curl on the whole mesh,
    checked on sampled elements against the oracle on patch meshes."""
    rng = np.random.default_rng(n)
    verts, tets = synth.kuhn_mesh(n, 0.1, rng)
    K = tets.shape[0]
    eps = rng.choice([1.0, 4.0], size=K)
    N = P.num_modes(p)
    m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
    Ecov = rng.standard_normal((3, N, K)).astype(np.float32)
    Hcov = rng.standard_normal((3, N, K)).astype(np.float32)
    dE, dH = m.apply_curl(dev(Ecov, torch.float32), dev(Hcov, torch.float32))
    dE, dH = host(dE), host(dH)
    centers = np.unique(np.concatenate([rng.integers(0, K, 12), [0, K - 1]]))
    keep, ptets, pos = patch(tets, centers)
    pr = Pair(verts, ptets, p, eps[keep], None)
    Ep = pr.to_phys(Ecov[:, :, keep].astype(np.float64))
    Hp = pr.to_phys(Hcov[:, :, keep].astype(np.float64))
    ref_dh = pr.to_cov(pr.s.rhs_h(Ep))[:, :, pos]
    ref_de = pr.to_cov(pr.s.rhs_e(Hp))[:, :, pos]
    eh = rel_err(dH[:, :, centers], ref_dh)
    ee = rel_err(dE[:, :, centers], ref_de)
    print(f"n={n} p={p} sampled {len(centers)}: dH {eh:.2e} dE {ee:.2e}")
    assert eh < 1e-5 and ee < 1e-5


def test_estimate_dt_fp32_path_at_p8():
    """Above the FP64 orders the power iteration runs on FP32 vectors; both sides
    approach rho from below, so they agree to within the iteration's convergence."""
    verts, tets = synth.kuhn_mesh(1)
    pr = Pair(verts, tets, 8)
    est_or = pr.s.spectral_radius(150, synth.splitmix64(5, 3 * pr.s.N * 6))
    m = P.Mesh(verts, tets).set_order(8)
    dt, est = m.estimate_dt(cfl=0.5, iters=150, seed=5)
    print(f"p=8 rho: library {est:.6e}, oracle {est_or:.6e}")
    assert abs(est - est_or) < 1e-2 * est_or


def test_config_16cube_p4_fp32_1000_steps():
    """The 16^3 x 6, p = 4 FP32 workload over its full 1000 steps: the leapfrog invariant Q
    (checked every 100 steps in FP64) drifts by less than 1e-6 relative, and the FP32 run
    stays within 1e-5 (energy norm) of the FP64 run of the same library, whose operator is
    pinned to the oracle above (the oracle itself is too slow for 24,576 tets x 1000 steps)."""
    from paper_1104_4208_amd.project import project_covariant

    w = synth.WORKLOADS["cube16_p4_f32"]
    d = synth.build_workload(w)
    verts, tets = d["verts"], d["tets"]
    m = P.Mesh(verts, tets).set_order(w.p).set_material(d["eps"], d["mu"])
    dt, _ = m.estimate_dt(cfl=0.5, iters=20, seed=w.seed)
    E0 = np.ascontiguousarray(project_covariant(verts, tets, w.p, d["field"].E))
    E32, H32 = dev(E0, torch.float32), torch.zeros((3, P.num_modes(w.p), tets.shape[0]), dtype=torch.float32, device="cuda")
    E64, H64 = dev(E0, torch.float64), torch.zeros_like(H32, dtype=torch.float64)
    _, Q0 = m.energy(E32, H32, dt=dt)
    worst_q = 0.0
    for blk in range(10):
        m.step(E32, H32, dt, 100)
        m.step(E64, H64, dt, 100)
        _, Q = m.energy(E32, H32, dt=dt)
        worst_q = max(worst_q, abs(Q - Q0) / Q0)
    dE, dH = E32.double() - E64, H32.double() - H64
    num, _ = m.energy(dE.contiguous(), dH.contiguous())
    den, _ = m.energy(E64, H64)
    err = math.sqrt(num / den)
    print(f"16^3 p4 1000 steps: Q drift {worst_q:.2e}, FP32 vs FP64 {err:.2e}")
    assert worst_q < 1e-6
    assert err < 1e-5


def test_rejected_material_leaves_mesh_unchanged():
    """set_material checks every value before it uploads anything: after a call
    rejected for a bad permeability the operator is still the previous one."""
    rng = np.random.default_rng(21)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K, N = tets.shape[0], P.num_modes(3)
    m = P.Mesh(verts, tets).set_order(3).set_material(rng.choice([1.0, 4.0], size=K), rng.uniform(1, 2, K))
    E = dev(rng.standard_normal((3, N, K)), torch.float64)
    H = dev(rng.standard_normal((3, N, K)), torch.float64)
    before = [host(x) for x in m.apply_curl(E, H)]
    bad_mu = np.ones(K)
    bad_mu[K - 1] = 0.0
    with pytest.raises(P.DGMError):
        m.set_material(np.full(K, 2.0), bad_mu)
    after = [host(x) for x in m.apply_curl(E, H)]
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    # and a later valid call takes effect
    m.set_material(np.full(K, 2.0), None)
    changed = host(m.apply_curl(None, H)[0])
    assert not np.array_equal(changed, before[0])


def test_operator_spectrum_six_tets_p4():
    """The library's FP64 operator on the six-tet cube at p = 4, assembled column by
    column, has the oracle's spectrum (which contains the cube's 2 pi^2 and 3 pi^2
    resonances with their multiplicities; see the oracle tests)."""
    verts, tets = synth.kuhn_mesh(1)
    pr = Pair(verts, tets, 4)
    Ah, Ae = pr.s.assemble()
    m = P.Mesh(verts, tets).set_order(4)
    n = 6 * pr.s.N * 3
    Ahg, Aeg = np.zeros((n, n)), np.zeros((n, n))
    for col in range(n):
        u = np.zeros(n)
        u[col] = 1.0
        Ucov = dev(pr.to_cov(u.reshape(6, pr.s.N, 3)), torch.float64)
        dE, dH = m.apply_curl(Ucov, Ucov)
        Ahg[:, col] = pr.to_phys(host(dH)).ravel()
        Aeg[:, col] = pr.to_phys(host(dE)).ravel()
    lo = np.sort(np.linalg.eigvals(-Ah @ Ae).real)
    lg = np.sort(np.linalg.eigvals(-Ahg @ Aeg).real)
    top = lo.max()
    print(f"max eigenvalue difference {np.abs(lg - lo).max() / top:.2e} of the largest")
    assert np.abs(lg - lo).max() < 1e-9 * top
    r = lg / np.pi ** 2
    assert np.sum(np.abs(r - 2) < 0.01) == 3 and np.sum(np.abs(r - 3) < 0.015) == 2


@pytest.mark.parametrize("n,p,dtype,tol", [(32, 6, torch.float32, 1e-5), (24, 8, torch.float32, 1e-5),
                                            (16, 4, torch.float32, 1e-5), (32, 6, torch.float64, 1e-10),
                                            (16, 4, torch.float64, 1e-10)])
def test_full_size_step_sampled(n, p, dtype, tol):
    """One leapfrog step of a full-size FP32 mesh (32^3 x 6 at p = 6 is the benchmark's,
    streaming instantiation; 24^3 x 6 at p = 8 the dense comparison's; 16^3 x 6 at p = 4 fits
    the cache, plain instantiation) through dgm_step with half the stable step, checked on
    sampled elements against the oracle stepping their two-ring patch.  The E update of an
    element reads the H update of its neighbours, which reads E of theirs, so the patch's own
    outer faces only touch elements two rings out.  Both the new state and its increment
    over the step are compared.  In FP64 the 32^3 mesh runs the streaming FP64 kernel."""
    rng = np.random.default_rng(n + p)
    verts, tets = synth.kuhn_mesh(n, 0.1, rng)
    K = tets.shape[0]
    N = P.num_modes(p)
    eps = rng.choice([1.0, 4.0], size=K)
    m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
    npt = np.float32 if dtype == torch.float32 else np.float64
    E0 = rng.standard_normal((3, N, K)).astype(npt)
    H0 = rng.standard_normal((3, N, K)).astype(npt)
    dt, _ = m.estimate_dt(cfl=0.5, iters=20, seed=n)
    E, H = dev(E0, dtype), dev(H0, dtype)
    m.step(E, H, dt, 1)
    E1, H1 = host(E), host(H)
    centers = np.unique(np.concatenate([rng.integers(0, K, 6), [0, K - 1]]))
    ring1, _, _ = patch(tets, centers)
    keep, ptets, _ = patch(tets, ring1)
    pos = [int(np.nonzero(keep == c)[0][0]) for c in centers]
    pr = Pair(verts, ptets, p, eps[keep], None)
    Er, Hr = pr.s.step(pr.to_phys(E0[:, :, keep].astype(np.float64)), pr.to_phys(H0[:, :, keep].astype(np.float64)),
                       dt, 1)
    ref_E, ref_H = pr.to_cov(Er)[:, :, pos], pr.to_cov(Hr)[:, :, pos]
    E0c, H0c = E0[:, :, centers].astype(np.float64), H0[:, :, centers].astype(np.float64)
    errs = [rel_err(E1[:, :, centers], ref_E), rel_err(H1[:, :, centers], ref_H),
            rel_err(E1[:, :, centers] - E0c, ref_E - E0c), rel_err(H1[:, :, centers] - H0c, ref_H - H0c)]
    print(f"{n}^3 p{p} {dtype} one step (dt {dt:.2e}), {len(centers)} sampled elements ({len(keep)} in the patches): "
          f"E {errs[0]:.2e} H {errs[1]:.2e} dE {errs[2]:.2e} dH {errs[3]:.2e}")
    assert max(errs) < tol


def test_check_interval_reports_unstable():
    """With a check interval, dgm_step stops a run whose state is no longer finite
    (time step far above 2/sqrt(rho): leapfrog grows by about (dt w)^2 per step, so FP32
    overflows within a few tens of steps) and returns DGM_ERR_UNSTABLE; a stable step
    passes every check, and without checks the same unstable call returns DGM_OK."""
    verts, tets = synth.kuhn_mesh(2)
    m = P.Mesh(verts, tets).set_order(2)
    K, N = tets.shape[0], P.num_modes(2)
    rng = np.random.default_rng(17)
    E0 = dev(rng.standard_normal((3, N, K)), torch.float32)
    dt, _ = m.estimate_dt(cfl=0.5, iters=20, seed=1)
    E, H = E0.clone(), torch.zeros_like(E0)
    m.set_check_interval(10)
    m.step(E, H, dt, 100)  # stable: every check passes
    assert torch.isfinite(E).all() and torch.isfinite(H).all()
    E, H = E0.clone(), torch.zeros_like(E0)
    with pytest.raises(P.DGMError, match="DGM_ERR_UNSTABLE"):
        m.step(E, H, 100 * dt, 200)
    m.set_check_interval(0)
    E, H = E0.clone(), torch.zeros_like(E0)
    m.step(E, H, 100 * dt, 200)
    assert not bool(torch.isfinite(E).all())
