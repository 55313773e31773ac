"""dgm_step_noalloc (the allocation-free step) against dgm_step, through the C-ABI.

Both entry points run the same kernels on the same inputs, so the results must be
bitwise equal (well inside the FP64 1e-10 / FP32 1e-5 tolerances against the oracle
that dgm_step itself is held to).  Two calls in a row on different meshes, the second
smaller, check that the shared static workspace carries nothing over from one call to
the next; a mesh beyond the workspace is rejected before any work.
"""

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1104_4208_amd as P  # noqa: E402
from paper_1104_4208_amd import dgmax as D  # noqa: E402


def _run(m, entry, E0, H0, dt, nsteps):
    E, H = E0.clone(), H0.clone()
    lib = P.load_library()
    fn = lib.dgm_step_noalloc if entry == "noalloc" else lib.dgm_step
    code = D.DGM_F32 if E.dtype == torch.float32 else D.DGM_F64
    D._check(fn(m.handle, code, D._ptr(E), D._ptr(H), float(dt), int(nsteps), D._stream()))
    torch.cuda.synchronize()
    return E.cpu(), H.cpu()


def _case(n, p, dtype, seed, nsteps, check_every=0):
    rng = np.random.default_rng(seed)
    verts, tets = synth.kuhn_mesh(n, 0.1, rng)
    K, N = tets.shape[0], P.num_modes(p)
    m = P.Mesh(verts, tets).set_order(p).set_material(rng.choice([1.0, 4.0], size=K), None)
    m.set_check_interval(check_every)
    E0 = torch.tensor(rng.standard_normal((3, N, K)), dtype=dtype, device="cuda")
    H0 = torch.tensor(rng.standard_normal((3, N, K)), dtype=dtype, device="cuda")
    dt, _ = m.estimate_dt(cfl=0.5, iters=10, seed=seed)
    print(f"no-alloc case: {n}^3 x 6 = {K} tets, p={p}, {dtype}, {nsteps} steps, check every {check_every}",
          flush=True)
    Ea, Ha = _run(m, "noalloc", E0, H0, dt, nsteps)
    Eb, Hb = _run(m, "step", E0, H0, dt, nsteps)
    tol = 1e-5 if dtype == torch.float32 else 1e-10
    scale = float(max(Eb.abs().max(), Hb.abs().max()))
    diff = float(max((Ea - Eb).abs().max(), (Ha - Hb).abs().max())) / scale
    assert diff <= tol, diff
    assert torch.equal(Ea, Eb) and torch.equal(Ha, Hb)
    return m


def test_noalloc_matches_step_two_calls_second_smaller():
    _case(8, 6, torch.float32, 31, 7)               # 3,072 tets: 5.5 MB of workspace
    _case(3, 4, torch.float32, 32, 5, check_every=2)  # smaller, with the finiteness checks
    _case(4, 3, torch.float64, 33, 4)               # FP64


def test_noalloc_rejects_meshes_beyond_the_workspace():
    verts, tets = synth.kuhn_mesh(20)  # 48,000 tets at p = 6: 86 MB of FP32 traces
    m = P.Mesh(verts, tets).set_order(6)
    E = m.zeros()
    H = m.zeros()
    lib = P.load_library()
    rc = lib.dgm_step_noalloc(m.handle, D.DGM_F32, D._ptr(E), D._ptr(H), 1e-3, 1, D._stream())
    assert rc == -1 and "too large" in lib.dgm_last_error().decode()
    assert int(lib.dgm_step_noalloc(m.handle, D.DGM_F32, D._ptr(E), D._ptr(H), 1e-3, 0, D._stream())) == -1
