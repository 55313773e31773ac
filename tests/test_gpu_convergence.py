"""h-convergence of the library against the closed-form TE101 standing wave of the
unit-cube cavity (FP64, T = 1, dt from the power iteration, so dt ~ h): the observed
spatial rates per order are printed and must reach at least p - 0.3 (central flux,
so p + 1 is not guaranteed).  Leapfrog is second order in time, so for p >= 3 the
step runs at CFL 0.05 instead of 0.5, which keeps the time error (dt^2) below the
space error at these meshes."""
import math

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1104_4208_amd as P  # noqa: E402
from paper_1104_4208_amd.project import project_covariant  # noqa: E402


def _error(n, p, cfl, T=1.0):
    verts, tets = synth.kuhn_mesh(n)
    mode = synth.te101()
    m = P.Mesh(verts, tets).set_order(p)
    dt0, _ = m.estimate_dt(cfl=cfl, iters=30, seed=1)
    nst = int(math.ceil(T / dt0))
    dt = T / nst
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    E = dev(project_covariant(verts, tets, p, mode.E))
    H = dev(project_covariant(verts, tets, p, lambda x: mode.H(x, -dt / 2)))  # leapfrog staggering
    m.step(E, H, dt, nst)
    Ee = dev(project_covariant(verts, tets, p, lambda x: mode.E(x, T)))
    He = dev(project_covariant(verts, tets, p, lambda x: mode.H(x, T - dt / 2)))
    num, _ = m.energy((E - Ee).contiguous(), (H - He).contiguous())
    den, _ = m.energy(Ee, He)
    return math.sqrt(num / den)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_te101_h_convergence(p):
    ns = (2, 4, 8)
    cfl = 0.5 if p <= 2 else 0.05
    errs = [_error(n, p, cfl) for n in ns]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(len(ns) - 1)]
    print(f"p={p} (CFL {cfl}): errors {['%.3e' % e for e in errs]}, rates {['%.2f' % r for r in rates]}")
    assert rates[-1] > p - 0.3
