"""Dense matrix-core variant (16-bit operands, FP32 accumulation) against the
FP64 oracle and against the FP32 sparse path.

Tolerances follow from the operand rounding: BF16 keeps 8 significant bits
(unit roundoff u = 2^-8), FP16 keeps 11 (u = 2^-11).  One application sums
at most 3N + 8 NF products of rounded operands, so the error relative to the
largest coefficient is bounded by a small multiple of u times the ratio of the
summed magnitudes to the result; 16 u (6e-2 BF16, 8e-3 FP16) leaves room for
that ratio on random fields.  Measured errors are printed.
"""
import math

import numpy as np
import pytest

import synth
from gpu_helpers import Pair, patch, rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1104_4208_amd as P  # noqa: E402

TOL = {P.DGM_BF16: 16 * 2.0 ** -8, P.DGM_F16: 16 * 2.0 ** -11}
NAME = {P.DGM_BF16: "bf16", P.DGM_F16: "fp16"}


def dev(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("prec", [P.DGM_BF16, P.DGM_F16])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_dense_apply_curl_parity(p, prec):
    rng = np.random.default_rng(200 + p)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    K = tets.shape[0]
    eps, mu = rng.uniform(1, 4, K), rng.uniform(1, 2, K)
    pr = Pair(verts, tets, p, eps, mu)
    E = rng.standard_normal((K, pr.s.N, 3))
    H = rng.standard_normal((K, pr.s.N, 3))
    m = P.Mesh(verts, tets).set_order(p).set_material(eps, mu)
    dE, dH = m.apply_curl_dense(dev(pr.to_cov(E)), dev(pr.to_cov(H)), prec=prec)
    eh = rel_err(host(dH), pr.to_cov(pr.s.rhs_h(E)))
    ee = rel_err(host(dE), pr.to_cov(pr.s.rhs_e(H)))
    print(f"dense {NAME[prec]} p={p}: dH {eh:.2e} dE {ee:.2e}")
    assert eh < TOL[prec] and ee < TOL[prec]


@pytest.mark.parametrize("prec", [P.DGM_BF16, P.DGM_F16])
def test_dense_step_against_oracle(prec):
    rng = np.random.default_rng(4)
    verts, tets = synth.kuhn_mesh(3, 0.1, rng)
    p = 4
    pr = Pair(verts, tets, p)
    E = pr.s.project(synth.te101().E)
    H = np.zeros_like(E)
    dt = 1.0 / math.sqrt(pr.s.spectral_radius(40, synth.splitmix64(4, E.size)))
    m = P.Mesh(verts, tets).set_order(p)
    Eg, Hg = dev(pr.to_cov(E)), dev(pr.to_cov(H))
    _, Q0 = m.energy(Eg, Hg, dt=dt)
    m.step_dense(Eg, Hg, dt, 50, prec=prec)
    E1, H1 = pr.s.step(E, H, dt, 50)
    err = pr.s.rel_error(pr.to_phys(host(Eg)), pr.to_phys(host(Hg)), E1, H1)
    _, Q = m.energy(Eg, Hg, dt=dt)
    print(f"dense {NAME[prec]} 50 steps: rel err {err:.2e}, Q drift {abs(Q - Q0) / Q0:.2e}")
    assert err < TOL[prec]


@pytest.mark.parametrize("prec", [P.DGM_BF16, P.DGM_F16])
def test_dense_full_size_p8_sampled(prec):
    """The dense-variant workload size: 24^3 x 6 = 82,944 tets at p = 8, sampled elements."""
    rng = np.random.default_rng(24)
    verts, tets = synth.kuhn_mesh(24, 0.0, None)
    K, p = tets.shape[0], 8
    N = P.num_modes(p)
    m = P.Mesh(verts, tets).set_order(p)
    Ecov = rng.standard_normal((3, N, K)).astype(np.float32)
    Hcov = rng.standard_normal((3, N, K)).astype(np.float32)
    dE, dH = m.apply_curl_dense(dev(Ecov), dev(Hcov), prec=prec)
    dE, dH = host(dE), host(dH)
    centers = np.unique(np.concatenate([rng.integers(0, K, 10), [0, K - 1]]))
    keep, ptets, pos = patch(tets, centers)
    pr = Pair(verts, ptets, p)
    ref_dh = pr.to_cov(pr.s.rhs_h(pr.to_phys(Ecov[:, :, keep].astype(np.float64))))[:, :, pos]
    ref_de = pr.to_cov(pr.s.rhs_e(pr.to_phys(Hcov[:, :, keep].astype(np.float64))))[:, :, pos]
    eh, ee = rel_err(dH[:, :, centers], ref_dh), rel_err(dE[:, :, centers], ref_de)
    print(f"dense {NAME[prec]} n=24 p=8 sampled: dH {eh:.2e} dE {ee:.2e}")
    assert eh < TOL[prec] and ee < TOL[prec]
