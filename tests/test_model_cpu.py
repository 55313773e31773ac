"""The kernels' formulation (product tables, derivative frame, stored frame,
tangential-trace jumps) against the oracle, on the CPU through a numpy model."""
import numpy as np
import pytest

import oracle
import synth
from kernel_model import Model
from paper_1104_4208_amd.project import project_covariant, sorted_geometry


def _case(name, rng):
    if name == "one":
        return synth.single_tet(np.array([[0.1, 0, 0], [1, 0.2, 0], [0, 1.1, 0.1], [0.2, 0.1, 0.9]]))
    if name == "two":
        return synth.two_tets(rng)
    return synth.kuhn_mesh(2, 0.1, rng)


@pytest.mark.parametrize("name", ["one", "two", "cube"])
@pytest.mark.parametrize("p", [1, 3])
def test_model_matches_oracle(name, p):
    rng = np.random.default_rng(7)
    verts, tets = _case(name, rng)
    K = tets.shape[0]
    eps, mu = rng.uniform(1, 4, K), rng.uniform(1, 2, K)
    ts, _, F = sorted_geometry(verts, tets)
    s = oracle.Solver(oracle.build_mesh(verts, ts), p, eps, mu)
    model = Model(verts, tets, p, eps, mu)
    # random physical coefficients, shared through the covariant map
    E = rng.standard_normal((K, s.N, 3))
    H = rng.standard_normal((K, s.N, 3))
    perm = _perm(p, s)
    Ecov = np.einsum("kji,kmj->imk", F, E)[:, perm, :]
    Hcov = np.einsum("kji,kmj->imk", F, H)[:, perm, :]
    dh = np.einsum("kji,kmj->imk", F, s.rhs_h(E))[:, perm, :]
    de = np.einsum("kji,kmj->imk", F, s.rhs_e(H))[:, perm, :]
    assert np.abs(model.rate(Ecov, 0) - dh).max() < 1e-10 * np.abs(dh).max()
    assert np.abs(model.rate(Hcov, 1) - de).max() < 1e-10 * np.abs(de).max()


def _perm(p, s):
    """Row permutation oracle order -> product order, matched by (i,j,k)."""
    from paper_1104_4208_amd.gen.basis import volume_modes

    idx = {m: r for r, m in enumerate(s.modes())}
    return [idx[m] for m in volume_modes(p)]


def test_projection_matches_oracle():
    rng = np.random.default_rng(3)
    verts, tets = synth.kuhn_mesh(2, 0.1, rng)
    p = 3
    ts, _, F = sorted_geometry(verts, tets)
    s = oracle.Solver(oracle.build_mesh(verts, ts), p)
    mode = synth.te101()
    e_or = np.einsum("kji,kmj->imk", F, s.project(mode.E))[:, _perm(p, s), :]
    e_pr = project_covariant(verts, tets, p, mode.E)
    assert np.abs(e_or - e_pr).max() < 1e-13
