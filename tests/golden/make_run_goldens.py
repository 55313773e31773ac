"""Write the run-length goldens of the FP32 workloads from the FP64 oracle.

    python tests/golden/make_run_goldens.py [cfg2|cfg3|cfg4|cfg3_var|cfg3_stab|cfg3_mixed ...]

Calls only the oracle (and the shared seeded input generators in synth/): no
value here comes from the HIP library.  Each workload's recipe (mesh kind,
order, material law, initial field, CFL 0.5 time step, full step count) is run
on a reduced cube of 4^3 cells x 6 tetrahedra, so that the FP64 oracle finishes
in minutes while the run keeps its full length (Section 3, symplectic Euler,
H first).  Stored per workload (``run_<name>.npz``, plain arrays, no pickles):

  verts, tets, eps, mu  the reduced mesh and material (inputs, as drawn)
  dt, steps, every      the step, the step count, the checkpoint interval
  init_checksum         sum of the oracle's initial E coefficients (input check)
  sample                element indices whose coefficients are stored
  E_s, H_s              (C, S, N, 3) physical Cartesian coefficients of the sampled
                        elements at each of the C checkpoints (oracle mode order)
  W, Q                  (C,) FP64 energy and leapfrog invariant of the whole mesh
  E0W                   energy of the initial state
  E_end, H_end          (K, N, 3) the whole final state, for the energy-norm error
                        of the run

Workload recipes (same seeds and draw order as the full-size workloads):
  cfg2  p = 4, eps = mu = 1, three cavity modes with N(0,1) amplitudes (seed 2),
        1000 steps, checkpoint every 100
  cfg3  p = 6, vertices jittered U(+-0.1 h), eps in {1,4} with probability 1/2,
        mu = 1, three cavity modes (seed 3), 500 steps, checkpoint every 50
  cfg4  p = 8, eps = mu = 1, random physical modal coefficients N(0,1) for E
        (oracle mode order), H = 0, rescaled to W = 1 (seed 4), 200 steps,
        checkpoint every 20
  cfg3_var  cfg3's mesh, draws and initial field with the material linear inside the
        elements (Section 3.3.2, oracle/varcoef.py): eps at each element's vertices =
        the element's eps in {1,4} times 1 + 0.25 sin(3x) cos(2z), mu = 1 + 0.2 y; eps
        and mu are stored as (K,4) vertex values (sorted vertex order); W and Q are taken
        with the approximate mass matrices
  cfg3_stab cfg3 with the stabilised central flux and face unknowns H^F (Section 2.1,
        oracle/stab.py, alpha = p^2), H^F = 0 at the start; the time step from the
        stabilised operator's power iteration; W and Q include the face term, and the
        final face unknowns are stored as b_end (faces, NF, 3)
  cfg3_mixed cfg3 with mixed orders (Section 2, oracle/mixed.py): E of degree 7, H of
        degree 6; the power iteration starts from an H-sized vector
The time step is 0.5 * 2 / sqrt(rho), rho from 40 oracle power iterations
started from SplitMix64(seed).
"""
from __future__ import annotations

import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

CELLS = 4

RECIPES = {
    "cfg2": dict(p=4, seed=2, jitter=0.0, eps=(1.0,), init="three_mode", steps=1000, every=100),
    "cfg3": dict(p=6, seed=3, jitter=0.1, eps=(1.0, 4.0), init="three_mode", steps=500, every=50),
    "cfg4": dict(p=8, seed=4, jitter=0.0, eps=(1.0,), init="random", steps=200, every=20),
    "cfg3_var": dict(p=6, seed=3, jitter=0.1, eps=(1.0, 4.0), init="three_mode", steps=500, every=50, linear=True),
    "cfg3_stab": dict(p=6, seed=3, jitter=0.1, eps=(1.0, 4.0), init="three_mode", steps=500, every=50, stab=True),
    "cfg3_mixed": dict(p=6, pE=7, seed=3, jitter=0.1, eps=(1.0, 4.0), init="three_mode", steps=500, every=50),
}


def linear_material(verts, tets, eps):
    """Vertex values (K,4) of the linear-material recipe from the per-element draw."""
    x = np.asarray(verts, float)[tets]
    eps_v = eps[:, None] * (1.0 + 0.25 * np.sin(3.0 * x[..., 0]) * np.cos(2.0 * x[..., 2]))
    mu_v = 1.0 + 0.2 * x[..., 1]
    return eps_v, mu_v


def setup(name):
    """Mesh, material, oracle solver and initial state of a reduced workload, drawn in
    the fixed order jitter -> eps -> amplitudes (or random coefficients)."""
    r = RECIPES[name]
    rng = np.random.default_rng(r["seed"])
    verts, tets = synth.kuhn_mesh(CELLS, r["jitter"], rng if r["jitter"] > 0 else None)
    tets = np.sort(tets, axis=1)
    K = tets.shape[0]
    eps = rng.choice(np.asarray(r["eps"]), size=K) if len(r["eps"]) > 1 else np.full(K, r["eps"][0])
    mu = np.ones(K)
    if r.get("linear"):
        from oracle.varcoef import VarMaterialSolver

        eps, mu = linear_material(verts, tets, eps)
        s = VarMaterialSolver(oracle.build_mesh(verts, tets), r["p"], eps, mu)
    elif r.get("pE"):
        from oracle.mixed import MixedSolver

        s = MixedSolver(oracle.build_mesh(verts, tets), r["pE"], r["p"], eps, mu)
        E = s.project(synth.three_mode_sum(rng).E, "E")
        return r, verts, tets, eps, mu, s, E, np.zeros((K, s.NH, 3))
    elif r.get("stab"):
        from oracle.stab import StabilizedSolver

        s = StabilizedSolver(oracle.build_mesh(verts, tets), r["p"], eps, mu, alpha0=1.0)
    else:
        s = oracle.Solver(oracle.build_mesh(verts, tets), r["p"], eps, mu)
    if r["init"] == "three_mode":
        E = s.project(synth.three_mode_sum(rng).E)
    else:
        E = rng.standard_normal((K, s.N, 3))
    H = np.zeros_like(E)
    if r["init"] == "random":
        E = E / math.sqrt(s.energy(E, H))
    return r, verts, tets, eps, mu, s, E, H


def sample_elements(K):
    """16 elements spread over the mesh, first and last included."""
    return np.unique(np.linspace(0, K - 1, 16).round().astype(np.int64))


def make(name):
    r, verts, tets, eps, mu, s, E, H = setup(name)
    if r.get("stab"):
        return make_stab(name, r, verts, tets, eps, mu, s, E, H)
    t0 = time.time()
    rho = s.spectral_radius(40, synth.splitmix64(r["seed"], H.size if r.get("pE") else E.size))
    dt = 1.0 / math.sqrt(rho)
    smp = sample_elements(s.K)
    C = r["steps"] // r["every"]
    E_s = np.empty((C, len(smp), E.shape[1], 3))
    H_s = np.empty((C, len(smp), H.shape[1], 3))
    W = np.empty(C)
    Q = np.empty(C)
    checksum = float(E.sum())
    W0 = s.energy(E, H)
    for c in range(C):
        E, H = s.step(E, H, dt, r["every"])
        E_s[c], H_s[c] = E[smp], H[smp]
        W[c] = s.energy(E, H)
        Q[c] = s.leapfrog_invariant(E, H, dt)
        print(f"{name}: step {(c + 1) * r['every']}/{r['steps']} W {W[c]:.15e} Q {Q[c]:.15e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(HERE, f"run_{name}.npz")
    np.savez_compressed(out, verts=verts, tets=tets, eps=eps, mu=mu, dt=dt, steps=r["steps"], every=r["every"],
                        p=r["p"], seed=r["seed"], init_checksum=checksum, sample=smp, E_s=E_s, H_s=H_s, W=W, Q=Q,
                        E0W=W0, E_end=E, H_end=H)
    print(f"{name}: wrote {out}", flush=True)


def make_stab(name, r, verts, tets, eps, mu, s, E, H):
    """The stabilised recipe: the same checkpoints, with the face unknowns in the state."""
    t0 = time.time()
    b = s.zeros_faces()
    rho = s.spectral_radius_stab(40, synth.splitmix64(r["seed"], E.size))
    dt = 1.0 / math.sqrt(rho)
    smp = sample_elements(s.K)
    C = r["steps"] // r["every"]
    E_s = np.empty((C, len(smp), s.N, 3))
    H_s = np.empty_like(E_s)
    W = np.empty(C)
    Q = np.empty(C)
    checksum = float(E.sum())
    W0 = s.energy_stab(E, H, b)
    for c in range(C):
        E, H, b = s.step_stab(E, H, b, dt, r["every"])
        E_s[c], H_s[c] = E[smp], H[smp]
        W[c] = s.energy_stab(E, H, b)
        Q[c] = s.leapfrog_invariant_stab(E, H, b, dt)
        print(f"{name}: step {(c + 1) * r['every']}/{r['steps']} W {W[c]:.15e} Q {Q[c]:.15e} "
              f"({time.time() - t0:.0f} s)", flush=True)
    out = os.path.join(HERE, f"run_{name}.npz")
    np.savez_compressed(out, verts=verts, tets=tets, eps=eps, mu=mu, dt=dt, steps=r["steps"], every=r["every"],
                        p=r["p"], seed=r["seed"], init_checksum=checksum, sample=smp, E_s=E_s, H_s=H_s, W=W, Q=Q,
                        E0W=W0, E_end=E, H_end=H, b_end=b)
    print(f"{name}: wrote {out}", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or list(RECIPES):
        make(nm)
