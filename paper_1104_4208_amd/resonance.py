"""Resonance frequencies of a cavity from the time signal of the leapfrog run.

The numerical example of Section 2.2 computes the smallest eigenvalues of the
discrete Maxwell operator of a resonator.  Here the resonator is the unit-cube PEC
cavity (exact values pi * sqrt(m^2 + n^2 + l^2) / sqrt(eps mu)) and the eigenvalues
come from the time domain: the symplectic Euler step maps a mode of the
semi-discrete system with frequency omega to the rotation exp(+-i theta) with
2 - 2 cos(theta) = dt^2 omega^2 (Section 3), so omega = (2 / dt) sin(theta / 2).
The run records a generic linear functional of E after every step
(dgm_step_probe) and the matrix-pencil method (Hua and Sarkar, 1990) extracts the
rotations of the signal's dominant components.

    python -m paper_1104_4208_amd.resonance [--n 8] [--p 4] [--t-end 12]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np


def pencil(signal, rank: int):
    """Matrix pencil of a uniformly sampled signal: the `rank` poles z_i and the
    complex amplitudes a_i of signal[n] ~ sum_i a_i z_i^n (least squares)."""
    y = np.asarray(signal, dtype=np.float64)
    T = len(y)
    L = T // 2
    Y = np.lib.stride_tricks.sliding_window_view(y, L + 1)  # Hankel rows, (T - L) x (L + 1)
    _, _, Vh = np.linalg.svd(Y, full_matrices=False)
    V = Vh[:rank].T
    z = np.linalg.eigvals(np.linalg.pinv(V[:-1]) @ V[1:])
    Z = z[None, :] ** np.arange(T)[:, None]
    a = np.linalg.lstsq(Z, y.astype(complex), rcond=None)[0]
    return z, a


def frequencies(signal, dt: float, rank: int = 61, k: int = 4, min_theta: float = 1e-6):
    """The k dominant angular frequencies of a leapfrog signal (largest amplitude
    first), from the pencil poles: theta = |arg z|, omega = (2/dt) sin(theta/2).
    Static components (theta ~ 0) and the conjugate twin of each pole are dropped."""
    z, a = pencil(signal, rank)
    th = np.abs(np.angle(z))
    keep = th > min_theta
    om = (2.0 / dt) * np.sin(th[keep] / 2.0)
    amp = np.abs(a[keep])
    out = []
    for i in np.argsort(-amp):
        if all(abs(om[i] - o) > 1e-9 * max(1.0, om[i]) for o, _ in out):
            out.append((float(om[i]), float(amp[i])))
        if len(out) == k:
            break
    return out


def exact_cube_frequencies(eps: float = 1.0, mu: float = 1.0, count: int = 6):
    """Smallest distinct resonance frequencies of the unit-cube PEC cavity:
    pi sqrt(m^2 + n^2 + l^2) / sqrt(eps mu) with at most one index zero."""
    vals = set()
    for m in range(4):
        for n in range(4):
            for l in range(4):
                if (m == 0) + (n == 0) + (l == 0) <= 1:
                    vals.add(m * m + n * n + l * l)
    return [math.pi * math.sqrt(v / (eps * mu)) for v in sorted(vals)[:count]]


# initial field of the resonance runs: four cube-cavity modes of distinct frequencies
# pi sqrt(2), pi sqrt(3), pi sqrt(5), pi sqrt(6) (divergence-free amplitude vectors)
FOUR_MODES = [((1, 0, 1), (0.0, 1.0, 0.0)), ((1, 1, 1), (0.8, -0.8, 0.0)),
              ((2, 0, 1), (0.0, 0.6, 0.0)), ((2, 1, 1), (0.5, -1.0, 0.0))]


def cavity_run(n: int, p: int, steps: int | None = None, dtype: str = "f32", eps: float = 1.0, rank: int = 61,
               k: int = 4, cfl: float = 0.5, seed: int = 6, t_end: float = 12.0):
    """Leapfrog run of the cube cavity (n^3 Kuhn cells, order p) from the four-mode
    field FOUR_MODES with H = 0, probed by a seeded random functional, for `steps`
    steps (default: up to time t_end, about ten periods of the lowest mode); returns
    the k dominant frequencies, each matched to the nearest exact cavity frequency,
    and the time of the run."""
    import torch

    import synth
    from . import dgmax as D
    from .project import project_covariant

    rng = np.random.default_rng(seed)
    verts, tets = synth.kuhn_mesh(n)
    K = tets.shape[0]
    m = D.Mesh(verts, tets).set_order(p).set_material(np.full(K, eps), None)
    dt, rho = m.estimate_dt(cfl=cfl, iters=30, seed=seed)
    if steps is None:
        steps = int(math.ceil(t_end / dt))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    fld = synth.ModeSum([synth.CavityMode(lmn, amp, eps, 1.0) for lmn, amp in FOUR_MODES])
    E = torch.tensor(np.ascontiguousarray(project_covariant(verts, tets, p, fld.E)), dtype=tdt, device="cuda")
    H = torch.zeros_like(E)
    w = torch.tensor(rng.standard_normal(E.shape), dtype=tdt, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sig = m.step_probe(E, H, dt, steps, w)
    run_s = time.perf_counter() - t0
    t1 = time.perf_counter()
    found = frequencies(sig, dt, rank=rank, k=k)
    fit_s = time.perf_counter() - t1
    m.close()
    exact = exact_cube_frequencies(eps, count=8)
    match = []
    for o, a in found:
        x = min(exact, key=lambda v: abs(v - o))
        match.append({"omega": o, "amplitude": a, "exact": x, "rel_err": abs(o - x) / x})
    return {"n": n, "tets": K, "p": p, "dtype": dtype, "eps": eps, "steps": steps, "dt": dt, "rank": rank,
            "init": "four cavity modes, omega = pi sqrt(2, 3, 5, 6)", "found": match,
            "run_s": run_s, "fit_s": fit_s, "dof_updates_per_s": 6 * D.num_modes(p) * K * steps / run_s}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--steps", type=int, default=None, help="default: up to time --t-end")
    ap.add_argument("--t-end", type=float, default=12.0)
    ap.add_argument("--dtype", default="f32")
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rep = cavity_run(a.n, a.p, a.steps, a.dtype, t_end=a.t_end)
    line = json.dumps(rep)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
