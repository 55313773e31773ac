"""Frequency extraction of the resonance workload (CPU): the matrix pencil recovers
known rotations exactly, and applied to a leapfrog signal of the oracle it returns
eigenvalues of the oracle's assembled operator (the discrete resonances)."""
import math

import numpy as np

import synth
from gpu_helpers import Pair
from paper_1104_4208_amd.resonance import exact_cube_frequencies, frequencies, pencil


def test_pencil_recovers_closed_form_rotations():
    n = np.arange(400)
    th = np.array([0.11, 0.37, 0.52])
    amp = np.array([1.0, 0.5, 0.25])
    y = (amp[:, None] * np.cos(th[:, None] * n[None, :] + np.array([0.3, 1.1, -0.7])[:, None])).sum(0) + 0.2
    z, a = pencil(y, 7)
    got = np.sort(np.abs(np.angle(z)))
    assert np.allclose(got[1::2], th, atol=1e-10) and np.allclose(got[2::2], th, atol=1e-10)
    assert abs(np.sort(np.abs(np.angle(z)))[0]) < 1e-10  # the constant
    dt = 0.01
    om = [o for o, _ in frequencies(y, dt, rank=7, k=3)]
    assert np.allclose(om, (2 / dt) * np.sin(th / 2), rtol=1e-9)


def test_exact_cube_frequencies():
    f = exact_cube_frequencies(4.0)
    assert abs(f[0] - math.pi * math.sqrt(2) / 2) < 1e-14 and abs(f[1] - math.pi * math.sqrt(3) / 2) < 1e-14


def test_leapfrog_signal_gives_discrete_eigenvalues():
    verts, tets = synth.kuhn_mesh(1)
    pr = Pair(verts, tets, 2)
    s = pr.s
    Ah, Ae = s.assemble()
    ev = np.sort(np.linalg.eigvals(-Ah @ Ae).real)
    dt = 1.0 / math.sqrt(ev[-1])
    E = s.project(synth.te101().E)
    H = np.zeros_like(E)
    w = np.random.default_rng(0).standard_normal(E.shape)
    sig = np.empty(1500)
    for i in range(len(sig)):
        E, H = s.step(E, H, dt, 1)
        sig[i] = (w * E).sum()
    for om, amp in frequencies(sig, dt, rank=61, k=3):
        near = ev[np.argmin(np.abs(ev - om * om))]
        assert abs(om * om - near) < 1e-6 * near, (om * om, near)
