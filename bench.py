#!/usr/bin/env python3
"""Benchmark: FP32 DG Maxwell leapfrog steps on one MI355X.

Workload (the p = 6 precision workload): the unit-cube PEC cavity split into
32^3 cells x 6 Kuhn tetrahedra = 196,608 tets, vertices jittered by U(+-0.1 h)
(seed 3), eps drawn from {1, 4} per element, mu = 1, order p = 6 (84 modes per
component, 99,090,432 DOFs), initial E = sum of three cavity modes with
N(0,1) amplitudes, H = 0, dt = 0.5 * 2 / sqrt(rho) from the library's power
iteration.  A step is one full symplectic-Euler step (H phase + E phase) over
the whole mesh.  Inputs are resident in HBM when the timed region starts.

    python bench.py [--gpus 1] [--steps 500] [--warmup 20]

Prints one JSON line.  value = 6 N K steps / wall time (DOF-updates/s).
roofline: the dominant kernel is the generated phase kernel; its algorithmic
traffic is 36 N + 40 bytes per element per launch (read the differentiated
field, read and write the updated field, 24 B of metric and 16 B of neighbour
codes); its average duration is measured live with HIP events on the stream it
is launched on (difference of a long and a one-step run, so the frame
conversions at the ends cancel).  roofline.alu: the generator's emitted
floating-point operations per element and launch against the FP32 vector peak
without packed FP32.  roofline.traffic and alu.valu_issue_frac: from the committed
counter summary when it was taken on the current kernel source.  The run then
continues to the configuration's 500 steps for the drift of the leapfrog
invariant.  stabilized_flux: the stabilised central flux (Section 2.1) on the same
mesh; mixed_orders: E of degree 7, H of degree 6 (Section 2) on the same mesh; linear_material:
eps and mu linear inside the elements through the approximate mass inverse (Section 3.3.2).  dense_variant: the p = 8 matrix-core comparison.  serving: the 256-request
trace, batched against sequential.  cpu_baseline: the FP64 oracle timed on a
bounded sample of the same workload (smaller cube, same order and recipe); the
same leg (the only code here that runs the oracle) reports under "accuracy" the
FP32 error against the oracle on that sample, each FP32 workload's recipe over its
full step count against the oracle's stored run, and the p = 8 operator errors of
the sparse and dense paths.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector peak without packed FP32 (the build disables packed FP32 instructions):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops (FMA) x 2.4 GHz
FP32_PEAK_TFLOPS = 78.6
# VALU instruction issue capacity: 256 CUs x 4 SIMDs, one wave64 instruction per 4 cycles, 2.4 GHz
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4
OPCOUNT_FILE = os.path.join(ROOT, "paper_1104_4208_amd", "csrc", "generated", "opcount.json")
WORKLOAD = dict(workload="pec_cube_cavity_kuhn32_p6_fp32", cells=32, tets=196608, p=6, modes=84,
                dofs=99090432, jitter=0.1, eps=[1, 4], steps_in_config=500, init="three cavity modes, seed 3")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phase_p6_cube32_traffic.json")


_T0 = time.perf_counter()


def progress(msg):
    """A line on stderr as each part of the run starts or ends (stdout carries the JSON line only)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def opcount(p):
    """Floating-point operations per element of one phase launch, as emitted by the
    generator (build step)."""
    with open(OPCOUNT_FILE) as fh:
        return json.load(fh)["orders"][str(p)]


def measured_counters():
    """The committed counter summary (bytes, VALU instructions per launch) if it was
    taken on the current generated p = 6 kernel source, else None."""
    import hashlib

    src = os.path.join(ROOT, "paper_1104_4208_amd", "csrc", "generated", "phase_p6.inc")
    if not (os.path.exists(TRAFFIC_FILE) and os.path.exists(src)):
        return None
    with open(TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    with open(src, "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()[:16]
    return tr if tr.get("kernel_source_sha256_16") == h else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-dense", action="store_true", help="skip the p=8 dense matrix-core comparison")
    ap.add_argument("--dense-steps", type=int, default=200)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving comparison")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--serve-nmax", type=int, default=24)
    ap.add_argument("--no-stab", action="store_true", help="skip the stabilised-flux leg")
    ap.add_argument("--stab-steps", type=int, default=100, help="steps of the stabilised and mixed-order legs")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-order leg")
    ap.add_argument("--no-var", action="store_true", help="skip the variable-material leg")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="first run three plain device copies of this many MiB (scale reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def build_inputs():
    import synth
    from paper_1104_4208_amd.project import project_covariant

    w = synth.WORKLOADS["cube32_p6_f32"]
    d = synth.build_workload(w)
    E0 = project_covariant(d["verts"], d["tets"], w.p, d["field"].E)
    return w, d, E0


def oracle_leg(target_seconds: float, dense: bool):
    """Everything that runs the FP64 oracle (nothing else in this file does).

    cpu_baseline: the oracle timed on a bounded sample of the workload (the same
    recipe on a 4^3-cell cube, 384 tets, p = 6), as many steps as fit in about
    target_seconds.  accuracy: the FP32 library run on the same sample and steps
    against the oracle (relative energy-norm error), and, with `dense`, one operator
    application of the p = 8 workload on sampled elements (patch meshes) for the
    sparse FP32 path and the dense BF16 / FP16 variants."""
    import torch

    import paper_1104_4208_amd as P
    import synth

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_helpers import Pair, patch, rel_err

    try:
        from threadpoolctl import threadpool_info

        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    rng = np.random.default_rng(3)
    verts, tets = synth.kuhn_mesh(4, 0.1, rng)
    K = tets.shape[0]
    eps = rng.choice([1.0, 4.0], size=K)
    pr = Pair(verts, tets, 6, eps)
    s = pr.s
    fld = synth.three_mode_sum(rng)
    E = s.project(fld.E)
    H = np.zeros_like(E)
    E0, H0 = E.copy(), H.copy()
    dt = 1e-3
    E, H = s.step(E, H, dt, 1)  # warm caches
    n, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < target_seconds or n < 2:
        E, H = s.step(E, H, dt, 1)
        n += 1
    el = time.perf_counter() - t0
    rate = 6 * s.N * K * n / el
    base = {"value": rate, "unit": "DOF-updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"FP64 oracle, 4^3 x 6 = {K} jittered tets, p=6, eps in {{1,4}}, {n} steps in {el:.1f} s"}
    # the FP32 library on the same sample, initial data and steps
    m = P.Mesh(verts, tets).set_order(6).set_material(eps, None)
    Eg = torch.tensor(np.ascontiguousarray(pr.to_cov(E0)), dtype=torch.float32, device="cuda")
    Hg = torch.tensor(np.ascontiguousarray(pr.to_cov(H0)), dtype=torch.float32, device="cuda")
    m.step(Eg, Hg, dt, n + 1)
    torch.cuda.synchronize()
    err = s.rel_error(pr.to_phys(Eg.double().cpu().numpy()), pr.to_phys(Hg.double().cpu().numpy()), E, H)
    acc = {"fp32_vs_oracle_p6_rel_energy_err": err, "steps": n + 1,
           "sample": f"the cpu_baseline sample ({K} tets, p=6), same initial field, dt = {dt}"}
    acc["config_runs_vs_oracle"] = run_goldens(P, torch, Pair)
    if dense:
        w = synth.WORKLOADS["cube24_p8_dense"]
        d = synth.build_workload(w)
        verts8, tets8 = d["verts"], d["tets"]
        K8, N8 = tets8.shape[0], P.num_modes(8)
        m8 = P.Mesh(verts8, tets8).set_order(8)
        r8 = np.random.default_rng(8)
        Hr = torch.tensor(np.ascontiguousarray(r8.standard_normal((3, N8, K8))), dtype=torch.float32, device="cuda")
        centers = np.arange(0, K8, K8 // 8)
        keep, ptets, pos = patch(tets8, centers)
        p8 = Pair(verts8, ptets, 8)
        ref = p8.to_cov(p8.s.rhs_e(p8.to_phys(Hr[:, :, keep].double().cpu().numpy())))[:, :, pos]
        for name, prec in (("fp32_sparse", None), ("bf16_dense", P.DGM_BF16), ("fp16_dense", P.DGM_F16)):
            dE, _ = m8.apply_curl(None, Hr) if prec is None else m8.apply_curl_dense(None, Hr, prec=prec)
            torch.cuda.synchronize()
            acc[f"p8_apply_rel_err_vs_oracle_{name}"] = rel_err(dE[:, :, centers].double().cpu().numpy(), ref)
        acc["p8_sample"] = f"dE = rate(random H) on {len(centers)} elements of the 24^3 x 6 mesh, oracle on patch meshes"
    return base, acc


def run_goldens(P, torch, Pair):
    """Each FP32 workload's recipe over its full step count on the 4^3-cell cube that the
    oracle ran (tests/golden/run_<name>.npz, written by the oracle alone): final energy-norm
    error of the library against the oracle and the drift of the leapfrog invariant Q."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("make_run_goldens",
                                                  os.path.join(ROOT, "tests", "golden", "make_run_goldens.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    out = {}
    for name, label in (("cfg2", "16cube_p4_1000_steps_recipe"), ("cfg3", "32cube_p6_500_steps_recipe"),
                        ("cfg4", "24cube_p8_200_steps_recipe")):
        path = os.path.join(ROOT, "tests", "golden", f"run_{name}.npz")
        if not os.path.exists(path):
            continue
        with np.load(path, allow_pickle=False) as z:
            g = {k: z[k] for k in z.files}
        r, verts, tets, eps, mu, s, E, H = mg.setup(name)
        pr = Pair(verts, tets, r["p"], eps, mu)
        dt = float(g["dt"])
        m = P.Mesh(verts, tets).set_order(r["p"]).set_material(eps, mu)
        Eg = torch.tensor(np.ascontiguousarray(pr.to_cov(E)), dtype=torch.float32, device="cuda")
        Hg = torch.tensor(np.ascontiguousarray(pr.to_cov(H)), dtype=torch.float32, device="cuda")
        _, Q0 = m.energy(Eg, Hg, dt=dt)
        m.step(Eg, Hg, dt, int(g["steps"]))
        _, Q1 = m.energy(Eg, Hg, dt=dt)
        err = pr.s.rel_error(pr.to_phys(Eg.double().cpu().numpy()), pr.to_phys(Hg.double().cpu().numpy()),
                             g["E_end"], g["H_end"])
        out[label] = {"p": r["p"], "steps": int(g["steps"]), "tets": int(tets.shape[0]),
                      "fp32_rel_energy_err_vs_oracle": err, "Q_rel_drift": abs(Q1 - Q0) / Q0}
    return out


def stab_leg(w, d, E0, steps: int):
    """Stabilised central flux with face unknowns (alpha = p^2) on the benchmark mesh:
    time per step of dgm_step_stab (FP32), the drift of its invariant, and its algorithmic
    traffic: the central phases' 72 N + 80 bytes per element-step plus the face unknowns
    (each face's 2 NF values read and written in the H phase, read in the E phase; two faces
    per element) and the owner's 2x2 update matrix (16 B per face)."""
    import torch

    import paper_1104_4208_amd as P

    K, p = d["tets"].shape[0], w.p
    N, NF = P.num_modes(p), P.num_face_modes(p)
    m = P.Mesh(d["verts"], d["tets"]).set_order(p).set_material(d["eps"], d["mu"]).set_stab_alpha(1.0)
    dt, rho = m.estimate_dt_stab(cfl=0.5, iters=20, seed=w.seed)
    E = torch.tensor(np.ascontiguousarray(E0), dtype=torch.float32, device="cuda")
    H = torch.zeros_like(E)
    HF = m.face_zeros(torch.float32)
    _, Q0 = m.energy_stab(E, H, HF, dt=dt)
    m.step_stab(E, H, HF, dt, 5)

    def timed(nsteps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        m.step_stab(E, H, HF, dt, nsteps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    one = min(timed(1) for _ in range(3))
    t = timed(steps)
    _, Q1 = m.energy_stab(E, H, HF, dt=dt)
    step_s = (t - one) / (steps - 1)
    bytes_step = K * (72 * N + 80 + 2 * 3 * 2 * NF * 4 + 2 * 16)
    del E, H, HF, m
    torch.cuda.empty_cache()
    return {"workload": "pec_cube_cavity_kuhn32_p6_fp32_stabilised", "alpha": f"p^2 = {p * p}", "dt": dt,
            "rho": rho, "steps": steps, "ms_per_step": step_s * 1e3,
            "dof_updates_per_s": 6 * N * K / step_s,
            "algorithmic_bytes_per_element_step": 72 * N + 80 + 2 * 3 * 2 * NF * 4 + 2 * 16,
            "hbm_frac": bytes_step / step_s / (HBM_PEAK_GBS * 1e9),
            "Q_rel_drift": abs(Q1 - Q0) / Q0, "steps_total": steps + 8}


def mixed_leg(w, d, steps: int, pE: int = 7, pH: int = 6):
    """Mixed orders (Section 2: E of degree pE = pH + 1, H of degree pH) on the benchmark
    mesh, FP32: time per step, DOF-updates/s over 3 (N_E + N_H) K unknowns, and the HBM
    fraction of its algorithmic traffic 36 (N_E + N_H) + 80 bytes per element-step (each
    phase reads the differentiated field, reads and writes the updated one, 24 B of metric
    and 16 B of codes)."""
    import torch

    import paper_1104_4208_amd as P

    from paper_1104_4208_amd.project import project_covariant

    K = d["tets"].shape[0]
    NE, NH = P.num_modes(pE), P.num_modes(pH)
    m = P.Mesh(d["verts"], d["tets"]).set_orders(pE, pH).set_material(d["eps"], d["mu"])
    dt, rho = m.estimate_dt(cfl=0.5, iters=20, seed=w.seed)
    E = torch.tensor(np.ascontiguousarray(project_covariant(d["verts"], d["tets"], pE, d["field"].E)),
                     dtype=torch.float32, device="cuda")
    H = m.zeros(torch.float32)
    _, Q0 = m.energy(E, H, dt=dt)
    m.step(E, H, dt, 5)

    def timed(nsteps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        m.step(E, H, dt, nsteps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    one = min(timed(1) for _ in range(3))
    t = timed(steps)
    _, Q1 = m.energy(E, H, dt=dt)
    step_s = (t - one) / (steps - 1)
    bpe = 36 * (NE + NH) + 80
    del E, H, m
    torch.cuda.empty_cache()
    return {"workload": f"pec_cube_cavity_kuhn32_mixed_pE{pE}_pH{pH}_fp32", "pE": pE, "pH": pH, "dt": dt,
            "rho": rho, "steps": steps, "ms_per_step": step_s * 1e3,
            "dof_updates_per_s": 3 * (NE + NH) * K / step_s, "algorithmic_bytes_per_element_step": bpe,
            "hbm_frac": K * bpe / step_s / (HBM_PEAK_GBS * 1e9), "Q_rel_drift": abs(Q1 - Q0) / Q0,
            "steps_total": steps + 8}


def var_leg(w, d, E0, steps: int):
    """Material linear inside the elements (Section 3.3.2) on the benchmark mesh, FP32, p = 6:
    eps at the vertices = the element's eps in {1, 4} times 1 + 0.25 sin(3x) cos(2z), mu =
    1 + 0.2 y.  A step is, per field, the unit-material phase (rate into a work buffer), the
    approximate mass inverse added into the field (dgm_mass_p6, sum factorisation on the 7^3
    collapsed Gauss points) and the field's traces.  Reports time per step, the drift of the
    invariant in the M~ inner product (energies by CG solves), and the mass kernel's emitted
    flops per element (its duration is in the committed kernel-trace summary)."""
    import torch

    import paper_1104_4208_amd as P
    from paper_1104_4208_amd.gen import mass as MS

    K, p = d["tets"].shape[0], w.p
    N = P.num_modes(p)
    x = d["verts"][d["tets"]]
    eps_v = d["eps"][:, None] * (1.0 + 0.25 * np.sin(3.0 * x[..., 0]) * np.cos(2.0 * x[..., 2]))
    mu_v = 1.0 + 0.2 * x[..., 1]
    m = P.Mesh(d["verts"], d["tets"]).set_order(p).set_material_linear(eps_v, mu_v)
    dt, rho = m.estimate_dt(cfl=0.5, iters=20, seed=w.seed)
    E = torch.tensor(np.ascontiguousarray(E0), dtype=torch.float32, device="cuda")
    H = torch.zeros_like(E)
    _, Q0 = m.energy(E, H, dt=dt)
    m.step(E, H, dt, 5)

    def timed(nsteps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        m.step(E, H, dt, nsteps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    one = min(timed(1) for _ in range(3))
    t = timed(steps)
    _, Q1 = m.energy(E, H, dt=dt)
    step_s = (t - one) / (steps - 1)
    mc = MS.mass_cost(p)
    # the mass kernel alone (dgm_apply_mass_inverse on an H-shaped field), HIP events on the
    # stream it is launched on
    X = torch.randn_like(H)
    Y = torch.empty_like(H)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        m.apply_mass_inverse(X, "H", out=Y)
    reps = 20
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        m.apply_mass_inverse(X, "H", out=Y)
    e1.record(stream)
    torch.cuda.synchronize()
    mass_s = e0.elapsed_time(e1) / 1e3 / reps
    mass_bytes = K * (24 * N + 16)  # this call writes Y without reading it (in the step it adds: 36 N + 16)
    del X, Y
    del E, H, m
    torch.cuda.empty_cache()
    return {"workload": "pec_cube_cavity_kuhn32_p6_fp32_linear_material", "dt": dt, "rho": rho, "steps": steps,
            "ms_per_step": step_s * 1e3, "dof_updates_per_s": 6 * N * K / step_s,
            "mass_kernel": {"name": "dgm_mass_p6<float>", "call": "dgm_apply_mass_inverse (Y = P X)", "bound": "alu",
                            "us": mass_s * 1e6, "flops_per_element": mc["flops"],
                            "flops_per_launch": mc["flops"] * K, "algorithmic_bytes_per_element": 24 * N + 16,
                            "hbm_frac": mass_bytes / mass_s / (HBM_PEAK_GBS * 1e9),
                            "alu_frac": mc["flops"] * K / mass_s / (FP32_PEAK_TFLOPS * 1e12)},
            "Q_rel_drift": abs(Q1 - Q0) / Q0, "steps_total": steps + 8}


def dense_comparison(steps: int):
    """p = 8 workload (24^3 x 6 = 82,944 tets, random modal data, seed 4): the FP32
    sparse path against the dense matrix-core variant with BF16 and FP16 operands.
    Reports time per step, DOF-updates/s, the difference of one dense operator
    application from the FP32 one, and the energy-norm distance of each dense run
    from the FP32 run after `steps` steps (errors against the oracle are in the
    accuracy block of the oracle leg)."""
    import torch

    import paper_1104_4208_amd as P
    import synth

    w = synth.WORKLOADS["cube24_p8_dense"]
    d = synth.build_workload(w)
    rng = d["field"]
    verts, tets = d["verts"], d["tets"]
    K, p = tets.shape[0], w.p
    N = P.num_modes(p)
    m = P.Mesh(verts, tets).set_order(p)
    # random physical Cartesian modal coefficients, mapped to the covariant layout
    ts = np.sort(tets, axis=1)
    Pv = verts[ts]
    F = np.stack([Pv[:, 1] - Pv[:, 0], Pv[:, 2] - Pv[:, 0], Pv[:, 3] - Pv[:, 0]], axis=2)
    e_phys = rng.standard_normal((K, N, 3))
    E0 = np.ascontiguousarray(np.einsum("kji,kmj->imk", F, e_phys))
    E = torch.tensor(E0, dtype=torch.float32, device="cuda")
    H = torch.zeros_like(E)
    W0, _ = m.energy(E, H)
    E /= math.sqrt(W0)  # rescaled to W = 1
    dt, _ = m.estimate_dt(cfl=0.5, iters=20, seed=w.seed)
    out = {"workload": "pec_cube_kuhn24_p8_random_modes", "tets": K, "p": p, "dofs": 6 * N * K, "steps": steps, "dt": dt}
    Hrand = torch.tensor(np.ascontiguousarray(rng.standard_normal((3, N, K))), dtype=torch.float32, device="cuda")
    ref, _ = m.apply_curl(None, Hrand)
    scale = float(ref.abs().max())
    runs = {}
    for name, prec in (("fp32_sparse", None), ("bf16_dense", P.DGM_BF16), ("fp16_dense", P.DGM_F16)):
        Ei, Hi = E.clone(), H.clone()
        stepf = (lambda a, b, n: m.step(a, b, dt, n)) if prec is None else (lambda a, b, n, q=prec: m.step_dense(a, b, dt, n, prec=q))
        stepf(Ei, Hi, 2)
        torch.cuda.synchronize()
        Ei, Hi = E.clone(), H.clone()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        stepf(Ei, Hi, steps)
        e1.record()
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) / 1e3
        runs[name] = (Ei, Hi)
        out[name] = {"ms_per_step": sec / steps * 1e3, "dof_updates_per_s": 6 * N * K * steps / sec}
        if prec is not None:
            dE, _ = m.apply_curl_dense(None, Hrand, prec=prec)
            out[name]["apply_rel_diff_from_fp32"] = float((dE - ref).abs().max()) / scale
    Es, Hs = runs["fp32_sparse"]
    Ws, _ = m.energy(Es, Hs)
    for name in ("bf16_dense", "fp16_dense"):
        Ed, Hd = runs[name]
        Wd, _ = m.energy(Ed - Es, Hd - Hs)
        out[name]["energy_norm_dist_from_fp32_after_run"] = math.sqrt(Wd / Ws)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch

    import paper_1104_4208_amd as P

    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible")
    if a.copy_mib > 0:
        n = a.copy_mib * 2 ** 20 // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w, d, E0 = build_inputs()
    K, p = d["tets"].shape[0], w.p
    N = P.num_modes(p)
    m = P.Mesh(d["verts"], d["tets"]).set_order(p).set_material(d["eps"], d["mu"])
    dt, rho = m.estimate_dt(cfl=0.5, iters=20, seed=w.seed)
    E = torch.tensor(np.ascontiguousarray(E0), dtype=torch.float32, device="cuda").contiguous()
    H = torch.zeros_like(E)
    torch.cuda.synchronize()
    progress("main leg: inputs ready, warm-up")
    W0, Q0 = m.energy(E, H, dt=dt)
    m.step(E, H, dt, a.warmup)
    stream = torch.cuda.current_stream()

    def timed(nsteps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        m.step(E, H, dt, nsteps)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / 1e3

    one = min(timed(1) for _ in range(3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev = timed(a.steps)
    wall = time.perf_counter() - t0
    W1, Q1 = m.energy(E, H, dt=dt)
    steps_done = a.warmup + 3 + a.steps
    phase_s = (ev - one) / (2 * (a.steps - 1)) if a.steps > 1 else ev / 2
    bytes_launch = K * (36 * N + 40)
    achieved = bytes_launch / phase_s / 1e9
    value = 6 * N * K * a.steps / wall
    ctr = measured_counters()
    traffic = ctr.get("bytes_per_launch") if ctr else None
    oc = opcount(p)
    flops_launch = K * oc["with_traces"]
    alu = {"flops_per_element_phase": oc["with_traces"], "flops_per_launch": flops_launch,
           "flops_per_dof_update": 2 * oc["with_traces"] / (6 * N),
           "achieved": flops_launch / phase_s / 1e12, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": flops_launch / phase_s / 1e12 / FP32_PEAK_TFLOPS,
           "peak_note": "FP32 vector FMA without packed FP32 (switched off by a compiler flag): "
                        "256 CUs x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz",
           "count_note": "emitted multiplies and adds (FMA = 2) per element, including the x=0/y=0 trace "
                         f"jobs ({oc['trace_stage_recomputed_faces']} flops) that run only in tiles with an "
                         "off-tile neighbour across those faces"}
    if ctr and ctr.get("valu_insts_per_launch"):
        alu["valu_insts_per_launch"] = ctr["valu_insts_per_launch"]
        alu["valu_issue_frac"] = ctr["valu_insts_per_launch"] / VALU_ISSUE_PER_S / phase_s
    out = {
        "metric": "DOF-updates/sec & %HBM roofline at p=6 (FP32 vs FP64 oracle err); serving p50/p99",
        "value": value,
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(WORKLOAD, dt=dt, rho=rho),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "dgm_phase_p6<float, true, false, false>", "phase_us": phase_s * 1e6,
                     "bytes_per_launch": bytes_launch, "alu": alu},
        "energy": {"W0": W0, "Q0": Q0, "Q_end": Q1, "Q_rel_drift": abs(Q1 - Q0) / Q0, "steps_total": steps_done},
    }
    # the config's full 500 steps at full size: drift of the leapfrog invariant (FP32 state,
    # FP64 reduction) over the whole run, after the timed region
    progress(f"main leg: {a.steps} timed steps done ({phase_s * 1e6:.1f} us per phase)")
    rest = max(0, w.steps - steps_done)
    if rest:
        m.step(E, H, dt, rest)
    W2, Q2 = m.energy(E, H, dt=dt)
    out["energy"]["Q_rel_drift_full_run"] = abs(Q2 - Q0) / Q0
    out["energy"]["steps_full_run"] = steps_done + rest
    del E, H
    torch.cuda.empty_cache()
    if not a.no_stab:
        progress("stabilized_flux leg")
        out["stabilized_flux"] = stab_leg(w, d, E0, a.stab_steps)
    if not a.no_mixed:
        progress("mixed_orders leg")
        out["mixed_orders"] = mixed_leg(w, d, a.stab_steps)
    if not a.no_var:
        progress("linear_material leg")
        out["linear_material"] = var_leg(w, d, E0, a.stab_steps)
    if not a.no_dense:
        progress("dense_variant leg")
        out["dense_variant"] = dense_comparison(a.dense_steps)
    if not a.no_serve:
        from paper_1104_4208_amd import serve

        progress("serving leg")
        rep = serve.serve_report(num=a.serve_requests, budget_gib=2.0, chunk=20, n_range=(4, a.serve_nmax),
                                  progress=True)
        rep["note"] = ("serving trace: Poisson arrivals at 50/s, n in 4..serve_nmax, p in 2..8, eps in {1,2,4}, "
                       "steps in 200..2000, jitter 0.1 h, 2 GiB admission budget, 20 steps per batched launch; "
                       "sequential = the same trace solved one request at a time with dgm_step")
        out["serving"] = rep
    if not a.no_cpu_baseline:
        progress("cpu baseline and accuracy leg")
        out["cpu_baseline"], out["accuracy"] = oracle_leg(a.cpu_seconds, dense=not a.no_dense)
    progress("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
