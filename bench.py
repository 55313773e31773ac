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
conversions at the ends cancel).  cpu_baseline: the FP64 oracle timed on a
bounded sample of the same workload (smaller cube, same order and recipe); the
same leg (the only code here that runs the oracle) reports the FP32 error against
the oracle on that sample, and at p = 8 for the sparse and dense paths, under
"accuracy".
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
WORKLOAD = dict(workload="pec_cube_cavity_kuhn32_p6_fp32", cells=32, tets=196608, p=6, modes=84,
                dofs=99090432, jitter=0.1, eps=[1, 4], steps_in_config=500, init="three cavity modes, seed 3")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "phase_p6_cube32_traffic.json")


def measured_traffic():
    """HBM bytes per launch from the committed counter summary, or None when the
    generated p = 6 kernel source differs from the one the counters were taken on."""
    import hashlib

    src = os.path.join(ROOT, "paper_1104_4208_amd", "csrc", "generated", "phase_p6.inc")
    if not (os.path.exists(TRAFFIC_FILE) and os.path.exists(src)):
        return None
    with open(TRAFFIC_FILE) as fh:
        tr = json.load(fh)
    with open(src, "rb") as fh:
        h = hashlib.sha256(fh.read()).hexdigest()[:16]
    return tr.get("bytes_per_launch") if tr.get("kernel_source_sha256_16") == h else None


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
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-nmax", type=int, default=10)
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
    traffic = measured_traffic()
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
                     "kernel": "dgm_phase_p6<float, true>", "phase_us": phase_s * 1e6, "bytes_per_launch": bytes_launch},
        "energy": {"W0": W0, "Q0": Q0, "Q_end": Q1, "Q_rel_drift": abs(Q1 - Q0) / Q0, "steps_total": steps_done},
    }
    del E, H
    torch.cuda.empty_cache()
    if not a.no_dense:
        out["dense_variant"] = dense_comparison(a.dense_steps)
    if not a.no_serve:
        from paper_1104_4208_amd import serve

        rep = serve.serve_report(num=a.serve_requests, budget_gib=2.0, chunk=20, n_range=(4, a.serve_nmax))
        rep["note"] = ("reduced trace of the serving workload (same recipe: Poisson arrivals at 50/s, p in 2..8, "
                       "eps in {1,2,4}, steps in 200..2000, jitter 0.1 h) with n <= serve_nmax so the default run stays "
                       "short; `python -m paper_1104_4208_amd.serve` runs the full 256-request trace")
        out["serving"] = rep
    if not a.no_cpu_baseline:
        out["cpu_baseline"], out["accuracy"] = oracle_leg(a.cpu_seconds, dense=not a.no_dense)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
