"""Continuous-batching serving loop for many cavity solves on one GPU.

Interface: Scheduler(hbm_budget_bytes, steps_per_launch).submit(mesh, p, eps, mu,
E0, H0, dt, nsteps) -> Ticket; Ticket.result() -> (E, H, (W, Q), latency).

Requests (a jittered cube mesh, order p, permittivity eps, step count) arrive
over time.  The server admits them into batch slots whenever the HBM budget
allows, advances every active slot together with one HIP-graph launch per
chunk of leapfrog steps (dgm_batch_advance), retires finished slots and admits
waiting requests as memory frees up.  The baseline solves the same arrival
trace one request at a time with plain dgm_step calls (FIFO).  Both report
per-request latency (completion - arrival), p50 / p99, and aggregate
DOF-updates/s over the makespan.

    python -m paper_1104_4208_amd.serve [--requests 256] [--budget-gib 2] [--chunk 20]

Request payloads (mesh, covariant initial field, dt) are prepared before the
clock starts, as a client would send them.  Each request's initial field is the
TE101 mode of the unit-cube cavity with its eps, so its final state also has a
closed-form check.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import threading
import time
from dataclasses import dataclass, field

import numpy as np

from . import dgmax as D
from .project import project_covariant


def device_bytes(K: int, p: int) -> int:
    """Device memory of one FP32 solve: the state (E, H), the two trace buffers and
    the per-element geometry the library keeps for the mesh handle."""
    nf = D.num_face_modes(p)
    trace = ((K + 63) // 64) * 64 * 4 * 2 * ((nf + 3) // 4 * 4)
    return 2 * 3 * D.num_modes(p) * K * 4 + 2 * trace * 4 + K * 400


@dataclass
class Request:
    rid: int
    arrival: float
    n: int
    p: int
    eps: float
    steps: int
    verts: np.ndarray = field(repr=False)
    tets: np.ndarray = field(repr=False)
    E0: np.ndarray = field(repr=False)
    H0: np.ndarray = field(repr=False)
    dt: float = 0.0

    @property
    def K(self):
        return self.tets.shape[0]

    @property
    def dofs(self):
        return 6 * D.num_modes(self.p) * self.K

    @property
    def work(self):
        return self.dofs * self.steps

    def device_bytes(self):
        return device_bytes(self.K, self.p)


def make_trace(num=256, rate=50.0, seed=5, n_range=(4, 24), p_range=(2, 8), eps_choices=(1.0, 2.0, 4.0),
               steps_range=(200, 2000), jitter=0.1, dt_cfl=0.5, progress=False):
    """Poisson arrivals (mean rate per second) of cavity solves, drawn in the fixed
    order: per request n, p, eps, steps, then the mesh jitter; arrival gaps last."""
    import synth

    rng = np.random.default_rng(seed)
    specs = []
    for r in range(num):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        eps = float(rng.choice(np.asarray(eps_choices)))
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        verts, tets = synth.kuhn_mesh(n, jitter, rng)
        specs.append((n, p, eps, steps, verts, tets))
    gaps = rng.exponential(1.0 / rate, size=num)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs = []
    for r, ((n, p, eps, steps, verts, tets), t) in enumerate(zip(specs, arrivals)):
        if progress and r % 16 == 0:
            print(f"[serve] preparing request {r}/{num}", file=sys.stderr, flush=True)
        mode = synth.te101(eps=eps)
        E0 = project_covariant(verts, tets, p, mode.E).astype(np.float32)
        # dt from the stability bound of this mesh (power iteration, 20 steps)
        m = D.Mesh(verts, tets).set_order(p).set_material(np.full(tets.shape[0], eps), None)
        dt, _ = m.estimate_dt(cfl=dt_cfl, iters=20, seed=r + 1)
        m.close()
        H0 = project_covariant(verts, tets, p, lambda x: mode.H(x, -dt / 2)).astype(np.float32)
        reqs.append(Request(r, float(t), n, p, eps, steps, verts, tets, E0, H0, dt))
    return reqs


def _percentile(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else float("nan")


class Server:
    def __init__(self, hbm_budget_bytes: int, chunk: int = 20):
        self.budget = int(hbm_budget_bytes)
        self.chunk = int(chunk)

    def _admit(self, req):
        import torch

        m = D.Mesh(req.verts, req.tets).set_order(req.p).set_material(np.full(req.K, req.eps), None)
        E = torch.tensor(req.E0, device="cuda")
        H = torch.tensor(req.H0, device="cuda")
        return m, E, H

    def run(self, trace, mode: str = "batched", keep_states=None):
        """Serve the trace in real time.  mode 'batched' or 'sequential'.
        keep_states: optional set of request ids whose final (E, H) are returned."""
        import torch

        reqs = sorted(trace, key=lambda r: r.arrival)
        queue = []
        nxt = 0
        used = 0
        live = {}
        done = {}
        states = {}
        batch = D.Batch(self.chunk) if mode == "batched" else None
        sid_of = {}
        if mode == "batched":
            # Requests are set up (mesh, material, field uploads) on a worker thread while
            # the GPU runs a chunk on the batch's own stream; the library calls release the
            # interpreter lock.  A launch that re-captures the batch's graph holds `gate`,
            # which every set-up holds too, so no other HIP call lands inside a capture.
            bs = torch.cuda.Stream()
            prep = cf.ThreadPoolExecutor(max_workers=1)
            gate = threading.Lock()

            def setup(r):
                with gate:
                    out = self._admit(r)
                    torch.cuda.current_stream().synchronize()  # uploads done before the batch stream reads them
                    return out

        pending = []  # (request, future of its set-up), in admission order
        t0 = time.perf_counter()
        while len(done) < len(reqs):
            now = time.perf_counter() - t0
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                queue.append(reqs[nxt])
                nxt += 1
            if mode == "batched":
                # reserve memory for what fits (one request always when nothing else holds any)
                while queue and (used + queue[0].device_bytes() <= self.budget or not (live or pending)):
                    r = queue.pop(0)
                    used += r.device_bytes()
                    pending.append((r, prep.submit(setup, r)))
                # add what is set up; wait for the oldest when the GPU would idle otherwise
                while pending and (pending[0][1].done() or not live):
                    r, fut = pending.pop(0)
                    m, E, H = fut.result()
                    with torch.cuda.stream(bs):
                        sid = batch.add(m, E, H, r.dt, r.steps)
                    sid_of[sid] = r.rid
                    live[r.rid] = (r, m, E, H)
                if live:
                    with torch.cuda.stream(bs):
                        if batch.needs_capture():
                            with gate:
                                batch.launch()
                        else:
                            batch.launch()
                    batch.wait()
                    for sid in batch.take_finished():
                        rid = sid_of.pop(sid)
                        r, m, E, H = live.pop(rid)
                        done[rid] = time.perf_counter() - t0
                        used -= r.device_bytes()
                        if keep_states is not None and rid in keep_states:
                            # on the default stream, the one the set-up thread allocates on
                            states[rid] = (E.clone(), H.clone())
                        m.close()
                        del E, H
            else:
                if queue:
                    r = queue.pop(0)
                    m, E, H = self._admit(r)
                    m.step(E, H, r.dt, r.steps)
                    torch.cuda.synchronize()
                    done[r.rid] = time.perf_counter() - t0
                    if keep_states is not None and r.rid in keep_states:
                        states[r.rid] = (E.clone(), H.clone())
                    m.close()
                    del E, H
            if not live and not queue and not pending and nxt < len(reqs) and len(done) < len(reqs):
                wait = reqs[nxt].arrival - (time.perf_counter() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.05))
        if batch is not None:
            batch.close()
            prep.shutdown()
        makespan = max(done.values()) - min(r.arrival for r in reqs)
        lat = [done[r.rid] - r.arrival for r in reqs]
        work = sum(r.work for r in reqs)
        return {"mode": mode, "requests": len(reqs), "makespan_s": makespan, "dof_updates": work,
                "dof_updates_per_s": work / makespan, "p50_latency_s": _percentile(lat, 50),
                "p99_latency_s": _percentile(lat, 99), "mean_latency_s": float(np.mean(lat))}, states


class Ticket:
    """Handle of one submitted solve.  result() drives the server until this solve
    has finished and returns (E, H, (W, Q), latency_s): the final covariant fields
    (device tensors, FP32), the FP64 energy W and leapfrog invariant Q at the end,
    and the time from submission to completion."""

    def __init__(self, server, tid):
        self.server, self.tid = server, tid

    def done(self) -> bool:
        return self.tid in self.server._results

    def result(self):
        while not self.done():
            self.server.poll()
        return self.server._results[self.tid]


class Scheduler:
    """Submission interface of the batched server: solves are queued by submit(),
    admitted into batch slots while the HBM budget allows (the oldest first; one
    solve is always admitted when none is running), and advanced together by
    poll(), chunk steps per call.  As in Server.run, an admitted solve is set up
    (mesh, material, field copies) on a worker thread while the batch's chunks run
    on its own stream, and a launch that re-captures the graph holds the lock every
    set-up holds."""

    def __init__(self, hbm_budget_bytes: int, steps_per_launch: int = 20):
        self.budget = int(hbm_budget_bytes)
        self.batch = D.Batch(int(steps_per_launch))
        self._queue = []
        self._pending = []  # (tid, t0, dt, nsteps, need, future of the set-up)
        self._live = {}
        self._results = {}
        self._used = 0
        self._next = 0
        self._stream = None
        self._prep = cf.ThreadPoolExecutor(max_workers=1)
        self._gate = threading.Lock()

    def submit(self, verts, tets, p, eps, mu, E0, H0, dt, nsteps) -> Ticket:
        """verts/tets: host mesh arrays; eps, mu: per-element arrays or scalars (None
        means 1); E0, H0: covariant (3, N, K) FP32 initial fields (host arrays or
        device tensors, copied); dt and nsteps of the leapfrog run."""
        tid = self._next
        self._next += 1
        self._queue.append((tid, time.perf_counter(), verts, tets, p, eps, mu, E0, H0, dt, nsteps))
        self._reserve()
        return Ticket(self, tid)

    def _setup(self, verts, tets, p, eps, mu, E0, H0):
        import torch

        with self._gate:
            K = np.asarray(tets).shape[0]
            full = lambda v: None if v is None else np.broadcast_to(np.asarray(v, dtype=np.float64), (K,)).copy()
            m = D.Mesh(verts, tets).set_order(p).set_material(full(eps), full(mu))
            E = torch.as_tensor(E0, dtype=torch.float32, device="cuda").clone().contiguous()
            H = torch.as_tensor(H0, dtype=torch.float32, device="cuda").clone().contiguous()
            torch.cuda.current_stream().synchronize()  # copies done before the batch stream reads them
            return m, E, H

    def _reserve(self):
        """Start the set-up of queued solves that fit the budget, oldest first."""
        while self._queue:
            tid, t0, verts, tets, p, eps, mu, E0, H0, dt, nsteps = self._queue[0]
            need = device_bytes(np.asarray(tets).shape[0], p)
            if (self._live or self._pending) and self._used + need > self.budget:
                break
            self._queue.pop(0)
            self._used += need
            fut = self._prep.submit(self._setup, verts, tets, p, eps, mu, E0, H0)
            self._pending.append((tid, t0, dt, nsteps, need, fut))

    def poll(self):
        """Admit what is set up, advance every active solve by one chunk, collect results."""
        import torch

        if self._stream is None:
            self._stream = torch.cuda.Stream()
        self._reserve()
        while self._pending and (self._pending[0][5].done() or not self._live):
            tid, t0, dt, nsteps, need, fut = self._pending.pop(0)
            m, E, H = fut.result()
            with torch.cuda.stream(self._stream):
                sid = self.batch.add(m, E, H, dt, nsteps)
            self._live[sid] = (tid, t0, m, E, H, dt, need)
        if self._live:
            with torch.cuda.stream(self._stream):
                if self.batch.needs_capture():
                    with self._gate:
                        self.batch.launch()
                else:
                    self.batch.launch()
            self.batch.wait()
        for sid in self.batch.take_finished():
            tid, t0, m, E, H, dt, need = self._live.pop(sid)
            energies = m.energy(E, H, dt=dt)
            self._results[tid] = (E, H, energies, time.perf_counter() - t0)
            self._used -= need
            m.close()
        self._reserve()

    def drain(self):
        while self._queue or self._pending or self._live:
            self.poll()

    def close(self):
        self.batch.close()
        self._prep.shutdown()


def closed_form_error(req, E, H):
    """Relative energy-norm distance of the final state from the projected exact
    TE101 standing wave at t = steps dt (E) and t - dt/2 (H), in FP64 on the host."""
    import synth

    mode = synth.te101(eps=req.eps)
    T = req.steps * req.dt
    Ee = project_covariant(req.verts, req.tets, req.p, lambda x: mode.E(x, T))
    He = project_covariant(req.verts, req.tets, req.p, lambda x: mode.H(x, T - req.dt / 2))
    m = D.Mesh(req.verts, req.tets).set_order(req.p).set_material(np.full(req.K, req.eps), None)
    import torch

    dE = (E.double() - torch.tensor(Ee, device="cuda"))
    dH = (H.double() - torch.tensor(He, device="cuda"))
    num, _ = m.energy(dE.contiguous(), dH.contiguous())
    den, _ = m.energy(torch.tensor(Ee, device="cuda"), torch.tensor(He, device="cuda"))
    m.close()
    return math.sqrt(num / den)


def serve_report(num=256, budget_gib=2.0, chunk=20, n_range=(4, 24), steps_range=(200, 2000), check=8,
                 progress=False):
    """Batched and sequential runs of the same trace, plus the alone-vs-mix check on
    `check` requests and their closed-form errors."""
    trace = make_trace(num=num, n_range=n_range, steps_range=steps_range, progress=progress)
    srv = Server(int(budget_gib * 2 ** 30), chunk)
    ids = set(range(min(check, num)))
    if progress:
        print("[serve] batched run", file=sys.stderr, flush=True)
    rb, sb = srv.run(trace, "batched", keep_states=ids)
    if progress:
        print("[serve] sequential run", file=sys.stderr, flush=True)
    rs, ss = srv.run(trace, "sequential", keep_states=ids)
    diffs, errs = [], []
    for rid in sorted(ids):
        Eb, Hb = sb[rid]
        Es, Hs = ss[rid]
        d = max(float((Eb - Es).abs().max()), float((Hb - Hs).abs().max()))
        scale = max(float(Es.abs().max()), float(Hs.abs().max()))
        diffs.append(d / scale)
        errs.append(closed_form_error(trace[rid], Es, Hs))
    return {"trace": {"requests": num, "rate_per_s": 50.0, "n_range": list(n_range), "p_range": [2, 8],
                      "eps": [1, 2, 4], "steps_range": list(steps_range), "budget_gib": budget_gib, "chunk": chunk},
            "batched": rb, "sequential": rs,
            "speedup_dof_updates": rb["dof_updates_per_s"] / rs["dof_updates_per_s"],
            "alone_vs_mix_max_rel_diff": max(diffs) if diffs else None,
            "closed_form_rel_err_max": max(errs) if errs else None}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--budget-gib", type=float, default=2.0)
    ap.add_argument("--chunk", type=int, default=20)
    ap.add_argument("--nmax", type=int, default=24)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rep = serve_report(a.requests, a.budget_gib, a.chunk, n_range=(4, a.nmax), progress=True)
    line = json.dumps(rep)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    main()
