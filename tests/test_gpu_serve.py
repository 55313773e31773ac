"""Batched serving: slots of different orders, sizes and step counts advanced
together give bitwise the same result as each solve alone; a small arrival
trace completes in both serving modes."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1104_4208_amd as P  # noqa: E402
from paper_1104_4208_amd import serve  # noqa: E402


def _case(n, p, seed):
    rng = np.random.default_rng(seed)
    verts, tets = synth.kuhn_mesh(n, 0.1, rng)
    K, N = tets.shape[0], P.num_modes(p)
    E = rng.standard_normal((3, N, K)).astype(np.float32)
    H = rng.standard_normal((3, N, K)).astype(np.float32)
    eps = rng.choice([1.0, 2.0, 4.0], size=K)
    return verts, tets, eps, E, H


def test_batch_matches_alone_bitwise():
    cases = [(2, 2, 1, 23), (3, 4, 2, 41), (2, 6, 3, 7), (4, 3, 4, 60), (1, 8, 5, 33), (3, 2, 6, 20)]
    dt = 2e-3
    alone, mixed = {}, {}
    for (n, p, seed, steps) in cases:
        verts, tets, eps, E, H = _case(n, p, seed)
        m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
        Eg, Hg = torch.tensor(E, device="cuda"), torch.tensor(H, device="cuda")
        m.step(Eg, Hg, dt, steps)
        torch.cuda.synchronize()
        alone[seed] = (Eg.cpu().numpy(), Hg.cpu().numpy())
    b = P.Batch(chunk=16)
    live = {}
    for (n, p, seed, steps) in cases:
        verts, tets, eps, E, H = _case(n, p, seed)
        m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
        Eg, Hg = torch.tensor(E, device="cuda"), torch.tensor(H, device="cuda")
        sid = b.add(m, Eg, Hg, dt, steps)
        live[sid] = (seed, m, Eg, Hg)
    rounds = 0
    while b.num_active():
        b.advance()
        rounds += 1
        for sid in b.take_finished():
            seed, m, Eg, Hg = live.pop(sid)
            mixed[seed] = (Eg.cpu().numpy(), Hg.cpu().numpy())
    assert not live and rounds == 4  # the longest solve takes ceil(60 / 16) launches
    for seed in alone:
        assert np.array_equal(alone[seed][0], mixed[seed][0]), seed
        assert np.array_equal(alone[seed][1], mixed[seed][1]), seed


def test_streaming_kernels_match_plain_bitwise():
    """Meshes whose fields and traces exceed the last-level cache run the phase kernels
    with nontemporal field accesses; that changes no arithmetic.  A (20^3 x 6, p = 6,
    174 MiB per step) alone runs the plain kernel, B (24^3 x 6, 301 MiB) alone the
    streaming one, and both together in a batch (475 MiB) the streaming batched kernel:
    every result agrees bitwise."""
    cases = [(20, 6, 11, 6), (24, 6, 12, 5)]
    dt = 2e-4  # below the stable step of both meshes
    alone, mixed = {}, {}
    for (n, p, seed, steps) in cases:
        verts, tets, eps, E, H = _case(n, p, seed)
        m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
        Eg, Hg = torch.tensor(E, device="cuda"), torch.tensor(H, device="cuda")
        m.step(Eg, Hg, dt, steps)
        torch.cuda.synchronize()
        alone[seed] = (Eg.cpu().numpy(), Hg.cpu().numpy())
        del m, Eg, Hg
    b = P.Batch(chunk=4)
    live = {}
    for (n, p, seed, steps) in cases:
        verts, tets, eps, E, H = _case(n, p, seed)
        m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
        Eg, Hg = torch.tensor(E, device="cuda"), torch.tensor(H, device="cuda")
        live[b.add(m, Eg, Hg, dt, steps)] = (seed, m, Eg, Hg)
    while b.num_active():
        b.advance()
        for sid in b.take_finished():
            seed, m, Eg, Hg = live.pop(sid)
            mixed[seed] = (Eg.cpu().numpy(), Hg.cpu().numpy())
    assert not live
    for seed in alone:
        assert np.all(np.isfinite(alone[seed][0]))
        assert np.array_equal(alone[seed][0], mixed[seed][0]), seed
        assert np.array_equal(alone[seed][1], mixed[seed][1]), seed


def test_launch_wait_matches_advance():
    """dgm_batch_launch + dgm_batch_wait is dgm_batch_advance in two halves: same results
    bitwise; a second launch or taking results before the wait is refused; a re-capture
    is reported only when the set of orders changes."""
    cases = [(2, 3, 31, 9), (3, 5, 32, 5)]
    dt = 1e-3
    runs = []
    for split in (False, True):
        b = P.Batch(chunk=4)
        out, live, caps = {}, {}, []
        for (n, p, seed, steps) in cases:
            verts, tets, eps, E, H = _case(n, p, seed)
            m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
            Eg, Hg = torch.tensor(E, device="cuda"), torch.tensor(H, device="cuda")
            live[b.add(m, Eg, Hg, dt, steps)] = (seed, m, Eg, Hg)
        while b.num_active():
            if split:
                caps.append(b.needs_capture())
                b.launch()
                with pytest.raises(P.DGMError):
                    b.launch()
                with pytest.raises(P.DGMError):
                    b.take_finished()
                b.wait()
            else:
                b.advance()
            for sid in b.take_finished():
                seed, m, Eg, Hg = live.pop(sid)
                out[seed] = (Eg.cpu().numpy(), Hg.cpu().numpy())
        b.close()
        runs.append(out)
        if split:
            # chunks of 4: both orders for two launches, then order 3 alone for one
            assert caps == [True, False, True], caps
    for seed in runs[0]:
        assert np.array_equal(runs[0][seed][0], runs[1][seed][0])
        assert np.array_equal(runs[0][seed][1], runs[1][seed][1])


def test_small_trace_both_modes():
    trace = serve.make_trace(num=10, rate=200.0, n_range=(2, 4), p_range=(2, 5), steps_range=(20, 80))
    srv = serve.Server(hbm_budget_bytes=4 * 2 ** 20, chunk=8)  # small budget: admission defers
    ids = set(range(10))
    rb, sb = srv.run(trace, "batched", keep_states=ids)
    rs, ss = srv.run(trace, "sequential", keep_states=ids)
    assert rb["requests"] == rs["requests"] == 10
    for rid in ids:
        assert torch.equal(sb[rid][0], ss[rid][0]) and torch.equal(sb[rid][1], ss[rid][1])
    print(rb, rs)
    assert rb["p99_latency_s"] >= rb["p50_latency_s"] > 0


def test_submit_tickets_match_alone():
    """The submission interface: tickets of mixed orders under a budget that defers
    admission return the same fields as each solve run alone, plus its energies."""
    cases = [(2, 3, 11, 30), (3, 5, 12, 17), (2, 8, 13, 9)]
    dt = 1e-3
    sch = serve.Scheduler(hbm_budget_bytes=2 * 2 ** 20, steps_per_launch=8)
    tickets, alone = [], []
    for (n, p, seed, steps) in cases:
        verts, tets, eps, E, H = _case(n, p, seed)
        tickets.append(sch.submit(verts, tets, p, eps, None, E, H, dt, steps))
        m = P.Mesh(verts, tets).set_order(p).set_material(eps, None)
        Eg, Hg = torch.tensor(E, device="cuda"), torch.tensor(H, device="cuda")
        m.step(Eg, Hg, dt, steps)
        alone.append((Eg, Hg, m.energy(Eg, Hg, dt=dt)))
    E2, H2, en2, lat2 = tickets[2].result()
    sch.drain()
    for t, (Ea, Ha, ena) in zip(tickets, alone):
        E, H, en, lat = t.result()
        assert torch.equal(E, Ea) and torch.equal(H, Ha)
        assert en == ena and lat > 0
    sch.close()
