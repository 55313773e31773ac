"""Emit the per-order HIP kernels (phase, batched phase, traces) as straight-line code.

Section 3.2.2 describes the reference implementation as C++ template
meta-programming that generates optimised code for every order up to an
a-priori maximum.  This module plays that role for CDNA4: for each order p
it writes kernel bodies in which every sparse operator entry of gen/tables.py
is an FMA with a literal coefficient.  One element per lane, 64 elements per
workgroup tile; the waves of a workgroup split the operator rows between them
(plan), and the tile's field and trace jumps are shared through LDS.

Phase contract (one leapfrog half step):
  U  (3,N,K)  stored-frame coefficients of the field that is differentiated
  V  (3,N,K)  stored-frame coefficients of the field that is updated, in place
  MU, MV (6,K)  symmetric conversions w = M S into the derivative frame
  nbr(4,K)    neighbour code nb*4 + local face of nb, or -1 on a wall
  Tin         tangential traces of U (trace buffer, layout in trace_strides)
  Tout        traces of the updated V for the next phase, or nullptr
  sdt         -dt for the H update, +dt for the E update
  wall        ghost factor on walls: the jump is (wall-1) * own trace
              (E_nb = -E gives wall = -1; H_nb = H gives wall = +1)
  V_k += sdt * ( c_k + sum_f T_f^T ( Lp_f[k,0] dtau_f0 + Lp_f[k,1] dtau_f1 ) )
where c is the curl in the derivative frame and dtau_fk = tau_fk(neighbour) -
tau_fk(own) are the jumps of the two tangential traces (u . t1, u . t2) of
face f, which both sides compute in the same (s,t) parametrisation because
vertices are sorted by global id.
"""
from __future__ import annotations

import os

import numpy as np

from . import mass as MS
from . import tables as TB


# Floating-point operations written into the kernel being emitted (multiplies and adds;
# an FMA counts two), per element: every wave's jobs together cover each element once.
FLOPS = [0]
OPCOUNT = {}


def _count(n):
    FLOPS[0] += n


def _lit(v: float) -> str:
    """Exact literal of an FP64 table entry, rounded once to the kernel's type R."""
    if v == 1.0:
        return "R(1)"
    if v == -1.0:
        return "R(-1)"
    return f"R({float(v).hex()})"


def _fma(acc, coef, x):
    if coef == 1.0:
        _count(1)
        return f"{acc} += {x};"
    if coef == -1.0:
        _count(1)
        return f"{acc} -= {x};"
    _count(2)
    return f"{acc} += {_lit(coef)} * {x};"


LANES = 64               # elements per workgroup tile (one per lane)
LDS_BUDGET = 160 * 1024  # bytes of LDS per compute unit
F64_MAX_ORDER = 6        # highest order also instantiated in FP64 (its staged field must fit in LDS)
TRACE_ROWS = 32          # face modes per trace job (bounds the job's accumulators)
LDS_GROUP = 8            # mode blocks per basic block in a stream
GROUP_LOADS = 32         # LDS loads per basic block in a stream (blocks of the factored traces are large)


class _Stream:
    """Emit a stream of mode blocks whose operands come from LDS.

    LDS_GROUP blocks share one basic block, behind an opaque uniform branch (an
    offset that is zero but hidden from the compiler by an empty asm statement):
    the loads of a group are issued first and the compiler schedules inside the
    group, while register pressure stays bounded by the group size; no value
    crosses a group boundary except the accumulators.
    """

    def __init__(self, a_, ind, tag):
        self.a_, self.ind, self.tag = a_, ind, tag

    def emit(self, blocks):
        """blocks: list of (loads, body) with loads = [LDS load expressions] and
        body(names) -> list of statements using the loaded values."""
        a_, ind = self.a_, self.ind
        if not blocks:
            return
        a_(ind + "size_t o = 0;")
        groups, cur = [], []
        for b in blocks:
            if cur and (len(cur) == LDS_GROUP or sum(len(x[0]) for x in cur) + len(b[0]) > GROUP_LOADS):
                groups.append(cur)
                cur = []
            cur.append(b)
        groups.append(cur)
        for grp in groups:
            a_(ind + "asm volatile(\"\" : \"+s\"(o));")
            a_(ind + "if (o == 0) {")
            names = []
            for gi, (ld, body) in enumerate(grp):
                nm = [f"x{gi}_{q}" for q in range(len(ld))]
                names.append(nm)
                a_(ind + "  const R " + ", ".join(f"{n} = {e}" for n, e in zip(nm, ld)) + ";")
            for gi, (ld, body) in enumerate(grp):
                a_(ind + "  {")
                for st in body(names[gi]):
                    a_(ind + "    " + st)
                a_(ind + "  }")
            a_(ind + "}")


OUT_ROWS = 32     # volume modes per output job (3 components each)
CYC = {0: (1, 2), 1: (2, 0), 2: (0, 1)}



FACTORED = (0, 3)  # faces whose trace goes through the collapsed tensor-product factors
# Faces whose own traces a phase recomputes from the staged field (cheap: the x = 0 face is
# a signed sum, y = 0 one factor); the phase that updates a field writes their traces only
# where the neighbour is in another tile.  The other faces' traces are written for every
# element and read back as the element's own traces; in-tile neighbours are read from LDS.
RECOMPUTED = (1, 2)


def read_faces(recomputed):
    return tuple(f for f in range(4) if f not in recomputed)


def _blocks(t):
    """Volume modes grouped by (m, k) = (i + j, k): the rows (i, m - i, k), i = 0..m,
    which the first trace factor A couples (one block per column block of A)."""
    idx = {md: r for r, md in enumerate(t.modes)}
    return [[idx[(i, m - i, k)] for i in range(m + 1)] for m in range(t.p + 1) for k in range(t.p - m + 1)]


def _fac_A(t, f):
    return t.fac["A3"] if f == 3 else t.fac["A0"]


def _tangent_terms(g, f, k):
    """Nonzero (component, weight) pairs of the tangential scalar g_fk . w."""
    return [(c, float(g[f][k][c])) for c in range(3) if g[f][k][c] != 0.0]


def _in_cost(g, f, k, nin):
    """LDS loads plus the tangential combination per streamed volume mode."""
    n = len(_tangent_terms(g, f, k))
    return nin * (2 * n - 1)


def _fac_trace_parts(t, f, rows):
    """Dependencies of a factored trace job producing face rows `rows` (psi basis) of
    face f: (rows accumulated before the face-basis change -- on face 0 the
    collapsed-basis rows C couples to `rows` -- and per (m, k) block the needed
    intermediates with their volume inputs)."""
    Bm, C, X = t.fac["B"], t.fac["C"], t.fac["X"]
    A = _fac_A(t, f)
    brows = sorted({int(c) for r in rows for c in np.nonzero(C[r])[0]}) if f == 0 else list(rows)
    xs = sorted({int(x) for c in brows for x in np.nonzero(Bm[c])[0]})
    byblk = {}
    for x in xs:
        a, m, k = X[x]
        byblk.setdefault((m, k), []).append(x)
    parts = []
    for key in sorted(byblk):
        xl = byblk[key]
        ins = sorted({int(c) for x in xl for c in np.nonzero(A[x])[0]})
        parts.append((xl, ins))
    return brows, parts


def _trace_costs(t, g, f, k, rows):
    """(direct, factored) instruction estimates of the trace job (face f, tangent k,
    face rows): streamed inputs, one FMA per operator entry, the 16-byte stores."""
    st = len({m // 4 for m in rows})
    T = t.T[f][rows]
    d = _in_cost(g, f, k, int(np.count_nonzero(np.any(T != 0, axis=0)))) + int(np.count_nonzero(T)) + st
    if f not in FACTORED:
        return d, None
    A, Bm, C = _fac_A(t, f), t.fac["B"], t.fac["C"]
    brows, parts = _fac_trace_parts(t, f, rows)
    c = st
    for xl, ins in parts:
        c += _in_cost(g, f, k, len(ins)) + int(np.count_nonzero(A[np.ix_(xl, ins)]))
        c += int(np.count_nonzero(Bm[np.ix_(brows, xl)]))
    if f == 0:
        c += int(np.count_nonzero(C[np.ix_(rows, brows)]))
    return d, c


def _trace_factored(t, g, f, k, rows):
    d, c = _trace_costs(t, g, f, k, rows)
    return c is not None and c < d


def _trace_job_cost(t, g, f, k, rows):
    d, c = _trace_costs(t, g, f, k, rows)
    return d if c is None else min(d, c)


def _fac_lift_parts(t, f, rows):
    """Dependencies of the factored lift of face f into volume rows `rows`: (needed
    intermediates, collapsed-basis face rows).  Face 0's jumps are converted to the
    collapsed basis once per element (stage C2), so both faces read them directly."""
    A, Bm = _fac_A(t, f), t.fac["B"]
    xs = sorted({int(x) for r in rows for x in np.nonzero(A[:, r])[0]})
    brows = sorted({int(c) for x in xs for c in np.nonzero(Bm[:, x])[0]})
    return xs, brows


def _fac_lift_cost(t, Lp, f, rows):
    A, Bm = _fac_A(t, f), t.fac["B"]
    rs = set(rows)
    groups, cur = [], []
    for blk in _blocks(t):
        if blk[0] not in rs:
            continue
        if cur and len(cur) + len(blk) > LIFT_Y:
            groups.append(cur)
            cur = []
        cur = cur + blk
    if cur:
        groups.append(cur)
    ks = sum(1 for k in range(3) for s_ in range(2) if Lp[f][k][s_] != 0.0)
    c = ks * len(rows)
    for grows in groups:
        xs, brows = _fac_lift_parts(t, f, grows)
        c += (2 * len(brows) + 2 * int(np.count_nonzero(Bm[np.ix_(brows, xs)]))
              + 2 * int(np.count_nonzero(A[np.ix_(xs, grows)])))
    return c


def _direct_lift_cost(t, Lp, f, rows):
    ks = sum(1 for k in range(3) if np.any(Lp[f][k] != 0))
    sub = t.T[f][:, rows]
    nm = int(np.count_nonzero(np.any(sub != 0, axis=1)))
    nnz = int(np.count_nonzero(sub))
    per_row = 2 * nnz + 2 * ks * len(rows) if _lift_per_scalar(t, f, rows, Lp) else ks * (nnz + nm)
    return nm * 4 + per_row


def _lift_factored(t, Lp, f, rows):
    """Face 0 always lifts through the factors (its jumps sit in LDS in the collapsed
    basis); face 3 does when that is cheaper."""
    if f == 0:
        return True
    return f == 3 and _fac_lift_cost(t, Lp, f, rows) < _direct_lift_cost(t, Lp, f, rows)


def _lift_per_scalar(t, f, rows, Lp):
    """Lift the two jumps separately (2 nnz + combine) when cheaper than one lift per
    component that face f reaches (one nnz each)."""
    nnz = int(np.count_nonzero(t.T[f][:, rows]))
    ncomp = sum(1 for k in range(3) if np.any(Lp[f][k] != 0))
    return 2 * nnz + 2 * ncomp * len(rows) < ncomp * nnz


def _out_job_cost(t, Lp, rows):
    """Instruction estimate of an output job: per streamed mode the LDS loads of the
    needed derivative-frame components and the curl FMAs; per face the lift (direct
    table or collapsed factors); the load-FMA-store update of 3 rows each."""
    c = _curl_cost(t, rows)
    for f in range(4):
        c += _fac_lift_cost(t, Lp, f, rows) if _lift_factored(t, Lp, f, rows) else _direct_lift_cost(t, Lp, f, rows)
    return c + 9 * len(rows)


def _curl_cost(t, rows):
    c = 0
    for a in range(t.N):
        hits = [[b for b in rows if t.D[d][b, a] != 0] for d in range(3)]
        if not any(hits):
            continue
        need = set()
        for k in range(3):
            i, j = CYC[k]
            if hits[i]:
                need.add(j)
            if hits[j]:
                need.add(i)
        c += len(need) + 2 + sum(2 * len(h) for h in hits)
    return c


def _balance(items, single, bin_cost, nw, cap, sweeps=4):
    """Partition items over nw bins: greedy (largest item first, into the bin whose
    cost grows least in absolute terms of its new load), then moves of single items
    off the most loaded bin while that lowers the maximum.  bin_cost(list) prices a
    bin; cap(list) says whether a bin may hold the list."""
    bins = [[] for _ in range(nw)]
    load = [0] * nw
    for it in sorted(items, key=lambda x: -single(x)):
        best = None
        for w in range(nw):
            cand = bins[w] + [it]
            if not cap(cand):
                continue
            c = bin_cost(cand)
            if best is None or c < best[0]:
                best = (c, w)
        c, w = best
        bins[w].append(it)
        load[w] = c
    for _ in range(sweeps * len(items)):
        hi = max(range(nw), key=lambda w: load[w])
        moved = False
        for it in sorted(bins[hi], key=single):
            rest = [x for x in bins[hi] if x != it]
            c_hi = bin_cost(rest)
            for w in sorted(range(nw), key=lambda w: load[w]):
                if w == hi or not cap(bins[w] + [it]):
                    continue
                c_w = bin_cost(bins[w] + [it])
                if max(c_hi, c_w) < load[hi]:
                    bins[hi], load[hi] = rest, c_hi
                    bins[w].append(it)
                    load[w] = c_w
                    moved = True
                    break
            if moved:
                break
        if not moved:
            break
    return bins, load


def _plan_traces(t, g, nw, faces=(0, 1, 2, 3), init=None):
    """Trace jobs: one per (face, tangent) -- the job streams the staged field once
    for all face rows of that tangent -- cut into s contiguous runs of quads (four
    face modes, one 16-byte store) where that balances the waves better.  The cut
    counts minimising (largest wave load + mean wave load) are kept; runs go to the
    waves longest first."""
    import itertools

    NF = t.NF
    NQ = (NF + 3) // 4
    units = [(f, k) for f in faces for k in range(2)]
    if not units:
        return [[] for _ in range(nw)], list(init) if init else [0] * nw
    rows_of = lambda i, j: list(range(4 * i, min(NF, 4 * j)))
    cap = 2 * TRACE_ROWS
    memo = {}

    def cost(u, i, j):
        key = (u, i, j)
        if key not in memo:
            r = rows_of(i, j)
            memo[key] = _trace_job_cost(t, g, u[0], u[1], r) if len(r) <= cap else 10 ** 9
        return memo[key]

    def cuts(u, s_u):
        INF = 10 ** 18
        best = [[INF] * (NQ + 1) for _ in range(s_u + 1)]
        arg = [[0] * (NQ + 1) for _ in range(s_u + 1)]
        best[0][0] = 0
        for r in range(1, s_u + 1):
            for j in range(1, NQ + 1):
                for i in range(r - 1, j):
                    v = max(best[r - 1][i], cost(u, i, j))
                    if v < best[r][j]:
                        best[r][j], arg[r][j] = v, i
        out, j = [], NQ
        for r in range(s_u, 0, -1):
            i = arg[r][j]
            out.append((i, j))
            j = i
        return out[::-1]

    smax = min(NQ, max(1, min(3 if nw > 8 else 2, (2 * nw) // len(units))))
    runs = {(u, s_u): cuts(u, s_u) for u in units for s_u in range(1, smax + 1)}
    best = None
    for split in itertools.product(range(1, smax + 1), repeat=len(units)):
        jobs = [(cost(u, i, j), u, i, j) for u, s_u in zip(units, split) for i, j in runs[(u, s_u)]]
        load = list(init) if init else [0] * nw
        assign = [[] for _ in range(nw)]
        for c, u, i, j in sorted(jobs, reverse=True):
            w = min(range(nw), key=lambda w: load[w])
            load[w] += c
            assign[w].append((u[0], u[1], rows_of(i, j)))
        key = (max(load) + sum(load) / nw, len(jobs))
        if best is None or key < best[0]:
            best = (key, assign, load)
    _, assign, load = best
    return [sorted(a) for a in assign], load


def _rebalance_intervals(t, tU, g, Lp, bins, nw, cap, rounds=400):
    """The curl (with the own-trace jobs) and the lift run in different barrier
    intervals, so what counts is each interval's most loaded wave.  Starting from the
    total-cost partition, move single (m, k) blocks between waves while that lowers
    max(curl + own traces) + max(lift + update)."""
    rows_of = lambda bl: sorted(r for b in bl for r in b)
    memo = {}

    def parts(bl):
        key = tuple(sorted(bl))
        if key not in memo:
            rows = rows_of(bl)
            cu = _curl_cost(t, rows) if rows else 0
            memo[key] = (cu, (_out_job_cost(t, Lp, rows) - cu) if rows else 0)
        return memo[key]

    def objective(bs):
        cs = [parts(b) for b in bs]
        _, own = _plan_traces(tU, g, nw, RECOMPUTED, init=[c[0] for c in cs])
        return max(own) + max(c[1] for c in cs)

    bins = [list(b) for b in bins]
    best = objective(bins)
    for _ in range(rounds):
        improved = False
        for a in range(nw):
            for blk in list(bins[a]):
                for b in range(nw):
                    if b == a or len(rows_of(bins[b] + [blk])) > cap:
                        continue
                    cand = [list(x) for x in bins]
                    cand[a].remove(blk)
                    cand[b].append(blk)
                    v = objective(cand)
                    if v < best:
                        best, bins, improved = v, cand, True
                        break
                if improved:
                    break
            if improved:
                break
        if not improved:
            break
    return bins


def _plan_c2(t, nw):
    """Stage C2 tasks (degree n, scalar s): face 0's jumps of degree n converted in
    place from psi to the collapsed basis (C^T), spread over the waves by cost."""
    tasks = sorted(((n + 1) ** 2, n, s_) for n in range(t.p + 1) for s_ in range(2))[::-1]
    load = [0] * nw
    out = [[] for _ in range(nw)]
    for c, n, s_ in tasks:
        w = min(range(nw), key=lambda w: load[w])
        load[w] += c
        out[w].append((n, s_))
    return out


def plan(p: int, nw: int, pU: int = None, pV: int = None):
    """One output job per wave (volume rows, all three components; unions of (m, k)
    blocks, the unit of the factored lift) and the trace jobs above, balanced over
    the nw waves with the instruction estimates above.  With pU, pV (mixed orders) the
    differentiated field U has order pU and the updated field V order pV: U's tables
    drive its own traces and the face-0 conversion, V's tables the trace stage, and
    the coupling tables the curl and the lift."""
    pU = p if pU is None else pU
    pV = p if pV is None else pV
    tU, tV, tC = TB.build(pU), TB.build(pV), TB.coupling(pU, pV)
    g, Lp = TB.face_weights(tU)
    tr_w, tr_load = _plan_traces(tV, g, nw)
    blks = [tuple(b) for b in _blocks(tC)]
    rows_of = lambda bl: sorted(r for b in bl for r in b)
    cap = out_rows_cap(max(pU, pV), min(pU, pV))
    ob, out_load = _balance(blks, lambda b: _out_job_cost(tC, Lp, list(b)),
                            lambda bl: _out_job_cost(tC, Lp, rows_of(bl)), nw,
                            lambda bl: len(rows_of(bl)) <= cap)
    ob = _rebalance_intervals(tC, tU, g, Lp, ob, nw, cap)
    out_load = [_out_job_cost(tC, Lp, rows_of(bl)) for bl in ob]
    out_w = [[rows_of(bl)] if bl else [] for bl in ob]
    # the own-trace jobs share a barrier interval with the curl: balance them together
    curl = [sum(_curl_cost(tC, rows) for rows in w) for w in out_w]
    own_w, own_load = _plan_traces(tU, g, nw, RECOMPUTED, init=curl)
    return dict(trace=tr_w, trace_load=tr_load, out=out_w, out_load=out_load, c2=_plan_c2(tU, nw),
                own=own_w, own_load=own_load)


def trace_strides(NF: int):
    """Trace buffer of one field: per element four faces of FS values (tangent 1,
    then tangent 2, each over the NF face modes padded to NFP, a multiple of four),
    ES = 4 FS per element.  Tile-blocked and quad-interleaved: for the 64 elements
    of a tile, the four values of chunk q (face f, values 4j..4j+3 of the face) of
    lane l sit at ((f FQ + j) 64 + l) 4, so a tile's threads store coalesced and a
    neighbour's chunk is one 16-byte load; a chunk never spans both tangents."""
    NFP = (NF + 3) & ~3
    FS = 2 * NFP
    return FS, 4 * FS


def _lin(terms):
    """Expression of a linear combination [(coef, name)] with literal coefficients."""
    _count(len(terms) - 1 + sum(1 for c, _ in terms if c not in (1.0, -1.0)))
    out = []
    for c, v in terms:
        if c == 1.0:
            out.append(f"+ {v}")
        elif c == -1.0:
            out.append(f"- {v}")
        else:
            out.append(f"+ {_lit(c)} * {v}")
    e = " ".join(out)
    return e[2:] if e.startswith("+ ") else "-" + e[2:]


def _tangent_input(g, f, k, x):
    """(expression statements, scale, name): the tangential scalar of one streamed
    mode from its loaded components x; a single-component tangent is not formed,
    its weight is folded into the operator coefficients instead."""
    terms = _tangent_terms(g, f, k)
    if len(terms) == 1:
        return [], terms[0][1], x[0]
    return [("q", _lin([(w, v) for (c, w), v in zip(terms, x)]))], 1.0, "q"


def _trace_job(a_, t, g, f, k, rows, ind, sink=None):
    """Tangential trace tau_k = g_fk . w on face f, face rows `rows` (whole quads of
    four face modes), of the field staged in LDS (derivative frame), stored to the
    tile's block of Tout with one 16-byte store per lane and quad.  Faces 0 and 3 go
    through the collapsed tensor-product factors when that is cheaper: per (m, k)
    block the inputs are transformed by A into intermediates, which B scatters into
    the face rows (on face 0 rows of the collapsed basis, mapped to psi by C at the
    end)."""
    N = t.N
    sink = sink or (lambda a_, ms, ind: _trace_stores(a_, t, f, k, ms, ind))
    comps = [c for c, _ in _tangent_terms(g, f, k)]
    loads = lambda a: [f"wl[({c * N + a}) * {LANES} + lane]" for c in comps]
    a_(ind + "{")
    blocks = []
    if _trace_factored(t, g, f, k, rows):
        A, Bm, C = _fac_A(t, f), t.fac["B"], t.fac["C"]
        brows, parts = _fac_trace_parts(t, f, rows)
        acc = (lambda c: f"tc_{c}") if f == 0 else (lambda c: f"ts_{c}")
        a_(ind + "  R " + ", ".join(f"{acc(c)} = R(0)" for c in brows) + ";")
        for xl, ins in parts:
            def body(x, xl=xl, ins=ins):
                out, names, sc = [], [], 1.0
                for n, a in enumerate(ins):
                    pre, sc, nm = _tangent_input(g, f, k, x[n * len(comps):(n + 1) * len(comps)])
                    for v, e in pre:
                        out.append(f"const R {v}{n} = {e};")
                        nm = f"{v}{n}"
                    names.append(nm)
                for xi in xl:
                    out.append(f"const R y_{xi} = " + _lin([(sc * A[xi, a], names[n]) for n, a in enumerate(ins)
                                                            if A[xi, a] != 0.0]) + ";")
                for xi in xl:
                    for c in brows:
                        if Bm[c, xi] != 0.0:
                            out.append(_fma(acc(c), Bm[c, xi], f"y_{xi}"))
                return out
            blocks.append(([l for a in ins for l in loads(a)], body))
        a_(ind + "  {")
        _Stream(a_, ind + "    ", "pf").emit(blocks)
        a_(ind + "  }")
        if f == 0:
            a_(ind + "  // change of face basis (collapsed towards the first vertex -> psi), per quad")
            for mq in sorted({m // 4 for m in rows}):
                ms = [m for m in range(4 * mq, 4 * mq + 4) if m in rows]
                a_(ind + "  {")
                for m in ms:
                    a_(ind + f"    const R ts_{m} = " + _lin([(C[m, c], f"tc_{c}") for c in brows if C[m, c] != 0.0]) + ";")
                sink(a_, ms, ind + "  ")
                a_(ind + "  }")
            a_(ind + "}")
            return
    else:
        T = t.T[f]
        a_(ind + "  R " + ", ".join(f"ts_{m} = R(0)" for m in rows) + ";")
        for a in range(N):
            ms = [m for m in rows if T[m, a] != 0]
            if not ms:
                continue

            def body(x, a=a, ms=ms):
                pre, sc, nm = _tangent_input(g, f, k, x)
                out = [f"const R {v} = {e};" for v, e in pre]
                for m in ms:
                    out.append(_fma(f"ts_{m}", sc * T[m, a], nm))
                return out
            blocks.append((loads(a), body))
        a_(ind + "  {")
        _Stream(a_, ind + "    ", "pf").emit(blocks)
        a_(ind + "  }")
    sink(a_, rows, ind)
    a_(ind + "}")


def _trace_stores(a_, t, f, k, rows, ind, pred=None):
    """16-byte stores of the quads of `rows` to the tile's block of Tout (only lanes with
    `pred`, if given)."""
    FS, ES = trace_strides(t.NF)
    NFP, FQ = FS // 2, FS // 4
    for mq in sorted({m // 4 for m in rows}):
        vals = [f"ts_{m}" if m in rows else "R(0)" for m in range(4 * mq, 4 * mq + 4)]
        chunk = f * FQ + (k * NFP + 4 * mq) // 4
        st = f"store4s<ST>(Tout + tb + ({chunk} * {LANES} + lane) * 4, {', '.join(vals)});"
        a_(ind + ("  " + st if pred is None else f"  if ({pred}) {st}"))


def _curl_job(a_, t, rows, ind):
    """Curl part of the rates of the wave's rows (all three components, derivative
    frame from LDS) into the accumulator slots 0..len(rows)-1."""
    N = t.N
    a_(ind + "{")
    blocks = []
    for a in range(N):
        hits = {d: [(j, b) for j, b in enumerate(rows) if t.D[d][b, a] != 0] for d in range(3)}
        if not any(hits.values()):
            continue
        need = set()
        for k in range(3):
            i, jj = CYC[k]
            if hits[i]:
                need.add(jj)
            if hits[jj]:
                need.add(i)

        def body(x, a=a, hits=hits, need=need):
            out = [f"const R w{c} = {v};" for c, v in zip(sorted(need), x)]
            for k in range(3):
                i, jj = CYC[k]
                for j, b in hits[i]:
                    out.append(_fma(f"acc{k}_{j}", t.D[i][b, a], f"w{jj}"))
                for j, b in hits[jj]:
                    out.append(_fma(f"acc{k}_{j}", -t.D[jj][b, a], f"w{i}"))
            return out

        blocks.append(([f"wl[({c * N + a}) * {LANES} + lane]" for c in sorted(need)], body))
    a_(ind + "  {")
    _Stream(a_, ind + "    ", "pf").emit(blocks)
    a_(ind + "  }")
    a_(ind + "}")



LIFT_Y = 8  # intermediates per scalar held at once by a factored lift (bounds its registers)


def _lift_face_fac(a_, t, Lp, f, rows, jd, ind):
    """Lift of face f's two jumps into the job's rows through the transposed
    collapsed tensor-product factors: B^T from the collapsed-basis face rows (face
    3: psi itself; face 0: the rows stage C2 converted) into the intermediates y_s,
    A^T into the rows, then the stored-frame map Lp_f of the two scalars into the
    three components.  The job's (m, k) blocks are taken in groups of at most LIFT_Y
    intermediates, each group streaming the face rows it needs."""
    A, Bm = _fac_A(t, f), t.fac["B"]
    pos = {b: j for j, b in enumerate(rows)}
    groups, cur = [], []
    for blk in _blocks(t):
        if blk[0] not in pos:
            continue
        if cur and len(cur) + len(blk) > LIFT_Y:
            groups.append(cur)
            cur = []
        cur = cur + blk
    if cur:
        groups.append(cur)
    a_(ind + f"  {{  // face {f}, collapsed tensor-product factors")
    for grows in groups:
        xs, brows = _fac_lift_parts(t, f, grows)
        a_(ind + "    {")
        a_(ind + "      R " + ", ".join(f"y{s_}_{x} = R(0)" for x in xs for s_ in range(2)) + ";")
        blocks = []
        for c in brows:
            def body(x, c=c, xs=xs):
                out = []
                for xi in xs:
                    if Bm[c, xi] != 0.0:
                        for s_ in range(2):
                            out.append(_fma(f"y{s_}_{xi}", Bm[c, xi], x[s_]))
                return out
            blocks.append(([jd(f, 0, c), jd(f, 1, c)], body))
        a_(ind + "      {")
        _Stream(a_, ind + "        ", "pj").emit(blocks)
        a_(ind + "      }")
        for b in grows:
            j = pos[b]
            terms = [(A[xi, b], xi) for xi in xs if A[xi, b] != 0.0]
            if not terms:
                continue
            for s_ in range(2):
                a_(ind + f"      const R l{s_}_{j} = " + _lin([(c, f"y{s_}_{xi}") for c, xi in terms]) + ";")
            for k in range(3):
                for s_ in range(2):
                    if Lp[f][k][s_] != 0.0:
                        a_(ind + "      " + _fma(f"acc{k}_{j}", Lp[f][k][s_], f"l{s_}_{j}"))
        a_(ind + "    }")
    a_(ind + "  }")


def _lift_job(a_, t, Lp, rows, ind):
    """Lifted jumps (from LDS) added to the rates of the wave's rows, face by face,
    then the update V = V_old + sdt * rate of the three components (old values
    fetched before the lift arithmetic when the registers allow)."""
    N, NF = t.NV, t.NF
    a_(ind + "{")
    early = vo_early(getattr(t, "launch_p", t.p))
    if early:
        a_(ind + "  // old values of the updated rows")
        for j, b in enumerate(rows):
            a_(ind + "  const R " + ", ".join(f"vo{k}_{j} = RATE ? R(0) : ldf<ST>(&V[({k * N + b}) * Ks + el])" for k in range(3)) + ";")
    jd = lambda f, k, m: f"wl[({(f * 2 + k) * NF + m}) * {LANES} + lane]"
    for f in range(4):
        if _lift_factored(t, Lp, f, rows):
            _lift_face_fac(a_, t, Lp, f, rows, jd, ind)
            continue
        ks = [k for k in range(3) if np.any(Lp[f][k] != 0)]
        ms = [m for m in range(NF) if np.any(t.T[f][m, rows] != 0)]
        if not ks or not ms:
            continue
        per_scalar = _lift_per_scalar(t, f, rows, Lp)
        lblocks = []
        for m in ms:
            def body(x, f=f, m=m, ks=ks, per_scalar=per_scalar):
                out = []
                for j, b in enumerate(rows):
                    c = t.T[f][m, b]
                    if c == 0:
                        continue
                    if per_scalar:
                        out.append(_fma(f"l0_{j}", c, x[0]))
                        out.append(_fma(f"l1_{j}", c, x[1]))
                for k in ks if not per_scalar else []:
                    c0, c1 = Lp[f][k]
                    terms = []
                    if c0 != 0.0:
                        terms.append(f"{_lit(c0)} * {x[0]}")
                    if c1 != 0.0:
                        terms.append(f"{_lit(c1)} * {x[1]}")
                    _count(2 * len(terms) - 1)
                    out.append(f"const R g{k} = {' + '.join(terms)};")
                    for j, b in enumerate(rows):
                        c = t.T[f][m, b]
                        if c != 0:
                            out.append(_fma(f"acc{k}_{j}", c, f"g{k}"))
                return out
            lblocks.append(([jd(f, 0, m), jd(f, 1, m)], body))
        a_(ind + f"  {{  // face {f}")
        used = [j for j, b in enumerate(rows) if np.any(t.T[f][:, b] != 0)]
        if per_scalar:
            a_(ind + "    R " + ", ".join(f"l{k}_{j} = R(0)" for j in used for k in range(2)) + ";")
        a_(ind + "    {")
        _Stream(a_, ind + "      ", "pj").emit(lblocks)
        a_(ind + "    }")
        if per_scalar:
            for j in used:
                for k in ks:
                    c0, c1 = Lp[f][k]
                    if c0 != 0.0:
                        a_(ind + "    " + _fma(f"acc{k}_{j}", c0, f"l0_{j}"))
                    if c1 != 0.0:
                        a_(ind + "    " + _fma(f"acc{k}_{j}", c1, f"l1_{j}"))
        a_(ind + "  }")
    # the new values stay in the accumulator slots (the traces of V are formed from them)
    for j, b in enumerate(rows):
        for k in range(3):
            old = f"vo{k}_{j}" if early else f"(RATE ? R(0) : ldf<ST>(&V[({k * N + b}) * Ks + el]))"
            _count(2)
            a_(ind + f"  acc{k}_{j} = {old} + sdt * acc{k}_{j};")
    a_(ind + "  if (act) {")
    for j, b in enumerate(rows):
        for k in range(3):
            a_(ind + f"    stf<ST>(&V[({k * N + b}) * Ks + e], acc{k}_{j});")
    a_(ind + "  }")
    a_(ind + "}")


def lds_words(p: int, q: int = None) -> int:
    """LDS words of one workgroup (with q: a mixed-order kernel of orders p and q, the
    larger of the two areas)."""
    if q is not None and q != p:
        return max(lds_words(p), lds_words(q))
    return _lds_words(p)


def _lds_words(p: int) -> int:
    """LDS words of one workgroup: one area, holding in turn the staged field
    (3N x 64) and the trace jumps (8NF x 64)."""
    t = TB.build(p)
    return max(3 * t.N, 8 * t.NF) * LANES


# Waves per workgroup and whether a wave fetches the old values of its rows before
# the lift (else at the update), per order; chosen by timing the p = 6, 7, 8 phase
# kernels on the 32^3 mesh (16 waves at p = 8 need the late fetch to avoid spills).
LAUNCH = {8: (16, False)}


def waves_for(p: int) -> int:
    return LAUNCH[p][0] if p in LAUNCH else (8 if p >= 4 else 4)


def vo_early(p: int) -> bool:
    return LAUNCH[p][1] if p in LAUNCH else True


def out_rows_cap(p: int, q: int = None) -> int:
    """Volume rows per output job: OUT_ROWS, or 12 where the launch leaves a lane 128
    registers (four waves per SIMD), so that the rows' accumulators, a factored lift's
    intermediates and a stream group fit without spilling."""
    waves_per_simd = max(1, waves_for(p) * groups_per_cu(p, 4, q) // 4)
    return 12 if 512 // waves_per_simd <= 128 else OUT_ROWS


def groups_per_cu(p: int, elem_bytes: int, q: int = None) -> int:
    """Workgroups that share a compute unit (LDS bound, at most 2)."""
    return max(1, min(2, LDS_BUDGET // (lds_words(p, q) * elem_bytes)))


def _stage_parts(t, nw, X, mp):
    """wl = M X for the tile (M from the 6-component table mp): wave w converts modes
    w, w + nw, ... of all 64 elements.  Returns (loads, stores): every load of the
    wave is issued before the first conversion (one memory round trip); the last mode
    index is clamped, so a wave past the end rewrites mode N - 1 with the same values."""
    N = t.N
    cnt = -(-N // nw)
    # an opaque copy of the element index keeps the compiler from sharing this
    # stage's address arithmetic with another stage (which would hold it in
    # registers across the barriers in between)
    ld = ["int ez = el, lz = lane;", "asm volatile(\"\" : \"+v\"(ez), \"+v\"(lz));",
          f"const R n00 = {mp}[0 * Ks + ez], n01 = {mp}[1 * Ks + ez], n02 = {mp}[2 * Ks + ez];",
          f"const R n11 = {mp}[3 * Ks + ez], n12 = {mp}[4 * Ks + ez], n22 = {mp}[5 * Ks + ez];"]
    st = []
    for i in range(cnt):
        idx = f"wave + {i * nw}" if i < cnt - 1 else f"min(wave + {i * nw}, {N - 1})"
        ld.append(f"const int a{i} = {idx};")
        ld.append(f"const R s{i}_0 = ldf<ST>(&{X}[(size_t)a{i} * Ks + ez]), "
                  f"s{i}_1 = ldf<ST>(&{X}[(size_t)({N} + a{i}) * Ks + ez]), "
                  f"s{i}_2 = ldf<ST>(&{X}[(size_t)({2 * N} + a{i}) * Ks + ez]);")
        _count(15)
        st.append(f"wl[a{i} * {LANES} + lz] = n00 * s{i}_0 + n01 * s{i}_1 + n02 * s{i}_2;")
        st.append(f"wl[({N} + a{i}) * {LANES} + lz] = n01 * s{i}_0 + n11 * s{i}_1 + n12 * s{i}_2;")
        st.append(f"wl[({2 * N} + a{i}) * {LANES} + lz] = n02 * s{i}_0 + n12 * s{i}_1 + n22 * s{i}_2;")
    return ld, st


def _stage_field(a_, t, nw, X, mp):
    ld, st = _stage_parts(t, nw, X, mp)
    a_("  {")
    for l in ld + st:
        a_("    " + l)
    a_("  }")


JUMP_BATCH = 4    # trace chunks per lane loaded before their LDS stores


def _jump_items(t, nw):
    NFP = trace_strides(t.NF)[0] // 2
    items = [(k, jq) for k in range(2) for jq in range(NFP // 4)]
    return items, -(-len(items) // nw)


def _jump_prefetch(t, nw):
    """Declarations of the jump stage at kernel scope: per face the neighbour code and
    whether the neighbour is in the tile, and the 16-byte chunks of the off-tile
    neighbours for this wave's items (loaded here, used after the next barrier)."""
    NF = t.NF
    FS, ES = trace_strides(NF)
    NFP, FQ = FS // 2, FS // 4
    items, cnt = _jump_items(t, nw)
    L = ["const int code0 = nbr[el], code1 = nbr[Ks + el], code2 = nbr[2 * Ks + el], code3 = nbr[3 * Ks + el];"]
    for f in range(4):
        L.append(f"const int nb{f} = code{f} >= 0 ? code{f} >> 2 : el, gf{f} = code{f} >= 0 ? code{f} & 3 : {f};")
        L.append(f"const bool in{f} = code{f} >= 0 && (nb{f} >> 6) == tile, off{f} = code{f} >= 0 && !in{f};")
    for i in range(cnt):
        L.append(f"R " + ", ".join(f"t{i}_{f}_{jj} = R(0)" for f in range(4) for jj in range(4)) + ";")
        guard = f"wave + {i * nw} < {len(items)}"
        L.append(f"{{ const int it = min(wave + {i * nw}, {len(items) - 1}), k = it / {NFP // 4}, c = 4 * (it - k * {NFP // 4});")
        for f in range(4):
            L.append(f"  if (off{f} && {guard}) {{")
            L.append(f"    const R* sn = (const R*)__builtin_assume_aligned(Tin + (size_t)(nb{f} >> 6) * {LANES * ES} "
                     f"+ ((size_t)(gf{f} * {FQ} + (k * {NFP} + c) / 4) * {LANES} + (nb{f} & 63)) * 4, 16);")
            L.append("    " + " ".join(f"t{i}_{f}_{jj} = sn[{jj}];" for jj in range(4)))
            L.append("  }")
        L.append("}")
    return L


def _jump_lines(t, nw):
    """Jumps of the tangential traces of U (own traces already in LDS, stage T):
    neighbour minus own on interior faces, (wall - 1) times own on walls.  A neighbour
    in the same tile is read from LDS, one in another tile was loaded from Tin (one
    16-byte load of its face block) before the barrier (_jump_prefetch).  Work item
    (k, j): tangent k, face modes 4j..4j+3 of all four faces; every read of an item's
    own and neighbour values (same tangent and modes, any face) is made by the wave
    that then overwrites them with the jumps, so the jumps replace the own traces in
    place without a barrier.  Wave w takes items w, w + nw, ...; items past the end
    are skipped (a duplicate would race with the in-place update)."""
    NF = t.NF
    NFP = trace_strides(NF)[0] // 2
    items, cnt = _jump_items(t, nw)
    L = ["const R cw = wall - R(1);"]
    for i in range(cnt):
        L.append(f"if (wave + {i * nw} < {len(items)}) {{" if (i + 1) * nw > len(items) else "{")
        L.append(f"  const int it = wave + {i * nw}, k = it / {NFP // 4}, c = 4 * (it - k * {NFP // 4});")
        for jj in range(4):
            L.append(f"  if (c + {jj} < {NF}) {{" if NF % 4 else "  {")
            L.append(f"    const int m = c + {jj};")
            for f in range(4):
                L.append(f"    const R ow{f} = wl[((({f} * 2 + k) * {NF}) + m) * {LANES} + lane];")
                L.append(f"    const R nv{f} = wl[(((gf{f} * 2 + k) * {NF}) + m) * {LANES} + (nb{f} & 63)];")
            _count(4)
            for f in range(4):
                L.append(f"    R jf{f} = code{f} < 0 ? cw * ow{f} : (in{f} ? nv{f} : t{i}_{f}_{jj}) - ow{f};")
            # stabilised flux, E phase: the face unknowns (held by the face's owner side)
            # enter the jump of H as -2 sigma (-4 sigma on walls, whose test-function jump is 2 e)
            L.append("    if constexpr (STAB) {")
            L.append("      if (wall > R(0)) {")
            L.append(f"        const size_t hb = (size_t)((k * {NF} + m) * 4) * Ks;")
            for f in range(4):
                L.append(f"        {{ const bool own = code{f} < 0 || el < nb{f};")
                L.append(f"          jf{f} -= (code{f} < 0 ? R(4) : R(2)) * HF[hb + (size_t)(own ? {f} : gf{f}) * Ks + (own ? el : nb{f})]; }}")
            L.append("      }")
            L.append("    }")
            for f in range(4):
                L.append(f"    wl[((({f} * 2 + k) * {NF}) + m) * {LANES} + lane] = jf{f};")
            L.append("  }")
        L.append("}")
    return L


def _stab_stage(a_, t, nw):
    """Stabilised flux, H phase: the face unknowns sigma (tangential components
    H^F . t_k of every face mode, held by the face's owner side: the element with the
    smaller index, or the element itself on a wall) advance from the jumps of E in
    LDS, sigma += fdt * C_f (dtau_0, dtau_1) with the owner's 2x2 matrix
    C_f = -(alpha / h_F) c_f, nu x t_k = sum_i c_f[k][i] t_i.  Layout of HF:
    ((k NF + m) 4 + f) K + e.  Wave w takes modes w, w + nw, ...; then a barrier
    (stage C2 overwrites face 0's jumps)."""
    NF = t.NF
    a_("  if constexpr (STAB) {")
    a_("    if (wall < R(0) && act) {")
    for f in range(4):
        a_(f"      const bool so{f} = code{f} < 0 || el < nb{f};")
        a_(f"      const R sc{f}_0 = SC[{4 * f + 0} * Ks + el], sc{f}_1 = SC[{4 * f + 1} * Ks + el], "
           f"sc{f}_2 = SC[{4 * f + 2} * Ks + el], sc{f}_3 = SC[{4 * f + 3} * Ks + el];")
    a_(f"      for (int m = wave; m < {NF}; m += {nw}) {{")
    for f in range(4):
        a_(f"        if (so{f}) {{")
        a_(f"          const R d0 = wl[({2 * f} * {NF} + m) * {LANES} + lane], d1 = wl[({2 * f + 1} * {NF} + m) * {LANES} + lane];")
        a_(f"          R* h0 = HF + ((size_t)(m * 4 + {f})) * Ks + el;")
        a_(f"          R* h1 = HF + ((size_t)(({NF} + m) * 4 + {f})) * Ks + el;")
        a_(f"          const R u0 = *h0 + fdt * (sc{f}_0 * d0 + sc{f}_1 * d1);")
        a_(f"          const R u1 = *h1 + fdt * (sc{f}_2 * d0 + sc{f}_3 * d1);")
        a_("          *h0 = u0;")
        a_("          *h1 = u1;")
        a_("        }")
    a_("      }")
    a_("    }")
    a_("    __syncthreads();")
    a_("  }")


def _c2_stage(a_, t, pl, nw):
    """Stage C2: face 0's jump rows of each degree n (both scalars) replaced by their
    coordinates in the collapsed face basis, C^T J (C only mixes equal degrees)."""
    C = t.fac["C"]
    NF = t.NF
    fdeg = [a + b for (a, b) in t.fmodes]
    for w in range(nw):
        if not pl["c2"][w]:
            continue
        a_(f"  if (wave == {w}) {{")
        for n, s_ in pl["c2"][w]:
            rs = [r for r in range(NF) if fdeg[r] == n]
            assert np.all(C[np.ix_([r for r in range(NF) if fdeg[r] != n], rs)] == 0.0)
            a_("    {")
            a_("      const R " + ", ".join(f"j{r} = wl[({s_ * NF + r}) * {LANES} + lane]" for r in rs) + ";")
            for c in rs:
                a_(f"      wl[({s_ * NF + c}) * {LANES} + lane] = " + _lin([(C[r, c], f"j{r}") for r in rs if C[r, c] != 0.0]) + ";")
            a_("    }")
        a_("  }")


def _trace_stage(a_, t, g, pl, nw, masked=True):
    """Trace jobs of the field staged in LDS, stored straight to the tile's block.  With
    `masked`, the recomputed faces are stored only by lanes whose neighbour across that
    face lies in another tile, and their jobs run only in waves that have such a lane."""
    a_(f"  const size_t tb = (size_t)tile * {LANES * trace_strides(t.NF)[1]};")
    if masked:
        for f in RECOMPUTED:
            a_(f"  const int cdf{f} = nbr[{f} * Ks + el];")
            a_(f"  const bool nd{f} = cdf{f} >= 0 && (cdf{f} >> 8) != tile;")
            a_(f"  const bool any{f} = __any(nd{f});")
    for w in range(nw):
        a_(f"  if (wave == {w}) {{")
        for (f, k, rows) in pl["trace"][w]:
            a_(f"    // face {f}, tangent {k}, face modes {rows[0]}..{rows[-1]}")
            if masked and f in RECOMPUTED:
                a_(f"    if (any{f})")
                _trace_job(a_, t, g, f, k, rows, "    ",
                           sink=lambda a_, ms, ind, f=f, k=k: _trace_stores(a_, t, f, k, ms, ind, pred=f"nd{f}"))
            else:
                _trace_job(a_, t, g, f, k, rows, "    ")
        a_("  }")


def _own_trace_stage(a_, t, g, pl, nw):
    """Stage T: the element's own traces of U on every face into LDS at
    ((f 2 + k) NF + m) 64 + lane -- the recomputed faces from the staged field (held in
    registers across the barrier that frees the area), the others read from the tile's
    block of Tin (one coalesced 16-byte load per lane and quad)."""
    NF = t.NF
    FS, ES = trace_strides(NF)
    NFP, FQ = FS // 2, FS // 4
    slots = [[(f, k, m) for (f, k, rows) in pl["own"][w] for m in rows] for w in range(nw)]
    M = max((len(x) for x in slots), default=0)
    if M:
        a_("  R " + ", ".join(f"ot{i}" for i in range(M)) + ";")
    for w in range(nw):
        if not slots[w]:
            continue
        pos = {x: i for i, x in enumerate(slots[w])}
        a_(f"  if (wave == {w}) {{")
        for (f, k, rows) in pl["own"][w]:
            def sink(a_, ms, ind, f=f, k=k, pos=pos):
                for m in ms:
                    a_(ind + f"  ot{pos[(f, k, m)]} = ts_{m};")
            a_(f"    // own trace: face {f}, tangent {k}, face modes {rows[0]}..{rows[-1]}")
            _trace_job(a_, t, g, f, k, rows, "    ", sink=sink)
        a_("  }")
    a_("  __syncthreads();")
    for w in range(nw):
        if not slots[w]:
            continue
        a_(f"  if (wave == {w}) {{")
        for i, (f, k, m) in enumerate(slots[w]):
            a_(f"    wl[{((f * 2 + k) * NF + m) * LANES} + lane] = ot{i};")
        a_("  }")
    # own traces of the read faces: chunk-parallel over the waves, loads issued first
    chunks = [f * FQ + j for f in read_faces(RECOMPUTED) for j in range(FQ)]
    cnt = -(-len(chunks) // nw) if chunks else 0
    if cnt:
        a_(f"  const R* __restrict__ tin = Tin + (size_t)tile * {LANES * ES} + (size_t)lane * 4;")
        a_("  static constexpr short kChunks[" + str(len(chunks)) + "] = {" + ", ".join(map(str, chunks)) + "};")
    for i in range(cnt):
        ci = f"wave + {i * nw}" if i < cnt - 1 else f"min(wave + {i * nw}, {len(chunks) - 1})"
        a_(f"  const int oq{i} = kChunks[{ci}];")
        a_(f"  const R* so{i} = (const R*)__builtin_assume_aligned(tin + (size_t)oq{i} * {LANES * 4}, 16);")
        a_(f"  const R o{i}_0 = so{i}[0], o{i}_1 = so{i}[1], o{i}_2 = so{i}[2], o{i}_3 = so{i}[3];")
    a_("  // the jump stage's off-tile neighbour chunks, in flight across the next barrier")
    for l in _jump_prefetch(t, nw):
        a_("  " + l)
    for i in range(cnt):
        a_(f"  {{ const int f = oq{i} / {FQ}, c = 4 * (oq{i} - f * {FQ}), k = c >= {NFP}, m = c - k * {NFP};")
        a_(f"    const int d = ((f * 2 + k) * {NF} + m) * {LANES} + lane;")
        for jj in range(4):
            st = f"wl[d + {jj * LANES}] = o{i}_{jj};"
            a_(f"    {st}" if (jj == 0 and NF % 4 == 0) else f"    if (m + {jj} < {NF}) {st}")
        a_("  }")


def _phase_body(a_, tU, tV, tC, g, Lp, pl, nw):
    """Stages of one phase (shared by the single-mesh and the batched kernel), one
    LDS area used in turn: A stage U (derivative frame), B curl of the wave's rows
    into registers, C jumps of the traces of U, D lift + update of V, and if Tout:
    E the updated rows (kept in registers) into LDS in the derivative frame of V,
    F its traces to Tout.  tU: tables of U's order (staging, own traces, jumps, face-0
    conversion), tV: of V's order (its traces), tC: the coupling (curl and lift)."""
    N = tV.N
    J = max(len(rows) for w in pl["out"] for rows in w) if any(pl["out"]) else 0
    for k in range(3):
        for j0 in range(0, J, 16):
            a_("  R " + ", ".join(f"acc{k}_{j} = R(0)" for j in range(j0, min(J, j0 + 16))) + ";")
    a_("  // A: the tile's own field in the derivative frame, w = M S, into LDS")
    _stage_field(a_, tU, nw, "U", "MU")
    a_("  __syncthreads();")
    a_("  // B: curl of the wave's rows (all components) into registers")
    for w in range(nw):
        a_(f"  if (wave == {w}) {{")
        for rows in pl["out"][w]:
            a_(f"    // volume modes {', '.join(map(str, rows))}")
            _curl_job(a_, tC, rows, "    ")
        a_("  }")
    a_("  // T: own traces of U on every face into LDS (recomputed faces from the staged")
    a_("  // field, the others from Tin)")
    _own_trace_stage(a_, tU, g, pl, nw)
    a_("  __syncthreads();")
    a_("  // C: jumps of the traces of U (neighbour from LDS in the tile, else from Tin)")
    a_("  {")
    for l in _jump_lines(tU, nw):
        a_("    " + l)
    a_("  }")
    a_("  __syncthreads();")
    _stab_stage(a_, tU, nw)
    a_("  // C2: face 0's jumps from psi to the collapsed basis of the lift factors, in place")
    _c2_stage(a_, tU, pl, nw)
    a_("  __syncthreads();")
    a_("  // D: lifted jumps and the component-separable update of V")
    for w in range(nw):
        a_(f"  if (wave == {w}) {{")
        for rows in pl["out"][w]:
            _lift_job(a_, tC, Lp, rows, "    ")
        a_("  }")
    FLOPS_NO_TRACE = FLOPS[0]
    a_("  if (Tout == nullptr) return;")
    a_("  // E: the updated rows (still in registers) in the derivative frame into LDS")
    a_("  {")
    a_("    const R n00 = MV[0 * Ks + el], n01 = MV[1 * Ks + el], n02 = MV[2 * Ks + el];")
    a_("    const R n11 = MV[3 * Ks + el], n12 = MV[4 * Ks + el], n22 = MV[5 * Ks + el];")
    a_("    __syncthreads();")
    for w in range(nw):
        a_(f"    if (wave == {w}) {{")
        for rows in pl["out"][w]:
            for j, b in enumerate(rows):
                _count(15)
                a_(f"      wl[{b} * {LANES} + lane] = n00 * acc0_{j} + n01 * acc1_{j} + n02 * acc2_{j};")
                a_(f"      wl[{N + b} * {LANES} + lane] = n01 * acc0_{j} + n11 * acc1_{j} + n12 * acc2_{j};")
                a_(f"      wl[{2 * N + b} * {LANES} + lane] = n02 * acc0_{j} + n12 * acc1_{j} + n22 * acc2_{j};")
        a_("    }")
    a_("  }")
    a_("  __syncthreads();")
    a_("  // F: its traces for the next phase")
    before_f = FLOPS[0]
    _trace_stage(a_, tV, g, pl, nw)
    return dict(no_traces=FLOPS_NO_TRACE, with_traces=FLOPS[0], trace_stage=FLOPS[0] - before_f)


def _kernel_setup(p, pU=None, pV=None):
    """Tables and plan of the kernel of order p, or of the mixed-order kernel
    differentiating order pU and updating order pV (launched as order max(pU, pV))."""
    pU = p if pU is None else pU
    pV = p if pV is None else pV
    tU, tV, tC = TB.build(pU), TB.build(pV), TB.coupling(pU, pV)
    if pU != pV:
        tC.launch_p = max(pU, pV)
    g, Lp = TB.face_weights(tU)
    nw = waves_for(max(pU, pV))
    return tU, tV, tC, g, Lp, nw, plan(p, nw, pU, pV)


def _launch_bounds(p, nw, q=None):
    """Threads per workgroup and minimum waves per SIMD (from the LDS-bound number
    of workgroups per CU at FP32), which caps the registers per lane."""
    return f"__launch_bounds__({nw * LANES}, {max(1, nw * groups_per_cu(p, 4, q) // 4)})"


def _tile_prologue(a_):
    a_("  const int nbk = gridDim.x, bid = blockIdx.x;")
    a_("  // XCD-aware tile order: block b runs on XCD b % 8, so give every XCD a")
    a_("  // contiguous range of element tiles and keep neighbour data in its L2")
    a_("  const int per = nbk >> 3, rem = nbk & 7, xcd = bid & 7;")
    a_("  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);")


def _elem_prologue(a_):
    a_(f"  const int lane = threadIdx.x & {LANES - 1};")
    a_("  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);")
    a_(f"  const int e = tile * {LANES} + lane;")
    a_("  const bool act = e < K;")
    a_("  const int el = act ? e : K - 1;")
    a_("  const size_t Ks = (size_t)K;")


def _header(a_, p, t, nw, pl, what, q=None):
    FS, ES = trace_strides(t.NF)
    a_(f"// Generated by gen/emit.py for order p = {p}: N = {t.N} volume modes, NF = {t.NF} face modes; {what}.")
    a_(f"// {nw} waves share {LANES} elements (one per lane), {lds_words(p, q)} LDS words; trace buffer")
    a_(f"// strides: face {FS}, element {ES}; per-wave cost of the trace jobs {pl['trace_load']},")
    a_(f"// of the update jobs {pl['out_load']}.")
    a_(f"static_assert(trace_face_stride({t.NF}) == {FS} && trace_elem_stride({t.NF}) == {ES}, \"trace layout\");")


def emit_phase(p: int, pU: int = None, pV: int = None, name: str = None) -> str:
    """Single-mesh phase kernel of order p, or (pU, pV) the mixed-order kernel that
    differentiates a field of order pU and updates one of order pV."""
    tU, tV, tC, g, Lp, nw, pl = _kernel_setup(p, pU, pV)
    mixed = tU.p != tV.p
    q = min(tU.p, tV.p) if mixed else None
    kp = max(tU.p, tV.p)
    name = name or f"dgm_phase_p{p}"
    L = []
    a_ = L.append
    _header(a_, kp, tU, nw, pl, f"single-mesh phase, U of order {tU.p}, V of order {tV.p}" if mixed
            else "single-mesh phase", q)
    if mixed:
        a_(f"static_assert(trace_face_stride({tV.NF}) == {trace_strides(tV.NF)[0]}, \"trace layout of V\");")
    a_("// ST: field loads and stores and trace stores carry the nontemporal hint (launch.h)")
    a_("// STAB: stabilised central flux with face unknowns HF (Section 2.1)")
    a_("// RATE: V is only written, V = sdt * rate (a rate into a buffer that is not cleared first)")
    a_("template <typename R, bool ST, bool STAB, bool RATE>")
    a_(f"__global__ void {_launch_bounds(kp, nw, q)} {name}(const R* __restrict__ U, R* __restrict__ V,")
    a_("    const R* __restrict__ MU, const R* __restrict__ MV, const int* __restrict__ nbr,")
    a_("    const R* __restrict__ Tin, R* __restrict__ Tout, R sdt, R wall, int K,")
    a_("    R* __restrict__ HF, const R* __restrict__ SC, R fdt)")
    a_("{")
    if mixed:
        a_("  static_assert(!STAB, \"the stabilised flux is built for equal orders\");")
    a_(f"  __shared__ R wl[{lds_words(kp, q)}];")
    _tile_prologue(a_)
    _elem_prologue(a_)
    FLOPS[0] = 0
    cnt = _phase_body(a_, tU, tV, tC, g, Lp, pl, nw)
    # the recomputed faces' trace jobs in stage F run only in tiles with an off-tile
    # neighbour across that face: their share is reported apart
    FLOPS[0] = 0
    for w in range(nw):
        for (f, k, rows) in pl["trace"][w]:
            if f in RECOMPUTED:
                _trace_job(lambda x: None, tV, g, f, k, rows, "", sink=lambda *a: None)
    cnt["trace_stage_recomputed_faces"] = FLOPS[0]
    if not mixed:
        OPCOUNT[p] = dict(cnt, N=tU.N, NF=tU.NF, waves=nw)
    a_("}")
    return "\n".join(L) + "\n"


def emit_trace(p: int) -> str:
    """Trace kernel of order p: the traces of one field (the first phase of a run
    and the rate operator need them before any phase has written them).  Like the
    phase kernels' trace stage it stores the x = 0 and y = 0 faces only where the
    neighbour across them lies in another tile (inside a tile they pass through LDS)."""
    t, _, _, g, Lp, nw, pl = _kernel_setup(p)
    L = []
    a_ = L.append
    _header(a_, p, t, nw, pl, "trace kernel")
    a_("template <typename R>")
    a_(f"__global__ void {_launch_bounds(p, nw)} dgm_trace_p{p}(const R* __restrict__ U,")
    a_("    const R* __restrict__ MU, const int* __restrict__ nbr, R* __restrict__ Tout, int K)")
    a_("{")
    a_("  constexpr bool ST = false;")
    a_(f"  __shared__ R wl[{lds_words(p)}];")
    _tile_prologue(a_)
    _elem_prologue(a_)
    _stage_field(a_, t, nw, "U", "MU")
    a_("  __syncthreads();")
    _trace_stage(a_, t, g, pl, nw, masked=True)
    a_("}")
    return "\n".join(L) + "\n"


def emit_batch(p: int) -> str:
    """Batched multi-mesh phase kernel of order p (FP32)."""
    t, _, _, g, Lp, nw, pl = _kernel_setup(p)
    L = []
    a_ = L.append
    _header(a_, p, t, nw, pl, "batched phase")
    a_("// One launch advances every slot (mesh) of this order.  Block b belongs to the last")
    a_("// slot s with tile0[s] <= b; blocks past the table, or of slots whose remaining")
    a_("// steps are exhausted at this sub-step, exit before any barrier.")
    a_("template <typename R, bool ST>")
    a_(f"__global__ void {_launch_bounds(p, nw)} dgm_phase_batch_p{p}(const BatchSlot* __restrict__ slots,")
    a_("    const int* __restrict__ tile0, const int* __restrict__ nslots, int phase, int substep)")
    a_("{")
    a_(f"  __shared__ R wl[{lds_words(p)}];")
    a_("  const int nsl = *nslots;")
    a_("  const int bid = blockIdx.x;")
    a_("  if (nsl <= 0 || bid >= tile0[nsl]) return;")
    a_("  int lo = 0, hi = nsl - 1;")
    a_("  while (lo < hi) { const int mid = (lo + hi + 1) >> 1; if (tile0[mid] <= bid) lo = mid; else hi = mid - 1; }")
    a_("  const BatchSlot sl = slots[lo];")
    a_("  if (substep >= sl.steps_left) return;")
    a_("  const R* __restrict__ U = (const R*)(phase ? sl.H : sl.E);")
    a_("  R* __restrict__ V = (R*)(phase ? sl.E : sl.H);")
    a_("  const R* __restrict__ MU = (const R*)(phase ? sl.MH : sl.ME);")
    a_("  const R* __restrict__ MV = (const R*)(phase ? sl.ME : sl.MH);")
    a_("  const R* __restrict__ Tin = (const R*)(phase ? sl.TH : sl.TE);")
    a_("  R* __restrict__ Tout = (R*)(phase ? sl.TE : sl.TH);")
    a_("  const int* __restrict__ nbr = sl.nbr;")
    a_("  const R sdt = (R)(phase ? sl.dt : -sl.dt);")
    a_("  const R wall = phase ? R(1) : R(-1);")
    a_("  const int K = sl.K;")
    a_("  constexpr bool STAB = false;  // batches use the central flux")
    a_("  constexpr bool RATE = false;  // batches update their fields")
    a_("  R* const HF = nullptr;")
    a_("  const R* const SC = nullptr;")
    a_("  const R fdt = R(0);")
    a_("  const int tile = bid - tile0[lo];")
    _elem_prologue(a_)
    _phase_body(a_, t, t, t, g, Lp, pl, nw)
    a_("}")
    return "\n".join(L) + "\n"


def _write_if_changed(path, src):
    old = open(path).read() if os.path.exists(path) else None
    if old != src:
        with open(path, "w") as fh:
            fh.write(src)
    return path


def emit_all(outdir: str, orders=range(1, TB.P_MAX + 1)):
    """Write one translation unit per order plus the shared frame constants.
    Returns the list of .hip translation units to compile."""
    os.makedirs(outdir, exist_ok=True)
    units = []
    for p in orders:
        nw = waves_for(p)
        assert lds_words(p) * 4 <= LDS_BUDGET, f"order {p}: LDS area too large"
        assert p > F64_MAX_ORDER or lds_words(p) * 8 <= LDS_BUDGET, f"order {p}: FP64 LDS area too large"
        _write_if_changed(os.path.join(outdir, f"phase_p{p}.inc"), emit_phase(p))
        _write_if_changed(os.path.join(outdir, f"batch_p{p}.inc"), emit_batch(p))
        tu = [f"// Generated by gen/emit.py: instantiation and launcher for order {p}.",
              "#include <hip/hip_runtime.h>",
              '#include "../launch.h"',
              f'#include "phase_p{p}.inc"',
              "template <typename R>",
              f"static hipError_t launch_p{p}(const PhaseArgs<R>& a) {{",
              "  if (a.overwrite && a.streaming)",
              f"    hipLaunchKernelGGL((dgm_phase_p{p}<R, true, false, true>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.U, a.V, a.MU, a.MV, a.nbr, a.Tin, a.Tout, a.sdt, a.wall, a.K, a.HF, a.SC, a.fdt);",
              "  else if (a.overwrite)",
              f"    hipLaunchKernelGGL((dgm_phase_p{p}<R, false, false, true>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.U, a.V, a.MU, a.MV, a.nbr, a.Tin, a.Tout, a.sdt, a.wall, a.K, a.HF, a.SC, a.fdt);",
              "  else if (a.HF && a.streaming)",
              f"    hipLaunchKernelGGL((dgm_phase_p{p}<R, true, true, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.U, a.V, a.MU, a.MV, a.nbr, a.Tin, a.Tout, a.sdt, a.wall, a.K, a.HF, a.SC, a.fdt);",
              "  else if (a.HF)",
              f"    hipLaunchKernelGGL((dgm_phase_p{p}<R, false, true, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.U, a.V, a.MU, a.MV, a.nbr, a.Tin, a.Tout, a.sdt, a.wall, a.K, a.HF, a.SC, a.fdt);",
              "  else if (a.streaming)",
              f"    hipLaunchKernelGGL((dgm_phase_p{p}<R, true, false, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.U, a.V, a.MU, a.MV, a.nbr, a.Tin, a.Tout, a.sdt, a.wall, a.K, a.HF, a.SC, a.fdt);",
              "  else",
              f"    hipLaunchKernelGGL((dgm_phase_p{p}<R, false, false, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.U, a.V, a.MU, a.MV, a.nbr, a.Tin, a.Tout, a.sdt, a.wall, a.K, a.HF, a.SC, a.fdt);",
              "  return hipGetLastError();",
              "}",
              f"hipError_t dgm_launch_phase_p{p}_f32(const PhaseArgs<float>& a) {{ return launch_p{p}<float>(a); }}"]
        if p <= F64_MAX_ORDER:
            tu.append(f"hipError_t dgm_launch_phase_p{p}_f64(const PhaseArgs<double>& a) {{ return launch_p{p}<double>(a); }}")
        units.append(_write_if_changed(os.path.join(outdir, f"phase_p{p}.hip"), "\n".join(tu) + "\n"))
        _write_if_changed(os.path.join(outdir, f"trace_p{p}.inc"), emit_trace(p))
        tt = [f"// Generated by gen/emit.py: trace kernel instantiation and launcher for order {p}.",
              "#include <hip/hip_runtime.h>",
              '#include "../launch.h"',
              f'#include "trace_p{p}.inc"',
              "template <typename R>",
              f"static hipError_t launch_trace_p{p}(const TraceArgs<R>& a) {{",
              f"  hipLaunchKernelGGL(dgm_trace_p{p}<R>, dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.U, a.MU, a.nbr, a.T, a.K);",
              "  return hipGetLastError();",
              "}",
              f"hipError_t dgm_launch_trace_p{p}_f32(const TraceArgs<float>& a) {{ return launch_trace_p{p}<float>(a); }}"]
        if p <= F64_MAX_ORDER:
            tt.append(f"hipError_t dgm_launch_trace_p{p}_f64(const TraceArgs<double>& a) {{ return launch_trace_p{p}<double>(a); }}")
        units.append(_write_if_changed(os.path.join(outdir, f"trace_p{p}.hip"), "\n".join(tt) + "\n"))
        tb = [f"// Generated by gen/emit.py: batched launcher for order {p}.",
              "#include <hip/hip_runtime.h>",
              '#include "../launch.h"',
              f'#include "batch_p{p}.inc"',
              f"hipError_t dgm_launch_batch_p{p}_f32(const BatchArgs& a) {{",
              "  if (a.streaming)",
              f"    hipLaunchKernelGGL((dgm_phase_batch_p{p}<float, true>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.slots, a.tile0, a.nslots, a.phase, a.substep);",
              "  else",
              f"    hipLaunchKernelGGL((dgm_phase_batch_p{p}<float, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, a.slots, a.tile0, a.nslots, a.phase, a.substep);",
              "  return hipGetLastError();",
              "}"]
        units.append(_write_if_changed(os.path.join(outdir, f"batch_p{p}.hip"), "\n".join(tb) + "\n"))
        if p + 1 in orders:
            units.append(_emit_mixed(outdir, p))
        _write_if_changed(os.path.join(outdir, f"mass_p{p}.inc"), MS.emit_mass(p))
        units.append(_write_if_changed(os.path.join(outdir, f"mass_p{p}.hip"), MS.emit_unit(p, p <= F64_MAX_ORDER)))
    fr = TB.frame()
    A, Ai = fr["A"], fr["Ainv"]
    lines = ["// Generated by gen/emit.py: derivative frame and compiled orders.",
             f"#define DGM_MAX_ORDER_F32 {max(orders)}",
             f"#define DGM_MAX_ORDER_F64 {max([p for p in orders if p <= F64_MAX_ORDER], default=0)}",
             "static const double kFrameA[9] = {" + ", ".join(float(v).hex() for v in A.ravel()) + "};",
             "static const double kFrameAinv[9] = {" + ", ".join(float(v).hex() for v in Ai.ravel()) + "};",
             f"static const double kFrameDetA = {float(fr['detA']).hex()};"]
    decl = []
    for p in orders:
        decl.append(f"hipError_t dgm_launch_phase_p{p}_f32(const PhaseArgs<float>& a);")
        if p <= F64_MAX_ORDER:
            decl.append(f"hipError_t dgm_launch_phase_p{p}_f64(const PhaseArgs<double>& a);")
    for p in orders:
        decl.append(f"hipError_t dgm_launch_trace_p{p}_f32(const TraceArgs<float>& a);")
        if p <= F64_MAX_ORDER:
            decl.append(f"hipError_t dgm_launch_trace_p{p}_f64(const TraceArgs<double>& a);")
    lines += decl
    for p in orders:
        lines.append(f"hipError_t dgm_launch_mass_p{p}_f32(const MassArgs<float>& a);")
        if p <= F64_MAX_ORDER:
            lines.append(f"hipError_t dgm_launch_mass_p{p}_f64(const MassArgs<double>& a);")
    for p in orders:
        lines.append(f"hipError_t dgm_launch_batch_p{p}_f32(const BatchArgs& a);")
        if p + 1 in orders:
            lines.append(f"hipError_t dgm_launch_mix_p{p}_f32(const PhaseArgs<float>& a, int dir);")
            if p + 1 <= F64_MAX_ORDER:
                lines.append(f"hipError_t dgm_launch_mix_p{p}_f64(const PhaseArgs<double>& a, int dir);")
    lines += launcher_tables(orders)
    _write_if_changed(os.path.join(outdir, "frame.inc"), "\n".join(lines) + "\n")
    _write_if_changed(os.path.join(outdir, "tables.inc"), emit_host_tables(orders))
    import json

    _write_if_changed(os.path.join(outdir, "opcount.json"), json.dumps(
        {"note": "floating-point operations (multiply and add; an FMA counts two) per element and phase "
                 "launch as emitted: no_traces (rate only), with_traces (the step's phase: also the traces of "
                 "the updated field), trace_stage_recomputed_faces (part of the trace stage that runs only "
                 "in tiles with an off-tile neighbour across the x = 0 or y = 0 face)",
         "orders": {str(p): OPCOUNT[p] for p in orders}}, indent=1) + "\n")
    return units


def _emit_mixed(outdir, p):
    """Mixed-order kernels of the pair (E of order p + 1, H of order p): dgm_phase_eh_p{p}
    updates H from E, dgm_phase_he_p{p} updates E from H; one launcher picks by direction."""
    nw = waves_for(p + 1)
    src = (emit_phase(p, p + 1, p, f"dgm_phase_eh_p{p}") + emit_phase(p, p, p + 1, f"dgm_phase_he_p{p}"))
    _write_if_changed(os.path.join(outdir, f"mix_p{p}.inc"), src)
    args = "a.U, a.V, a.MU, a.MV, a.nbr, a.Tin, a.Tout, a.sdt, a.wall, a.K, a.HF, a.SC, a.fdt"
    tu = [f"// Generated by gen/emit.py: mixed-order kernels (E of order {p + 1}, H of order {p}) and launcher.",
          "#include <hip/hip_runtime.h>",
          '#include "../launch.h"',
          f'#include "mix_p{p}.inc"',
          "// dir 0: H update from E (U = E of order p + 1, V = H); 1: E update from H",
          "template <typename R>",
          f"static hipError_t launch_mix_p{p}(const PhaseArgs<R>& a, int dir) {{",
          "  if (dir == 0 && a.streaming)",
          f"    hipLaunchKernelGGL((dgm_phase_eh_p{p}<R, true, false, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, {args});",
          "  else if (dir == 0)",
          f"    hipLaunchKernelGGL((dgm_phase_eh_p{p}<R, false, false, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, {args});",
          "  else if (a.streaming)",
          f"    hipLaunchKernelGGL((dgm_phase_he_p{p}<R, true, false, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, {args});",
          "  else",
          f"    hipLaunchKernelGGL((dgm_phase_he_p{p}<R, false, false, false>), dim3(a.blocks), dim3({nw * LANES}), 0, a.stream, {args});",
          "  return hipGetLastError();",
          "}",
          f"hipError_t dgm_launch_mix_p{p}_f32(const PhaseArgs<float>& a, int dir) {{ return launch_mix_p{p}<float>(a, dir); }}"]
    if p + 1 <= F64_MAX_ORDER:
        tu.append(f"hipError_t dgm_launch_mix_p{p}_f64(const PhaseArgs<double>& a, int dir) {{ return launch_mix_p{p}<double>(a, dir); }}")
    return _write_if_changed(os.path.join(outdir, f"mix_p{p}.hip"), "\n".join(tu) + "\n")


def launcher_tables(orders):
    """Launcher tables indexed by order: entry p is the launcher of order p, nullptr
    where order p was not built (or is not instantiated for that precision).  Every
    table has DGM_MAX_ORDER_F32 + 1 entries, so the host may index it by any order
    up to that bound and must check the entry before calling it."""
    top = max(orders)

    def table(decl, name, present):
        ents = ", ".join(name.format(p=p) if (p in orders and present(p)) else "nullptr" for p in range(top + 1))
        return f"static {decl.format(n=top + 1)} = {{{ents}}};"

    f64 = lambda p: p <= F64_MAX_ORDER
    mix = lambda p: p + 1 in orders
    return [
        table("hipError_t (*const kMixF32[{n}])(const PhaseArgs<float>&, int)", "dgm_launch_mix_p{p}_f32", mix),
        table("hipError_t (*const kMixF64[{n}])(const PhaseArgs<double>&, int)", "dgm_launch_mix_p{p}_f64",
              lambda p: mix(p) and p + 1 <= F64_MAX_ORDER),
        table("hipError_t (*const kTraceF32[{n}])(const TraceArgs<float>&)", "dgm_launch_trace_p{p}_f32", lambda p: True),
        table("hipError_t (*const kTraceF64[{n}])(const TraceArgs<double>&)", "dgm_launch_trace_p{p}_f64", f64),
        table("hipError_t (*const kPhaseF32[{n}])(const PhaseArgs<float>&)", "dgm_launch_phase_p{p}_f32", lambda p: True),
        table("hipError_t (*const kPhaseF64[{n}])(const PhaseArgs<double>&)", "dgm_launch_phase_p{p}_f64", f64),
        table("hipError_t (*const kBatchF32[{n}])(const BatchArgs&)", "dgm_launch_batch_p{p}_f32", lambda p: True),
        table("hipError_t (*const kMassF32[{n}])(const MassArgs<float>&)", "dgm_launch_mass_p{p}_f32", lambda p: True),
        table("hipError_t (*const kMassF64[{n}])(const MassArgs<double>&)", "dgm_launch_mass_p{p}_f64", f64),
    ]


def emit_host_tables(orders):
    """Sparse reference tables for the host (dense-operator assembly at set-up):
    per order the derivative operators D0..D2 and trace operators T0..T3 as
    (row, col, value) triplets, the tangential weights g[f][k] and the stored-frame
    lift weights Lp[f][k][s]."""
    L = ["// Generated by gen/emit.py: sparse reference tables for host-side assembly.",
         "struct SparseEntry { short r, c; double v; };",
         "struct OrderTables { int N, NF; const SparseEntry* D[3]; int nD[3]; const SparseEntry* T[4]; int nT[4];",
         "                     double g[4][2][3]; double Lp[4][3][2]; };"]
    for p in orders:
        t = TB.build(p)
        g, Lp = TB.face_weights(t)
        for d in range(3):
            r, c = np.nonzero(t.D[d])
            L.append(f"static const SparseEntry kD{d}_p{p}[] = {{" + ", ".join(f"{{{i},{j},{float(t.D[d][i, j]).hex()}}}" for i, j in zip(r, c)) + "};")
        for f in range(4):
            r, c = np.nonzero(t.T[f])
            L.append(f"static const SparseEntry kT{f}_p{p}[] = {{" + ", ".join(f"{{{i},{j},{float(t.T[f][i, j]).hex()}}}" for i, j in zip(r, c)) + "};")
    empty = "  {0, 0, {nullptr, nullptr, nullptr}, {0, 0, 0}, {nullptr, nullptr, nullptr, nullptr}, {0, 0, 0, 0}, {}, {}},"
    L.append("// indexed by order; N = 0 marks an order that was not built")
    L.append(f"static const OrderTables kTables[{max(orders) + 1}] = {{")
    for p in range(max(orders) + 1):
        if p not in orders:
            L.append(empty)
            continue
        t = TB.build(p)
        g, Lp = TB.face_weights(t)
        nD = [int(np.count_nonzero(t.D[d])) for d in range(3)]
        nT = [int(np.count_nonzero(t.T[f])) for f in range(4)]
        gs = "{" + ", ".join("{" + ", ".join("{" + ", ".join(float(v).hex() for v in g[f][k]) + "}" for k in range(2)) + "}" for f in range(4)) + "}"
        ls = "{" + ", ".join("{" + ", ".join("{" + ", ".join(float(v).hex() for v in Lp[f][k]) + "}" for k in range(3)) + "}" for f in range(4)) + "}"
        L.append(f"  {{{t.N}, {t.NF}, {{kD0_p{p}, kD1_p{p}, kD2_p{p}}}, {{{nD[0]}, {nD[1]}, {nD[2]}}}, "
                 f"{{kT0_p{p}, kT1_p{p}, kT2_p{p}, kT3_p{p}}}, {{{nT[0]}, {nT[1]}, {nT[2]}, {nT[3]}}}, {gs}, {ls}}},")
    L.append("};")
    return "\n".join(L) + "\n"
