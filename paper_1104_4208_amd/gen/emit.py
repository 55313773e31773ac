"""Emit the per-order HIP phase kernels as straight-line code.

Section 3.2.2 describes the reference implementation as C++ template
meta-programming that generates optimised code for every order up to an
a-priori maximum.  This module plays that role for CDNA4: for each order p
it writes one kernel body in which every sparse operator entry of
gen/tables.py is an FMA with a literal coefficient, so the 64 lanes of a
wavefront (one element per lane) run an identical, branch-free instruction
stream with all data in registers.

Kernel contract (one leapfrog half step, "phase"):
  U  (3,N,K)  stored-frame coefficients of the field that is differentiated
  V  (3,N,K)  stored-frame coefficients of the field that is updated, in place
  MU (6,K)    symmetric conversion w = MU S (derivative frame) for U
  nbr(4,K)    neighbour code nb*4 + local face of nb, or -1 on a wall
  sdt         -dt for the H update, +dt for the E update
  wall        ghost factor on walls: the jump is (wall-1) * own trace
              (E_nb = -E gives wall = -1; H_nb = H gives wall = +1)
  V_k += sdt * ( c_k + sum_f T_f^T ( Lp_f[k,0] dtau_f0 + Lp_f[k,1] dtau_f1 ) )
where dtau_fk = tau_fk(neighbour) - tau_fk(own) are the jumps of the two
tangential traces (u . t1, u . t2) of face f, which both sides compute in the
same (s,t) parametrisation because vertices are sorted by global id.
"""
from __future__ import annotations

import os

import numpy as np

from . import tables as TB


def _lit(v: float) -> str:
    """Exact literal of an FP64 table entry, rounded once to the kernel's type R."""
    if v == 1.0:
        return "R(1)"
    if v == -1.0:
        return "R(-1)"
    return f"R({float(v).hex()})"


def _fma(acc, coef, x):
    if coef == 1.0:
        return f"{acc} += {x};"
    if coef == -1.0:
        return f"{acc} -= {x};"
    return f"{acc} += {_lit(coef)} * {x};"


def _dot(gv, w, name):
    terms = []
    for c, x in zip(gv, w):
        if c == 0.0:
            continue
        if c == 1.0:
            terms.append(x)
        elif c == -1.0:
            terms.append(f"-{x}")
        else:
            terms.append(f"{_lit(c)} * {x}")
    return f"const R {name} = {' + '.join(terms) if terms else 'R(0)'};"


WAVES = 4
LANES = 64


def _chunks(items, costs, max_cost):
    """Split an ordered list into consecutive chunks whose summed cost stays <= max_cost."""
    out, cur, c = [], [], 0
    for it, w in zip(items, costs):
        if cur and c + w > max_cost:
            out.append(cur)
            cur, c = [], 0
        cur.append(it)
        c += w
    if cur:
        out.append(cur)
    return out


def _assign(jobs, costs, nw):
    """Longest-processing-time assignment of jobs to nw waves; returns per-wave job lists."""
    order = sorted(range(len(jobs)), key=lambda i: -costs[i])
    load = [0] * nw
    out = [[] for _ in range(nw)]
    for i in order:
        w = min(range(nw), key=lambda k: load[k])
        out[w].append(jobs[i])
        load[w] += costs[i]
    return out, load


def plan(p: int, nw: int = WAVES):
    """Split the work of one phase into trace jobs (face f, face rows) and output jobs
    (component k, volume rows), balanced over nw waves by FMA count."""
    t = TB.build(p)
    N, NF = t.N, t.NF
    g, Lp = TB.face_weights(t)
    # trace jobs: cost = own trace + worst neighbour trace of those rows (2 scalars each)
    tr_items, tr_cost = [], []
    for f in range(4):
        rows = list(range(NF))
        rc = [2 * (np.count_nonzero(t.T[f][m]) + max(np.count_nonzero(t.T[h][m]) for h in range(4))) for m in rows]
        tot = sum(2 * (np.count_nonzero(t.T[ff]) * 2) for ff in range(4))
        for ch in _chunks(rows, rc, max(1, tot // (2 * nw))):
            tr_items.append((f, ch))
            tr_cost.append(sum(rc[m] for m in ch))
    cyc = {0: (1, 2), 1: (2, 0), 2: (0, 1)}
    out_items, out_cost = [], []
    for k in range(3):
        i, j = cyc[k]
        rows = list(range(N))
        rc = []
        for b in rows:
            c = np.count_nonzero(t.D[i][b]) + np.count_nonzero(t.D[j][b])
            for f in range(4):
                if np.any(Lp[f][k] != 0):
                    c += np.count_nonzero(t.T[f][:, b])
            rc.append(c + 1)
        tot = sum(rc)
        for ch in _chunks(rows, rc, max(1, -(-tot // nw))):
            out_items.append((k, ch))
            out_cost.append(sum(rc[b] for b in ch))
    tr_w, tr_load = _assign(tr_items, tr_cost, nw)
    out_w, out_load = _assign(out_items, out_cost, nw)
    return dict(trace=tr_w, trace_load=tr_load, out=out_w, out_load=out_load)


def _self_trace(a_, t, g, f, rows, ind):
    """Own tangential traces of face f, face rows `rows`, into ts{k}_{m}."""
    N = t.N
    a_(ind + "R " + ", ".join(f"ts{k}_{m} = R(0)" for m in rows for k in range(2)) + ";")
    a_(ind + "{ const R* Ul = U; asm volatile(\"\" : \"+s\"(Ul));")
    for a in range(N):
        ms = [m for m in rows if t.T[f][m, a] != 0]
        if not ms:
            continue
        a_(ind + "  {")
        a_(ind + f"    const R s0 = Ul[({a}) * Ks + el], s1 = Ul[({N + a}) * Ks + el], s2 = Ul[({2 * N + a}) * Ks + el];")
        a_(ind + "    const R w0 = m00 * s0 + m01 * s1 + m02 * s2;")
        a_(ind + "    const R w1 = m01 * s0 + m11 * s1 + m12 * s2;")
        a_(ind + "    const R w2 = m02 * s0 + m12 * s1 + m22 * s2;")
        for k in range(2):
            a_(ind + "    " + _dot(g[f][k], ["w0", "w1", "w2"], f"q{k}"))
        for m in ms:
            for k in range(2):
                a_(ind + "    " + _fma(f"ts{k}_{m}", t.T[f][m, a], f"q{k}"))
        a_(ind + "  }")
    a_(ind + "}")


def _nb_trace(a_, t, g, f, rows, ind):
    """Neighbour tangential traces on face f (neighbour's own face code & 3) minus own,
    stored to the jump buffer in LDS."""
    N, NF = t.N, t.NF
    a_(ind + "{")
    a_(ind + f"  const int code = nbr[{f} * Ks + el];")
    a_(ind + "  if (code < 0) {")
    for m in rows:
        for k in range(2):
            a_(ind + f"    ts{k}_{m} = (wall - R(1)) * ts{k}_{m};")
    a_(ind + "  } else {")
    a_(ind + "    const size_t nb = (size_t)(code >> 2);")
    a_(ind + "    const R n00 = MU[0 * Ks + nb], n01 = MU[1 * Ks + nb], n02 = MU[2 * Ks + nb];")
    a_(ind + "    const R n11 = MU[3 * Ks + nb], n12 = MU[4 * Ks + nb], n22 = MU[5 * Ks + nb];")
    a_(ind + "    R " + ", ".join(f"tn{k}_{m} = R(0)" for m in rows for k in range(2)) + ";")
    a_(ind + "    switch (code & 3) {")
    for gf in range(4):
        a_(ind + f"    case {gf}: {{")
        for a in range(N):
            ms = [m for m in rows if t.T[gf][m, a] != 0]
            if not ms:
                continue
            a_(ind + "      {")
            a_(ind + f"        const R s0 = U[({a}) * Ks + nb], s1 = U[({N + a}) * Ks + nb], s2 = U[({2 * N + a}) * Ks + nb];")
            a_(ind + "        const R w0 = n00 * s0 + n01 * s1 + n02 * s2;")
            a_(ind + "        const R w1 = n01 * s0 + n11 * s1 + n12 * s2;")
            a_(ind + "        const R w2 = n02 * s0 + n12 * s1 + n22 * s2;")
            for k in range(2):
                a_(ind + "        " + _dot(g[gf][k], ["w0", "w1", "w2"], f"q{k}"))
            for m in ms:
                for k in range(2):
                    a_(ind + "        " + _fma(f"tn{k}_{m}", t.T[gf][m, a], f"q{k}"))
            a_(ind + "      }")
        a_(ind + "      break;")
        a_(ind + "    }")
    a_(ind + "    }")
    for m in rows:
        for k in range(2):
            a_(ind + f"    ts{k}_{m} = tn{k}_{m} - ts{k}_{m};")
    a_(ind + "  }")
    for m in rows:
        for k in range(2):
            a_(ind + f"  jmp[({(f * 2 + k) * NF + m}) * {LANES} + lane] = ts{k}_{m};")
    a_(ind + "}")


def _output(a_, t, Lp, k, rows, ind):
    """Component k of the update for volume rows `rows`: curl in the derivative frame
    plus the lifted face jumps read back from LDS."""
    N, NF = t.N, t.NF
    cyc = {0: (1, 2), 1: (2, 0), 2: (0, 1)}
    i, j = cyc[k]
    Mi = {0: "m00 * s0 + m01 * s1 + m02 * s2", 1: "m01 * s0 + m11 * s1 + m12 * s2", 2: "m02 * s0 + m12 * s1 + m22 * s2"}
    rs = set(rows)
    a_(ind + "{")
    a_(ind + "  R " + ", ".join(f"acc{b} = R(0)" for b in rows) + ";")
    a_(ind + "  { const R* Ul = U; asm volatile(\"\" : \"+s\"(Ul));")
    for a in range(N):
        ri = [b for b in rows if t.D[i][b, a] != 0]
        rj = [b for b in rows if t.D[j][b, a] != 0]
        if not ri and not rj:
            continue
        a_(ind + "    {")
        a_(ind + f"      const R s0 = Ul[({a}) * Ks + el], s1 = Ul[({N + a}) * Ks + el], s2 = Ul[({2 * N + a}) * Ks + el];")
        if ri:
            a_(ind + f"      const R wj = {Mi[j]};")
        if rj:
            a_(ind + f"      const R wi = {Mi[i]};")
        for b in ri:
            a_(ind + "      " + _fma(f"acc{b}", t.D[i][b, a], "wj"))
        for b in rj:
            a_(ind + "      " + _fma(f"acc{b}", -t.D[j][b, a], "wi"))
        a_(ind + "    }")
    a_(ind + "  }")
    for f in range(4):
        c0, c1 = Lp[f][k]
        if c0 == 0.0 and c1 == 0.0:
            continue
        for m in range(NF):
            bs = [b for b in rows if t.T[f][m, b] != 0]
            if not bs:
                continue
            terms = []
            if c0 != 0.0:
                terms.append(f"{_lit(c0)} * jmp[({(f * 2 + 0) * NF + m}) * {LANES} + lane]")
            if c1 != 0.0:
                terms.append(f"{_lit(c1)} * jmp[({(f * 2 + 1) * NF + m}) * {LANES} + lane]")
            a_(ind + "  {")
            a_(ind + f"    const R gf = {' + '.join(terms)};")
            for b in bs:
                a_(ind + "    " + _fma(f"acc{b}", t.T[f][m, b], "gf"))
            a_(ind + "  }")
    a_(ind + "  if (act) {")
    for b in rows:
        a_(ind + f"    V[({k * N + b}) * Ks + e] += sdt * acc{b};")
    a_(ind + "  }")
    a_(ind + "}")


def emit_phase(p: int, nw: int = WAVES) -> str:
    t = TB.build(p)
    N, NF = t.N, t.NF
    g, Lp = TB.face_weights(t)
    pl = plan(p, nw)
    L = []
    a_ = L.append
    a_(f"// Generated by gen/emit.py for order p = {p}: N = {N} volume modes, NF = {NF} face modes.")
    a_(f"// {nw} waves share {LANES} elements (one per lane); trace FMA load per wave {pl['trace_load']},")
    a_(f"// output FMA load per wave {pl['out_load']}.")
    a_(f"static constexpr int kJumpSlots_p{p} = {8 * NF};")
    a_("template <typename R>")
    a_(f"__global__ void __launch_bounds__({nw * LANES}) dgm_phase_p{p}(const R* __restrict__ U, R* __restrict__ V,")
    a_("    const R* __restrict__ MU, const int* __restrict__ nbr, R sdt, R wall, int K)")
    a_("{")
    a_(f"  __shared__ R jmp[{8 * NF * LANES}];")
    a_(f"  const int lane = threadIdx.x & {LANES - 1};")
    a_(f"  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);")
    a_("  // XCD-aware tile order: block b runs on XCD b % 8, so give every XCD a")
    a_("  // contiguous range of element tiles and keep neighbour data in its L2")
    a_("  const int nbk = gridDim.x, bid = blockIdx.x;")
    a_("  const int per = nbk >> 3, rem = nbk & 7, xcd = bid & 7;")
    a_("  const int tile = xcd * per + (xcd < rem ? xcd : rem) + (bid >> 3);")
    a_(f"  const int e = tile * {LANES} + lane;")
    a_("  const bool act = e < K;")
    a_("  const int el = act ? e : K - 1;")
    a_("  const size_t Ks = (size_t)K;")
    a_("  const R m00 = MU[0 * Ks + el], m01 = MU[1 * Ks + el], m02 = MU[2 * Ks + el];")
    a_("  const R m11 = MU[3 * Ks + el], m12 = MU[4 * Ks + el], m22 = MU[5 * Ks + el];")
    a_("  // stage 1: jumps of the tangential traces (neighbour minus own) into LDS")
    for w in range(nw):
        a_(f"  if (wave == {w}) {{")
        for (f, rows) in pl["trace"][w]:
            a_(f"    // face {f}, face modes {rows[0]}..{rows[-1]}")
            a_("    {")
            _self_trace(a_, t, g, f, rows, "      ")
            _nb_trace(a_, t, g, f, rows, "      ")
            a_("    }")
        a_("  }")
    a_("  __syncthreads();")
    a_("  // stage 2: curl and lifted jumps, component-separable update")
    for w in range(nw):
        a_(f"  if (wave == {w}) {{")
        for (k, rows) in pl["out"][w]:
            a_(f"    // component {k}, volume modes {rows[0]}..{rows[-1]}")
            _output(a_, t, Lp, k, rows, "    ")
        a_("  }")
    a_("}")
    return "\n".join(L) + "\n"


F64_MAX_ORDER = 6


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
        _write_if_changed(os.path.join(outdir, f"phase_p{p}.inc"), emit_phase(p))
        tu = [f"// Generated by gen/emit.py: instantiation and launcher for order {p}.",
              "#include <hip/hip_runtime.h>",
              '#include "../launch.h"',
              f'#include "phase_p{p}.inc"',
              "template <typename R>",
              f"static hipError_t launch_p{p}(const PhaseArgs<R>& a) {{",
              f"  hipLaunchKernelGGL(dgm_phase_p{p}<R>, dim3(a.blocks), dim3({WAVES * LANES}), 0, a.stream, a.U, a.V, a.MU, a.nbr, a.sdt, a.wall, a.K);",
              "  return hipGetLastError();",
              "}",
              f"hipError_t dgm_launch_phase_p{p}_f32(const PhaseArgs<float>& a) {{ return launch_p{p}<float>(a); }}"]
        if p <= F64_MAX_ORDER:
            tu.append(f"hipError_t dgm_launch_phase_p{p}_f64(const PhaseArgs<double>& a) {{ return launch_p{p}<double>(a); }}")
        units.append(_write_if_changed(os.path.join(outdir, f"phase_p{p}.hip"), "\n".join(tu) + "\n"))
    fr = TB.frame()
    A, Ai = fr["A"], fr["Ainv"]
    lines = ["// Generated by gen/emit.py: derivative frame and compiled orders.",
             f"#define DGM_MAX_ORDER_F32 {max(orders)}",
             f"#define DGM_MAX_ORDER_F64 {min(max(orders), F64_MAX_ORDER)}",
             "static const double kFrameA[9] = {" + ", ".join(float(v).hex() for v in A.ravel()) + "};",
             "static const double kFrameAinv[9] = {" + ", ".join(float(v).hex() for v in Ai.ravel()) + "};",
             f"static const double kFrameDetA = {float(fr['detA']).hex()};"]
    decl = []
    for p in orders:
        decl.append(f"hipError_t dgm_launch_phase_p{p}_f32(const PhaseArgs<float>& a);")
        if p <= F64_MAX_ORDER:
            decl.append(f"hipError_t dgm_launch_phase_p{p}_f64(const PhaseArgs<double>& a);")
    lines += decl
    lines.append("static hipError_t (*const kPhaseF32[])(const PhaseArgs<float>&) = {nullptr, " + ", ".join(f"dgm_launch_phase_p{p}_f32" for p in orders) + "};")
    lines.append("static hipError_t (*const kPhaseF64[])(const PhaseArgs<double>&) = {nullptr, " + ", ".join(f"dgm_launch_phase_p{p}_f64" for p in orders if p <= F64_MAX_ORDER) + "};")
    _write_if_changed(os.path.join(outdir, "frame.inc"), "\n".join(lines) + "\n")
    return units
