"""Emit the approximate mass-inverse kernels (Section 3.3.2) as straight-line code.

With a material that varies inside an element the mass matrix is no longer the flat
one, and its inverse is replaced by the approximate inverse of Section 3.3.2: the
point values of a rate at the points of a quadrature rule (the reverse of numerical
integration), divided by the material there, integrated back.  On the collapsed Gauss
rule with q = p + 1 points per direction and the orthonormal basis this is the
scalar operator, applied to every Cartesian (or covariant, or stored-frame)
component alike:

    (P r)_a = sum_x w_x phi_a(x) (sum_b phi_b(x) r_b) / m(x)

with m the material, linear on the element, from its values at the four vertices
(sorted by global vertex id, the element's reference map).  P commutes with the
per-element 3x3 frame maps, so the kernel applies it to whatever frame its input is in.

Sum factorisation (tables.mass_factors): phi_ijk(a, b, c) = C1[ijk, a] Fb[i, j, b] Fc[i, c]
in the collapsed coordinates, so the evaluation runs over k, then j, then i, and the
integration back over i, j, k; every step is done one a-slice of the points at a
time, which keeps q^2 values of the slice in registers.  O(p^4) multiply-adds per
component instead of the O(p^6) of a dense point matrix.

Layout and parallelism: a workgroup takes one component of a tile of 64 elements (one
per lane, so field loads and stores are coalesced as in the phase kernels) with one
wave per a-slice of the points.  The slice index is uniform in a wave, so the k-step and
its transpose, whose coefficients depend on the slice, are literal code in a switch on it;
the j- and c-steps have literal coefficients shared by all waves.  The tile's input column
is staged in LDS and read by every wave for the k-step; the LDS then holds the slices'
results h_ij(a) of the steps back, in sets of pairs (i, j) small enough for three
workgroups per CU, and for each set the waves share its rows for the k-step back over
the q slices.  The Legendre c-step uses the mirror symmetry of the Gauss-Legendre nodes
(even and odd degrees summed once for two nodes).  A lane holds about eighty values at
p = 6, so several workgroups share a CU and their loads, arithmetic and stores overlap.
"""
from __future__ import annotations

import numpy as np

from . import tables as TB

LANES = 64
LDS_SET_BYTES = 53248  # LDS per set of h: three workgroups per CU


def _h(v):
    return float(v).hex()


def _rules(q):
    from scipy.special import roots_jacobi

    xa, wa = roots_jacobi(q, 2, 0)
    xb, wb = roots_jacobi(q, 1, 0)
    xc, wc = roots_jacobi(q, 0, 0)
    # Gauss-Legendre: nodes and weights mirror about 0 (the even/odd split relies on it)
    assert np.abs(xc + xc[::-1]).max() < 1e-14 and np.abs(wc - wc[::-1]).max() < 1e-14
    return xa, wa, xb, wb, xc, wc


def _column_cost(p, q):
    """Multiply-adds of the c-step and its transpose on one b-column (even/odd split)."""
    h = q // 2
    ne, no = (p + 2) // 2, (p + 1) // 2  # even and odd Legendre degrees 0..p
    fwd = h * (p + 1) + 2 * h + (ne if q % 2 else 0)
    back = 2 * h + (p + 1) * h + (ne if q % 2 else 0)
    return fwd + back


def mass_cost(p: int) -> dict:
    """Floating-point operations per element (3 components) of one application: every
    multiply-add of the k-, j- and c-steps and their transposes counts two, and so do the
    adds of the even/odd split (a slight overcount); the point scale counts three per point
    (material, reciprocal, product) and the column bases four per column."""
    t = TB.build(p)
    q = p + 1
    npairs = (p + 1) * (p + 2) // 2
    per_slice_fma = 2 * t.N + 2 * npairs * q  # k-step, j-step and their transposes
    per_slice = 2 * per_slice_fma + 2 * q * _column_cost(p, q) + 3 * q * q + 4 * q  # + point scale, column bases
    flops = 3 * (q * per_slice + 2 * t.N)  # + V = V + s out
    return dict(flops=int(flops))


def emit_mass(p: int) -> str:
    t = TB.build(p)
    f = TB.mass_factors(p)
    q, C1, Fb, Fc = f["q"], f["C1"], f["Fb"], f["Fc"]
    N = t.N
    xa, wa, xb, wb, xc, wc = _rules(q)
    h = q // 2
    mid = h if q % 2 else None
    for i in range(p + 1):
        assert np.abs(Fc[i, ::-1] - (-1) ** i * Fc[i]).max() < 1e-13
        if mid is not None and i % 2:
            assert abs(Fc[i, mid]) < 1e-14
    pairs = [(i, j) for i in range(p + 1) for j in range(p + 1 - i)]
    pidx = {ij: n for n, ij in enumerate(pairs)}
    NP = len(pairs)
    modes_of = {ij: [] for ij in pairs}
    for r, (i, j, k) in enumerate(t.modes):
        modes_of[(i, j)].append(r)
    nthreads = q * LANES
    # the slices' h_ij pass through LDS in sets of pairs small enough for three workgroups
    # per CU (FP32); the rows of each set are split among the waves
    nsets = -(-NP * q * LANES * 4 // LDS_SET_BYTES)
    per = -(-NP // nsets)
    sets = [list(range(k * per, min(NP, (k + 1) * per))) for k in range(nsets)]
    set_rows = [[r for r, (i, j, k) in enumerate(t.modes) if pidx[(i, j)] in st] for st in sets]
    wave_rows = [[[r for n, r in enumerate(rs) if n % q == w] for w in range(q)] for rs in set_rows]
    nvo = max(sum(len(wave_rows[k][w]) for k in range(nsets)) for w in range(q))
    lds = max(N, per * q) * LANES
    L = []
    a_ = L.append
    a_(f"// Generated by gen/emit.py (gen/mass.py) for order p = {p}: N = {N} modes, {q}^3 collapsed Gauss points.")
    a_("// Approximate mass inverse (Section 3.3.2):")
    a_("//   V[c] = (acc ? V[c] : 0) + s * P X[c],  (P r)_a = sum_x w_x phi_a(x) (sum_b phi_b(x) r_b) / m(x),")
    a_("// m linear on the element from mat[v * K + e], v = 0..3 its sorted vertices.")
    a_(f"// Workgroup: one component c of a tile of {LANES} elements (one per lane), {q} waves; wave w")
    a_(f"// takes the a-slice w of the points: the k-, j- and c-steps of the evaluation, the point")
    a_(f"// scale and the c- and j-steps back, giving h_ij(a_w) ({NP} values), which pass through LDS")
    a_(f"// in {nsets} set(s) of pairs; for each set the waves finish its rows by the k-step back over")
    a_(f"// the {q} slices.  Per-slice coefficients are literals in a switch on the uniform w.")
    a_("#ifndef DGM_MASS_RCP")
    a_("#define DGM_MASS_RCP")
    a_("template <typename R>")
    a_("__device__ inline R mass_rcp(R x) {")
    a_("  if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);")
    a_("  else return R(1) / x;")
    a_("}")
    a_("#endif")
    a_("template <typename R>")
    a_(f"__global__ void __launch_bounds__({nthreads}) dgm_mass_p{p}(const R* __restrict__ X, R* __restrict__ V,")
    a_("    const R* __restrict__ mat, R s, int acc, int K)")
    a_("{")
    a_(f"  // the input column ({N} x {LANES}) until every wave has read it, then one set of h_ij(a)")
    a_(f"  __shared__ R sh[{lds}];")
    a_(f"  const int lane = threadIdx.x & {LANES - 1};")
    a_("  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);")
    a_("  const int c = blockIdx.x % 3, tile = blockIdx.x / 3;")
    a_(f"  const int e = tile * {LANES} + lane;")
    a_("  const bool act = e < K;")
    a_("  const int el = act ? e : K - 1;")
    a_("  const size_t Ks = (size_t)K;")
    a_(f"  const R* __restrict__ xc = X + (size_t)c * {N} * Ks + el;")
    a_(f"  R* __restrict__ vc = V + (size_t)c * {N} * Ks + e;")
    a_(f"  for (int r = w; r < {N}; r += {q}) sh[r * {LANES} + lane] = xc[r * Ks];")
    # the old values of the wave's rows, loaded now (their latency hides behind the work)
    # the old values of the wave's rows, loaded first (their latency hides behind the work)
    a_(f"  R vo[{nvo}];")
    a_(f"  for (int k = 0; k < {nvo}; ++k) vo[k] = R(0);")
    a_("  if (acc) {")
    a_("    switch (w) {")
    for w in range(q):
        rs = [r for k in range(nsets) for r in wave_rows[k][w]]
        a_(f"      case {w}:")
        for n, r in enumerate(rs):
            a_(f"        vo[{n}] = V[(size_t)(c * {N} + {r}) * Ks + el];")
        a_("        break;")
    a_("    }")
    a_("  }")
    a_("  const R m0 = mat[el], dm1 = mat[Ks + el] - m0, dm2 = mat[2 * Ks + el] - m0, dm3 = mat[3 * Ks + el] - m0;")
    for (i, j) in pairs:
        a_(f"  R g{i}_{j};")
    a_("  R mslice, ya, za;")
    a_("  __syncthreads();")
    # k-step per slice: g_ij = sum_k C1[ijk, a_w] r_ijk, literal per wave
    a_("  switch (w) {")
    for w in range(q):
        a_(f"    case {w}:")
        for (i, j) in pairs:
            rs = modes_of[(i, j)]
            a_(f"      g{i}_{j} = " + " + ".join(f"R({_h(C1[r, w])}) * sh[{r * LANES} + lane]" for r in rs) + ";")
        a_(f"      mslice = m0 + dm1 * R({_h((1 + xa[w]) / 2)});")
        a_(f"      ya = R({_h((1 - xa[w]) / 4)});")
        a_(f"      za = R({_h((1 - xa[w]) / 8)});")
        a_("      break;")
    a_("  }")
    a_("  __syncthreads();  // the column is dead: its LDS holds the slices' h next")
    # j-step: u_ib = sum_j Fb[i, j, b] g_ij
    for i in range(p + 1):
        for b in range(q):
            js = list(range(p + 1 - i))
            e0 = f"R({_h(Fb[i, js[0], b])}) * g{i}_{js[0]}"
            rest = "".join(f" + R({_h(Fb[i, jj, b])}) * g{i}_{jj}" for jj in js[1:])
            a_(f"  R u{i}_{b} = {e0}{rest};")
    ev = [i for i in range(p + 1) if i % 2 == 0]
    od = [i for i in range(p + 1) if i % 2 == 1]

    def lin(terms):
        return " + ".join(f"R({_h(cf_)}) * {x}" for cf_, x in terms) if terms else "R(0)"

    # c-step, point scale and c-step back per b-column; nodes j and q-1-j share the even
    # and odd Legendre sums
    for b in range(q):
        a_("  {")
        a_(f"    const R mrow = mslice + dm2 * (ya * R({_h(1 + xb[b])}));")
        a_(f"    const R dz = dm3 * (za * R({_h(1 - xb[b])}));")
        for j in range(h):
            jj = q - 1 - j
            a_(f"    const R e{j} = {lin([(Fc[i, j], f'u{i}_{b}') for i in ev])};")
            a_(f"    const R o{j} = {lin([(Fc[i, j], f'u{i}_{b}') for i in od])};")
            a_(f"    const R f{j} = (e{j} + o{j}) * mass_rcp<R>(mrow + dz * R({_h(1 + xc[j])}));")
            a_(f"    const R f{jj} = (e{j} - o{j}) * mass_rcp<R>(mrow + dz * R({_h(1 + xc[jj])}));")
            a_(f"    const R sp{j} = f{j} + f{jj}, sm{j} = f{j} - f{jj};")
        if mid is not None:
            a_(f"    const R f{mid} = ({lin([(Fc[i, mid], f'u{i}_{b}') for i in ev])}) * mass_rcp<R>(mrow + dz * R({_h(1 + xc[mid])}));")
        for i in range(p + 1):
            terms = [(Fc[i, j] * wc[j], (f"sp{j}" if i % 2 == 0 else f"sm{j}")) for j in range(h)]
            if mid is not None and i % 2 == 0:
                terms.append((Fc[i, mid] * wc[mid], f"f{mid}"))
            a_(f"    u{i}_{b} = {lin(terms)};")
        a_("  }")
    # j-step back: h_ij = sum_b Fb[i, j, b] w_b u_ib
    for (i, j) in pairs:
        terms = [(Fb[i, j, b] * wb[b], f"u{i}_{b}") for b in range(q)]
        a_(f"  const R h{i}_{j} = {lin(terms)};")
    # per set: h to LDS as sh[(n q + w) LANES + lane] (n the pair's place in the set), then the
    # k-step back over the slices for the wave's rows of the set
    for k, st in enumerate(sets):
        if k:
            a_("  __syncthreads();")
        for n, pi in enumerate(st):
            i, j = pairs[pi]
            a_(f"  sh[({n * q} + w) * {LANES} + lane] = h{i}_{j};")
        a_("  __syncthreads();")
        a_("  switch (w) {")
        for w in range(q):
            base = sum(len(wave_rows[kk][w]) for kk in range(k))
            a_(f"    case {w}:")
            for n, r in enumerate(wave_rows[k][w]):
                i, j, _ = t.modes[r]
                pn = st.index(pidx[(i, j)])
                expr = " + ".join(f"R({_h(C1[r, sa] * wa[sa] / 64.0)}) * sh[{(pn * q + sa) * LANES} + lane]" for sa in range(q))
                a_(f"      if (act) vc[{r} * Ks] = vo[{base + n}] + s * ({expr});")
            a_("      break;")
        a_("  }")
    a_("}")
    return "\n".join(L) + "\n"


def emit_unit(p: int, f64: bool) -> str:
    tu = [f"// Generated by gen/emit.py: approximate mass-inverse kernel and launcher for order {p}.",
          "#include <hip/hip_runtime.h>",
          '#include "../launch.h"',
          f'#include "mass_p{p}.inc"',
          "template <typename R>",
          f"static hipError_t launch_mass_p{p}(const MassArgs<R>& a) {{",
          f"  hipLaunchKernelGGL(dgm_mass_p{p}<R>, dim3(3 * a.blocks), dim3({(p + 1) * LANES}), 0, a.stream, a.X, a.V, a.mat, a.s, a.acc, a.K);",
          "  return hipGetLastError();",
          "}",
          f"hipError_t dgm_launch_mass_p{p}_f32(const MassArgs<float>& a) {{ return launch_mass_p{p}<float>(a); }}"]
    if f64:
        tu.append(f"hipError_t dgm_launch_mass_p{p}_f64(const MassArgs<double>& a) {{ return launch_mass_p{p}<double>(a); }}")
    return "\n".join(tu) + "\n"
