"""The generated approximate mass-inverse kernels (Section 3.3.2), executed on the CPU.

The emitted kernel body of every order is interpreted line by line in Python (one lane
of every wave of a workgroup: the per-slice k-step of the wave's case, the shared j- and
c-steps, the LDS hand-off of the slices' results and the k-step back of each wave's rows)
and compared with the plain definition
    (P r)_a = sum_x w_x phi_a(x) (sum_b phi_b(x) r_b) / m(x)
evaluated with the oracle's own basis and collapsed Gauss rule (p + 1 points per
direction) and m linear from four vertex values.  Also pins the sum-factorisation tables
(tables.mass_factors) against the oracle's basis at the oracle's points."""
import re

import numpy as np
import pytest

import oracle
from paper_1104_4208_amd.gen import mass as MS
from paper_1104_4208_amd.gen import tables as TB
from paper_1104_4208_amd.gen.basis import volume_modes

LANES = MS.LANES


def _lit(s):
    return re.sub(r"R\((-?0x[^)]*)\)", lambda m: repr(float.fromhex(m.group(1))), s)


def _python(lines):
    out = []
    for ln in lines:
        s = ln.strip()
        if (not s or s in ("{", "}", "break;") or s.startswith(("//", "__syncthreads", "case", "for (int k",
                                                                   "if (acc", "switch", "vo[", "R vo["))):
            continue
        s = _lit(s.rstrip(";"))
        s = s.replace("const R ", "").replace("R ", "").replace("mass_rcp<R>", "1.0/")
        s = re.sub(r"sh\[(\d+) \+ lane\]", lambda m: f"sh[{int(m.group(1)) // LANES}]", s)
        if ", " in s and "=" in s.split(",")[1]:
            out += [x.strip() for x in s.split(", ")]
        else:
            out.append(s)
    return "\n".join(out)


def _cases(block, q):
    out = {}
    for w in range(q):
        a = block.index(f"case {w}:")
        out[w] = block[a:block.index("break;", a)].split("\n")[1:]
    return out


def run_emitted(p, col, mv):
    """One lane's output of dgm_mass_p{p} (acc = 0, s = 1) for input column col."""
    src = MS.emit_mass(p)
    q, N = p + 1, TB.build(p).N
    body = src.split("R mslice, ya, za;")[1]
    dead = "__syncthreads();  // the column is dead: its LDS holds the slices' h next"
    kstep, rest = body.split(dead)
    mid_end = rest.index("  sh[(")
    middle = _python(rest[:mid_end].split("\n"))
    kc = _cases(kstep, q)
    h = {}
    for w in range(q):
        env = dict(sh=col, m0=mv[0], dm1=mv[1] - mv[0], dm2=mv[2] - mv[0], dm3=mv[3] - mv[0])
        exec(_python(kc[w]), env)
        exec(middle, env)
        h[w] = {k: v for k, v in env.items() if re.fullmatch(r"h\d+_\d+", k)}
    out = {}
    parts = rest[mid_end:].split("  switch (w) {")
    writes = parts[0]
    for blk in parts[1:]:
        sh = {}
        for m in re.finditer(r"sh\[\((\d+) \+ w\) \* %d \+ lane\] = (h\d+_\d+);" % LANES, writes):
            for w in range(q):
                sh[int(m.group(1)) + w] = h[w][m.group(2)]
        shl = np.zeros(max(sh) + 1)
        for k, v in sh.items():
            shl[k] = v
        for w, lines in _cases(blk, q).items():
            for ln in lines:
                m = re.search(r"vc\[(\d+) \* Ks\] = vo\[\d+\] \+ s \* \((.*)\);", ln)
                if m:
                    expr = re.sub(r"sh\[(\d+) \+ lane\]", lambda mm: f"shl[{int(mm.group(1)) // LANES}]", _lit(m.group(2)))
                    assert int(m.group(1)) not in out, "row written twice"
                    out[int(m.group(1))] = eval(expr, {"shl": shl})
        writes = blk
    assert sorted(out) == list(range(N)), "every row written once"
    return np.array([out[r] for r in range(N)])


def definition(p, col, mv):
    """P col from the oracle's basis and rule, in the library's mode order."""
    x, w = oracle.tet_quadrature(p + 1)
    V = oracle.eval_basis(p, x)  # (N, Q), oracle mode order
    idx = {m: r for r, m in enumerate(oracle.mode_list(p))}
    perm = np.array([idx[m] for m in volume_modes(p)])
    V = V[perm]
    lam = np.stack([1 - x.sum(1), x[:, 0], x[:, 1], x[:, 2]], axis=1)
    return V @ (w / (lam @ mv) * (V.T @ col))


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_emitted_mass_kernel_matches_the_definition(p):
    rng = np.random.default_rng(90 + p)
    N = TB.build(p).N
    for _ in range(2):
        col = rng.standard_normal(N)
        mv = rng.uniform(0.5, 4.0, 4)
        got, ref = run_emitted(p, col, mv), definition(p, col, mv)
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [2, 5, 8])
def test_mass_factors_reproduce_the_oracle_basis(p):
    f = TB.mass_factors(p)
    t = TB.build(p)
    x, _ = oracle.tet_quadrature(p + 1)  # the same collapsed points, in (a, b, c) order
    idx = {m: r for r, m in enumerate(oracle.mode_list(p))}
    V = oracle.eval_basis(p, x)[[idx[m] for m in volume_modes(p)]].reshape(t.N, p + 1, p + 1, p + 1)
    for r, (i, j, k) in enumerate(t.modes):
        prod = f["C1"][r][:, None, None] * f["Fb"][i, j][None, :, None] * f["Fc"][i][None, None, :]
        assert np.abs(prod - V[r]).max() < 1e-11 * max(1.0, np.abs(V[r]).max())


def test_constant_material_gives_the_identity_over_m():
    """m constant: P = I / m exactly (the rule is exact on products of two basis functions)."""
    p = 4
    N = TB.build(p).N
    col = np.random.default_rng(3).standard_normal(N)
    got = run_emitted(p, col, np.full(4, 2.5))
    assert np.abs(got - col / 2.5).max() < 1e-13
