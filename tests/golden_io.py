"""Readers for the text fixtures under tests/golden (printed relations of the paper)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _expr(src):
    allowed = set("ijkn0123456789+-*() ")
    if not set(src) <= allowed:
        raise ValueError(f"unexpected characters in fixture expression {src!r}")
    code = compile(src, "<fixture>", "eval")
    return lambda **kw: eval(code, {"__builtins__": {}}, kw)


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        for ln in fh:
            ln = ln.strip()
            if ln and not ln.startswith("#"):
                yield ln


def legendre_relation():
    """[(coef(n), shift, deriv)] for S_n^2 D + (-2n-3) S_n - D."""
    out = []
    for ln in _lines("legendre_relations.txt"):
        c, s, d = [t.strip() for t in ln.split("|")]
        out.append((_expr(c), int(s), int(d)))
    return out


def relations_2d():
    """{'dx': [(coef(i,j), (si,sj), 'x'|'-')], 'dy': [...]}"""
    rel, cur = {}, None
    for ln in _lines("relations_2d.txt"):
        if ln.startswith("["):
            cur = ln.strip("[]")
            rel[cur] = []
            continue
        c, s, d = [t.strip() for t in ln.split("|")]
        rel[cur].append((_expr(c), tuple(int(v) for v in s.split()), d))
    return rel


def support_dx_3d():
    out = []
    for ln in _lines("support_dx_3d.txt"):
        s, d = [t.strip() for t in ln.split("|")]
        out.append((tuple(int(v) for v in s.split()), d))
    return out
