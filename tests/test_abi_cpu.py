"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, reports the mode order, and rejects bad meshes before any
device allocation."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1104_4208_amd as P
from paper_1104_4208_amd import dgmax as D

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "dgmax.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dgm_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    lib = P.load_library()
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
        assert s in D.SIGNATURES, f"binding misses {s}"
    assert set(D.SIGNATURES) == set(syms)


def test_mode_counts_and_order():
    for p in range(0, 9):
        assert P.num_modes(p) == (p + 1) * (p + 2) * (p + 3) // 6
        assert P.num_face_modes(p) == (p + 1) * (p + 2) // 2
    for p in (1, 4, 6):
        tab = P.mode_table(p)
        assert len(set(tab)) == len(tab)
        deg = [sum(m) for m in tab]
        assert deg == sorted(deg)
        assert all(0 <= min(m) and sum(m) <= p for m in tab)
    with pytest.raises(P.DGMError):
        P.mode_index(2, 10)
    assert P.max_order(P.DGM_F32) >= 8 and P.max_order(P.DGM_F64) >= 4


def _create(verts, tets):
    lib = P.load_library()
    v = np.ascontiguousarray(verts, dtype=np.float64)
    t = np.ascontiguousarray(tets, dtype=np.int64)
    h = ctypes.c_void_p()
    rc = lib.dgm_create_mesh(v.ctypes.data_as(D._pd), v.shape[0], t.ctypes.data_as(D._pi64), t.shape[0], ctypes.byref(h))
    return rc, lib.dgm_last_error().decode()


def test_mesh_errors_are_reported_before_device_work():
    flat = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)
    assert _create(flat, [[0, 1, 2, 3]])[0] == -2
    assert _create(flat, [[0, 1, 2, 2]])[0] == -2
    assert _create(flat, [[0, 1, 2, 7]])[0] == -1
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1]], float)
    rc, msg = _create(v, [[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]])
    assert rc == -3 and "more than two" in msg
    rc, msg = _create(flat, np.zeros((0, 4), np.int64))  # empty mesh
    assert rc == -1
    lib = P.load_library()
    # the element-count limit is checked before the arrays are read
    v = np.ascontiguousarray(v)
    t = np.zeros((1, 4), np.int64)
    h = ctypes.c_void_p()
    rc = lib.dgm_create_mesh(v.ctypes.data_as(D._pd), v.shape[0], t.ctypes.data_as(D._pi64), (1 << 28) - 63,
                             ctypes.byref(h))
    assert rc == -1 and "too many elements" in lib.dgm_last_error().decode()
    assert lib.dgm_create_mesh(None, 0, None, 0, None) == -1
    assert lib.dgm_set_order(None, 2) == -1
    assert lib.dgm_step(None, 0, None, None, 0.1, 1, None) == -1


def _hostmesh(monkeypatch, K=6, p=2):
    """A Mesh object without a device handle whose field check accepts host tensors, so
    the binding's argument checks can run here; any library call fails the test."""
    import torch

    m = object.__new__(P.Mesh)
    m._h, m.K, m.p = None, K, p
    N = (p + 1) * (p + 2) * (p + 3) // 6
    monkeypatch.setattr(P.Mesh, "N", property(lambda self: N))

    def field(self, t, name):
        if t is None:
            return None
        if tuple(t.shape) != (3, N, K) or not t.is_contiguous():
            raise D.DGMError(f"{name} shape")
        return t

    monkeypatch.setattr(P.Mesh, "_field", field)

    def no_lib(*a, **k):
        raise AssertionError("reached the library")

    monkeypatch.setattr(D, "load_library", no_lib)
    z = lambda dt: torch.zeros((3, N, K), dtype=dt)
    return m, z


def test_binding_rejects_mixed_dtypes_before_the_library(monkeypatch):
    import torch

    m, z = _hostmesh(monkeypatch)
    f32, f64 = torch.float32, torch.float64
    with pytest.raises(D.DGMError, match="H has dtype"):
        m.apply_curl(z(f64), z(f32))
    with pytest.raises(D.DGMError, match="dE has dtype"):
        m.apply_curl(None, z(f64), dE=z(f32))
    with pytest.raises(D.DGMError, match="dH has dtype"):
        m.apply_curl(z(f32), None, dH=z(f64))
    with pytest.raises(D.DGMError, match="H_next has dtype"):
        m.energy(z(f64), z(f64), H_next=z(f32))
    with pytest.raises(D.DGMError, match="H has dtype"):
        m.energy(z(f64), z(f32))
    with pytest.raises(D.DGMError, match="dH has dtype"):
        m.apply_curl_dense(z(f32), None, dH=z(f64))
    with pytest.raises(D.DGMError, match="float32"):
        m.apply_curl_dense(None, z(f64), dE=z(f64))
    with pytest.raises(D.DGMError, match="shape"):
        m.apply_curl(None, z(f32), dE=torch.zeros((3, 10, 5)))
    with pytest.raises(D.DGMError, match="needs"):
        m.energy(None, z(f32))
