"""Thin ctypes binding of libdgmax.so (include/dgmax.h).

Argument marshalling only: every operation runs in the library's HIP kernels
on the caller's current torch stream.  Field tensors are CUDA (HIP) tensors of
shape (3, N, K), contiguous, float32 or float64, holding reference covariant
modal coefficients in the library's mode order.  There is no fallback: if the
shared library is missing or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgmax.so")

DGM_F32, DGM_F64 = 0, 1
DGM_BF16, DGM_F16 = 2, 3
ERRORS = {
    -1: "DGM_ERR_ARG", -2: "DGM_ERR_MESH_DEGENERATE", -3: "DGM_ERR_MESH_NONMANIFOLD", -4: "DGM_ERR_MATERIAL",
    -5: "DGM_ERR_OOM", -6: "DGM_ERR_HIP", -7: "DGM_ERR_UNSTABLE", -8: "DGM_ERR_STATE",
}

_c_i = ctypes.c_int
_c_i64 = ctypes.c_int64
_c_d = ctypes.c_double
_c_p = ctypes.c_void_p
_pd = ctypes.POINTER(ctypes.c_double)
_pi = ctypes.POINTER(ctypes.c_int)
_pi64 = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes): every symbol declared in include/dgmax.h
SIGNATURES = {
    "dgm_last_error": (ctypes.c_char_p, []),
    "dgm_num_modes": (_c_i, [_c_i]),
    "dgm_num_face_modes": (_c_i, [_c_i]),
    "dgm_max_order": (_c_i, [_c_i]),
    "dgm_mode_index": (_c_i, [_c_i, _c_i, _pi, _pi, _pi]),
    "dgm_create_mesh": (_c_i, [_pd, _c_i64, _pi64, _c_i64, ctypes.POINTER(_c_p)]),
    "dgm_destroy": (_c_i, [_c_p]),
    "dgm_num_elements": (_c_i, [_c_p, _pi64]),
    "dgm_set_order": (_c_i, [_c_p, _c_i]),
    "dgm_set_orders": (_c_i, [_c_p, _c_i, _c_i]),
    "dgm_orders": (_c_i, [_c_p, _pi, _pi]),
    "dgm_set_material": (_c_i, [_c_p, _pd, _pd]),
    "dgm_set_material_linear": (_c_i, [_c_p, _pd, _pd]),
    "dgm_apply_mass_inverse": (_c_i, [_c_p, _c_i, _c_i, _c_p, _c_p, _c_p]),
    "dgm_set_check_interval": (_c_i, [_c_p, _c_i64]),
    "dgm_apply_curl": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "dgm_step": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_d, _c_i64, _c_p]),
    "dgm_step_noalloc": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_d, _c_i64, _c_p]),
    "dgm_energy": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p, _c_d, _pd, _c_p]),
    "dgm_step_probe": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_d, _c_i64, _c_p, _pd, _c_p]),
    "dgm_estimate_dt": (_c_i, [_c_p, _c_d, _c_i, ctypes.c_uint64, _pd, _pd, _c_p]),
    "dgm_set_stab_alpha": (_c_i, [_c_p, _c_d]),
    "dgm_num_face_unknowns": (_c_i, [_c_p, _pi64]),
    "dgm_apply_stab": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "dgm_step_stab": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p, _c_d, _c_i64, _c_p]),
    "dgm_energy_stab": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p, _c_d, _pd, _c_p]),
    "dgm_estimate_dt_stab": (_c_i, [_c_p, _c_d, _c_i, ctypes.c_uint64, _pd, _pd, _c_p]),
    "dgm_apply_curl_dense": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_p, _c_p, _c_p]),
    "dgm_step_dense": (_c_i, [_c_p, _c_i, _c_p, _c_p, _c_d, _c_i64, _c_p]),
    "dgm_batch_create": (_c_i, [_c_i, ctypes.POINTER(_c_p)]),
    "dgm_batch_destroy": (_c_i, [_c_p]),
    "dgm_batch_add": (_c_i, [_c_p, _c_p, _c_p, _c_p, _c_d, _c_i64, _c_p, _pi64]),
    "dgm_batch_num_active": (_c_i, [_c_p, _pi64]),
    "dgm_batch_advance": (_c_i, [_c_p, _c_p]),
    "dgm_batch_launch": (_c_i, [_c_p, _c_p]),
    "dgm_batch_wait": (_c_i, [_c_p]),
    "dgm_batch_needs_capture": (_c_i, [_c_p, ctypes.POINTER(_c_i)]),
    "dgm_batch_take_finished": (_c_i, [_c_p, _pi64, _c_i64, _pi64]),
}

_lib = None


class DGMError(RuntimeError):
    pass


def load_library(path: str = LIB_PATH):
    """Load libdgmax.so and declare its signatures; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise DGMError(f"{path} is missing: build it with `python -m paper_1104_4208_amd.build`")
    # torch ships its own HIP runtime with the same soname as the system one; importing
    # it first makes the loader bind the library to that copy, so the process has one
    # HIP runtime (two of them do not see the same devices)
    import torch  # noqa: F401

    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(rc):
    if rc != 0:
        msg = load_library().dgm_last_error().decode(errors="replace")
        raise DGMError(f"{ERRORS.get(rc, rc)}: {msg}")


def num_modes(p: int) -> int:
    return load_library().dgm_num_modes(p)


def num_face_modes(p: int) -> int:
    return load_library().dgm_num_face_modes(p)


def max_order(dtype: int = DGM_F32) -> int:
    return load_library().dgm_max_order(dtype)


def mode_index(p: int, m: int):
    i, j, k = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().dgm_mode_index(p, m, ctypes.byref(i), ctypes.byref(j), ctypes.byref(k)))
    return i.value, j.value, k.value


def mode_table(p: int):
    return [mode_index(p, m) for m in range(num_modes(p))]


def _torch():
    import torch

    return torch


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t):
    torch = _torch()
    if t.dtype == torch.float32:
        return DGM_F32
    if t.dtype == torch.float64:
        return DGM_F64
    raise DGMError("field tensors must be float32 or float64")


class Mesh:
    """A tetrahedral mesh on the device, with order and material."""

    def __init__(self, verts, tets):
        lib = load_library()
        v = np.ascontiguousarray(np.asarray(verts, dtype=np.float64))
        t = np.ascontiguousarray(np.asarray(tets, dtype=np.int64))
        if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 4:
            raise DGMError("verts must be (nv,3) and tets (nt,4)")
        h = ctypes.c_void_p()
        _check(lib.dgm_create_mesh(v.ctypes.data_as(_pd), v.shape[0], t.ctypes.data_as(_pi64), t.shape[0],
                                   ctypes.byref(h)))
        self._h = h
        self.K = int(t.shape[0])
        self._tets = t
        self.nv = int(v.shape[0])
        self.p = None   # order of H (and of E unless set_orders gave E one more)
        self.pE = None

    def close(self):
        if getattr(self, "_h", None):
            load_library().dgm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    @property
    def N(self):
        """Modes per component of H (and of E with equal orders)."""
        return num_modes(self.p)

    @property
    def NE(self):
        return num_modes(self.pE)

    def set_order(self, p: int):
        _check(load_library().dgm_set_order(self._h, int(p)))
        self.p = self.pE = int(p)
        return self

    def set_orders(self, pE: int, pH: int):
        """Mixed orders (Section 2): E of degree pE = pH + 1, H of degree pH (pE == pH is
        set_order).  E-shaped arrays then have NE modes per component, H-shaped ones N."""
        _check(load_library().dgm_set_orders(self._h, int(pE), int(pH)))
        self.p, self.pE = int(pH), int(pE)
        return self

    def set_material(self, eps=None, mu=None):
        def arr(x):
            if x is None:
                return None, None
            a = np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (self.K,)))
            return a, a.ctypes.data_as(_pd)

        ea, ep = arr(eps)
        ma, mp = arr(mu)
        _check(load_library().dgm_set_material(self._h, ep, mp))
        return self

    def set_material_linear(self, eps=None, mu=None):
        """Material linear inside every element (Section 3.3.2): (K, 4) values at each
        element's vertices, in the order the element was given; None means 1."""
        def arr(x):
            if x is None:
                return None, None
            a = np.ascontiguousarray(np.broadcast_to(np.asarray(x, dtype=np.float64), (self.K, 4)))
            return a, a.ctypes.data_as(_pd)

        ea, ep = arr(eps)
        ma, mp = arr(mu)
        _check(load_library().dgm_set_material_linear(self._h, ep, mp))
        return self

    def set_material_nodal(self, eps=None, mu=None):
        """Material continuous and piecewise linear over the mesh: values at the mesh
        vertices (length nv); each element takes those of its four vertices
        (dgm_set_material_linear).  None means 1."""
        def at_elements(x):
            if x is None:
                return None
            a = np.asarray(x, dtype=np.float64)
            if a.shape != (self.nv,):
                raise DGMError(f"nodal material must have shape ({self.nv},)")
            return a[self._tets]

        return self.set_material_linear(at_elements(eps), at_elements(mu))

    def set_check_interval(self, every: int):
        """dgm_step checks the state every `every` steps (0: never) and raises
        DGMError (DGM_ERR_UNSTABLE) on a non-finite one."""
        _check(load_library().dgm_set_check_interval(self._h, int(every)))
        return self

    # fields shaped like E (NE modes) and like H (N modes)
    _E_LIKE = ("E", "dE", "w")

    def _field(self, t, name):
        torch = _torch()
        if t is None:
            return None
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise DGMError(f"{name} must be a device tensor")
        n = self.NE if name in self._E_LIKE else self.N
        if tuple(t.shape) != (3, n, self.K) or not t.is_contiguous():
            raise DGMError(f"{name} must be contiguous with shape (3, {n}, {self.K})")
        return t

    def _fields(self, **named):
        """Check every given field (None skipped) with _field and that they share one
        dtype; returns the checked tensors in order and the common dtype code."""
        out = [self._field(t, n) for n, t in named.items()]
        given = [(n, t) for n, t in zip(named, out) if t is not None]
        if not given:
            raise DGMError("no field given")
        dt = given[0][1].dtype
        for n, t in given:
            if t.dtype != dt:
                raise DGMError(f"{n} has dtype {t.dtype}, expected {dt} (all fields must share one dtype)")
        return out, _dtype_code(given[0][1])

    def zeros(self, dtype=None, field="H"):
        """Zeroed (3, N, K) array shaped like H (field="E": like E)."""
        torch = _torch()
        n = self.NE if field == "E" else self.N
        return torch.zeros((3, n, self.K), dtype=dtype or torch.float32, device="cuda")

    def apply_curl(self, E=None, H=None, dE=None, dH=None):
        """Returns (dE, dH) = (-M_eps^{-1} C^T H, M_mu^{-1} C E)."""
        torch = _torch()
        if E is None and H is None:
            raise DGMError("apply_curl needs E or H")
        (E, H, dE, dH), code = self._fields(E=E, H=H, dE=dE if H is not None else None,
                                            dH=dH if E is not None else None)
        if H is not None and dE is None:
            dE = torch.empty((3, self.NE, self.K), dtype=H.dtype, device=H.device)
        if E is not None and dH is None:
            dH = torch.empty((3, self.N, self.K), dtype=E.dtype, device=E.device)
        _check(load_library().dgm_apply_curl(
            self._h, code, _ptr(E), _ptr(H), _ptr(dE if H is not None else None),
            _ptr(dH if E is not None else None), _stream()))
        return (dE if H is not None else None), (dH if E is not None else None)

    def apply_mass_inverse(self, X, field: str = "E", out=None):
        """dgm_apply_mass_inverse: out[c] = P X[c], the approximate mass inverse of the
        material linear on the elements (field "E": eps, "H": mu)."""
        torch = _torch()
        if field not in ("E", "H"):
            raise DGMError("field must be 'E' or 'H'")
        X = self._field(X, field)
        out = torch.empty_like(X) if out is None else self._field(out, field)
        if out.dtype != X.dtype:
            raise DGMError("X and out must share a dtype")
        _check(load_library().dgm_apply_mass_inverse(self._h, _dtype_code(X), 0 if field == "E" else 1, _ptr(X),
                                                      _ptr(out), _stream()))
        return out

    def step(self, E, H, dt: float, nsteps: int = 1):
        E, H = self._field(E, "E"), self._field(H, "H")
        if E.dtype != H.dtype:
            raise DGMError("E and H must share a dtype")
        _check(load_library().dgm_step(self._h, _dtype_code(E), _ptr(E), _ptr(H), float(dt), int(nsteps), _stream()))
        return E, H

    def step_noalloc(self, E, H, dt: float, nsteps: int = 1):
        """dgm_step_noalloc: dgm_step with the library's static device workspace (no
        device allocation; meshes above the workspace size raise)."""
        E, H = self._field(E, "E"), self._field(H, "H")
        if E.dtype != H.dtype:
            raise DGMError("E and H must share a dtype")
        _check(load_library().dgm_step_noalloc(self._h, _dtype_code(E), _ptr(E), _ptr(H), float(dt), int(nsteps),
                                               _stream()))
        return E, H

    def step_probe(self, E, H, dt: float, nsteps: int, w):
        """nsteps steps in place; returns the FP64 signal w . S(E) after every step
        (numpy array of nsteps values; see dgm_step_probe)."""
        E, H, w = self._field(E, "E"), self._field(H, "H"), self._field(w, "w")
        if not (E.dtype == H.dtype == w.dtype):
            raise DGMError("E, H and w must share a dtype")
        sig = (ctypes.c_double * max(int(nsteps), 1))()
        _check(load_library().dgm_step_probe(self._h, _dtype_code(E), _ptr(E), _ptr(H), float(dt), int(nsteps),
                                             _ptr(w), sig, _stream()))
        import numpy as np

        return np.array(sig[:int(nsteps)], dtype=np.float64)

    def energy(self, E, H, H_next=None, dt: float = 0.0):
        """(W, Q) in FP64; Q uses H_next (computed as H + dt dH(E) when None)."""
        if E is None or H is None:
            raise DGMError("energy needs E and H")
        (E, H, Hn), code = self._fields(E=E, H=H, H_next=H_next)
        out = (ctypes.c_double * 2)()
        _check(load_library().dgm_energy(self._h, code, _ptr(E), _ptr(H), _ptr(Hn), float(dt), out,
                                         _stream()))
        return out[0], out[1]

    # -- stabilised central flux with face unknowns (include/dgmax.h) --------------
    def set_stab_alpha(self, alpha0: float = 1.0):
        """Use alpha = alpha0 p^2 in the stabilised-flux calls below."""
        _check(load_library().dgm_set_stab_alpha(self._h, float(alpha0)))
        return self

    @property
    def num_face_unknowns(self) -> int:
        n = ctypes.c_int64()
        _check(load_library().dgm_num_face_unknowns(self._h, ctypes.byref(n)))
        return n.value

    def face_zeros(self, dtype=None):
        """A zeroed face-unknown buffer, shape (2, NF, 4, K)."""
        torch = _torch()
        return torch.zeros((2, num_face_modes(self.p), 4, self.K), dtype=dtype or torch.float32, device="cuda")

    def _faces(self, t, name, dtype):
        torch = _torch()
        if t is None:
            return None
        shape = (2, num_face_modes(self.p), 4, self.K)
        if not isinstance(t, torch.Tensor) or not t.is_cuda or tuple(t.shape) != shape or not t.is_contiguous():
            raise DGMError(f"{name} must be a contiguous device tensor of shape {shape}")
        if t.dtype != dtype:
            raise DGMError(f"{name} has dtype {t.dtype}, expected {dtype}")
        return t

    def apply_stab(self, E=None, H=None, HF=None, want_dE=True, want_dH=True, want_dHF=True):
        """Stabilised rates: (dE from H and HF, dH from E, dHF from E); an output is
        computed when its inputs are given and it is wanted, else None."""
        torch = _torch()
        (E, H), code = self._fields(E=E, H=H)
        dtype = (E if E is not None else H).dtype
        HF = self._faces(HF, "HF", dtype)
        dE = torch.empty_like(H) if (H is not None and HF is not None and want_dE) else None
        dH = torch.empty_like(E) if (E is not None and want_dH) else None
        dHF = torch.empty((2, num_face_modes(self.p), 4, self.K), dtype=dtype, device="cuda") \
            if (E is not None and want_dHF) else None
        _check(load_library().dgm_apply_stab(self._h, code, _ptr(E), _ptr(H), _ptr(HF), _ptr(dE), _ptr(dH), _ptr(dHF),
                                             _stream()))
        return dE, dH, dHF

    def step_stab(self, E, H, HF, dt: float, nsteps: int = 1):
        (E, H), code = self._fields(E=E, H=H)
        HF = self._faces(HF, "HF", E.dtype)
        if E is None or H is None or HF is None:
            raise DGMError("step_stab needs E, H and HF")
        _check(load_library().dgm_step_stab(self._h, code, _ptr(E), _ptr(H), _ptr(HF), float(dt), int(nsteps),
                                            _stream()))
        return E, H, HF

    def energy_stab(self, E, H, HF, dt: float = 0.0):
        """(W, Q) with the face-unknown term, FP64."""
        (E, H), code = self._fields(E=E, H=H)
        HF = self._faces(HF, "HF", E.dtype)
        if E is None or H is None or HF is None:
            raise DGMError("energy_stab needs E, H and HF")
        out = (ctypes.c_double * 2)()
        _check(load_library().dgm_energy_stab(self._h, code, _ptr(E), _ptr(H), _ptr(HF), float(dt), out, _stream()))
        return out[0], out[1]

    def estimate_dt_stab(self, cfl: float = 0.5, iters: int = 50, seed: int = 1):
        dt, rho = ctypes.c_double(), ctypes.c_double()
        _check(load_library().dgm_estimate_dt_stab(self._h, float(cfl), int(iters), int(seed), ctypes.byref(dt),
                                                   ctypes.byref(rho), _stream()))
        return dt.value, rho.value

    def apply_curl_dense(self, E=None, H=None, prec: int = DGM_BF16, dE=None, dH=None):
        """Dense matrix-core variant of apply_curl (FP32 fields, 16-bit operands)."""
        torch = _torch()
        if E is None and H is None:
            raise DGMError("apply_curl_dense needs E or H")
        (E, H, dE, dH), _ = self._fields(E=E, H=H, dE=dE if H is not None else None,
                                         dH=dH if E is not None else None)
        for t in (E, H, dE, dH):
            if t is not None and t.dtype != torch.float32:
                raise DGMError("the dense variant takes float32 fields")
        if H is not None and dE is None:
            dE = torch.empty_like(H)
        if E is not None and dH is None:
            dH = torch.empty_like(E)
        _check(load_library().dgm_apply_curl_dense(
            self._h, int(prec), _ptr(E), _ptr(H), _ptr(dE if H is not None else None),
            _ptr(dH if E is not None else None), _stream()))
        return (dE if H is not None else None), (dH if E is not None else None)

    def step_dense(self, E, H, dt: float, nsteps: int = 1, prec: int = DGM_BF16):
        E, H = self._field(E, "E"), self._field(H, "H")
        torch = _torch()
        if E.dtype != torch.float32 or H.dtype != torch.float32:
            raise DGMError("the dense variant takes float32 fields")
        _check(load_library().dgm_step_dense(self._h, int(prec), _ptr(E), _ptr(H), float(dt), int(nsteps), _stream()))
        return E, H

    def estimate_dt(self, cfl: float = 0.5, iters: int = 50, seed: int = 1):
        dt, rho = ctypes.c_double(), ctypes.c_double()
        _check(load_library().dgm_estimate_dt(self._h, float(cfl), int(iters), int(seed), ctypes.byref(dt),
                                              ctypes.byref(rho), _stream()))
        return dt.value, rho.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Batch:
    """Slots of independent solves advanced together (dgm_batch_*)."""

    def __init__(self, chunk: int = 20):
        h = ctypes.c_void_p()
        _check(load_library().dgm_batch_create(int(chunk), ctypes.byref(h)))
        self._h = h
        self.chunk = int(chunk)
        self._keep = {}

    def close(self):
        if getattr(self, "_h", None):
            load_library().dgm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add(self, mesh: "Mesh", E, H, dt: float, nsteps: int) -> int:
        E, H = mesh._field(E, "E"), mesh._field(H, "H")
        torch = _torch()
        if E.dtype != torch.float32 or H.dtype != torch.float32:
            raise DGMError("batched slots take float32 fields")
        sid = ctypes.c_int64()
        _check(load_library().dgm_batch_add(self._h, mesh.handle, _ptr(E), _ptr(H), float(dt), int(nsteps),
                                            _stream(), ctypes.byref(sid)))
        self._keep[sid.value] = (mesh, E, H)
        return sid.value

    def num_active(self) -> int:
        n = ctypes.c_int64()
        _check(load_library().dgm_batch_num_active(self._h, ctypes.byref(n)))
        return n.value

    def advance(self):
        _check(load_library().dgm_batch_advance(self._h, _stream()))

    def launch(self):
        """First half of advance(): enqueue the next chunk and return."""
        _check(load_library().dgm_batch_launch(self._h, _stream()))

    def wait(self):
        """Second half of advance(): wait for the launched chunk."""
        _check(load_library().dgm_batch_wait(self._h))

    def needs_capture(self) -> bool:
        """Whether the next launch re-captures its HIP graph."""
        y = _c_i()
        _check(load_library().dgm_batch_needs_capture(self._h, ctypes.byref(y)))
        return bool(y.value)

    def take_finished(self):
        cap = 4096
        ids = (ctypes.c_int64 * cap)()
        n = ctypes.c_int64()
        _check(load_library().dgm_batch_take_finished(self._h, ids, cap, ctypes.byref(n)))
        out = [ids[i] for i in range(n.value)]
        for i in out:
            self._keep.pop(i, None)
        return out
