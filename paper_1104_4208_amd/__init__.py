"""MI355X-native DG Maxwell curl engine (arxiv 1104.4208, flat-element path).

    from paper_1104_4208_amd import Mesh
    m = Mesh(verts, tets).set_order(6).set_material(eps, mu)
    m.step(E, H, dt, nsteps)          # E, H: (3, N, K) device tensors

Everything runs in libdgmax.so (C-ABI in include/dgmax.h); this package only
marshals arguments.  Build the library with ``python -m paper_1104_4208_amd.build``.
"""
from .dgmax import (DGM_BF16, DGM_F16, DGM_F32, DGM_F64, Batch, DGMError, Mesh, load_library, max_order, mode_index,  # noqa: F401
                    mode_table, num_face_modes, num_modes)
