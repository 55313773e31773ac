"""Oracle: a plain, slow, FP64 CPU implementation of the central-flux DG
Maxwell solver, written from the paper's statement of the method.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` (``oracle_leg``) may import it.  The product
(``paper_1104_4208_amd``) never imports or calls it, and it shares no code
with the product: its Jacobi polynomials, quadrature, basis, geometry,
neighbour search and operators are written here independently.

Contents
  jacobi  -- Jacobi polynomials (three-term recurrence), Gauss-Jacobi rules
  basis   -- orthonormal Dubiner basis on the reference tetrahedron (Section 4.2.2)
  dg      -- mesh geometry, L2 projection, strong-form H / weak-form E central-flux
             right-hand sides, symplectic Euler (Section 3), energies, power
             iteration for the time-step bound, dense operator assembly.
  stab    -- the stabilised central flux with face unknowns H^F (Section 2.1):
             per-face tangential unknowns, their update from the tangential
             jump of E, the extra E-equation term, energies, assembly.
  mixed   -- mixed orders, E of degree p+1 and H of degree p (Section 2).
  varcoef -- material varying inside the elements through the approximate mass
             inverse of Section 3.3.2 (reverse integration, division by the
             material at the points, integration).

Pins (tests/test_oracle.py) tie each function to something other than
itself: closed-form norms, orthogonality, integration by parts, exact
polynomial reproduction of curl, skew-symmetry of the semi-discrete system,
exact conservation of the leapfrog invariant, the scalar stability
threshold, and h-convergence to the exact PEC cube eigenmodes
(tests/test_oracle_stab.py for the stabilised flux: skew-symmetry, the
null-space dimension in closed form, cavity eigenvalues kept and spurious
ones removed, reduction to the central flux, exact leapfrog invariant;
tests/test_oracle_mixed.py for mixed orders: skew-symmetry, exact curls of
global polynomials, exact invariant, no spurious mode below the first cavity
mode, TE101 convergence; tests/test_oracle_varcoef.py for the approximate mass
inverse: exact for constant material, symmetric positive definite, second-order
agreement with the exact inverse, skew in its own inner product, exact invariant).

Parity unpinned: the paper's own experiments (the spherical resonator of
Section 2.2 and the timings of Section 3.5) cannot be reproduced here: the
meshes and the reference data are not available.
"""
from .basis import eval_basis, mode_list, num_modes, tet_quadrature, triangle_quadrature  # noqa: F401
from .dg import Mesh, Solver, build_mesh  # noqa: F401
from .stab import StabilizedSolver  # noqa: F401
from .mixed import MixedSolver  # noqa: F401
from .varcoef import VarMaterialSolver  # noqa: F401
from .jacobi import djacobi, gauss_jacobi, jacobi  # noqa: F401
