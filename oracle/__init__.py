"""Plain, slow FP64 CPU oracle for discrete flow mapping (DFM) on tetrahedral meshes.

TEST INFRASTRUCTURE ONLY.  This package exists to check the GPU library; it is
not part of the product path.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with
the HIP library (no headers, helpers, tables or constants): every step here is
written from the paper (Bajars, Chappell, Sondergaard, Tanner, "Transport of
phase space densities through tetrahedral meshes using discrete flow mapping").

Module map (paper section -> module):
  Sec. 2 (mesh, phase space on tetrahedron faces)          -> mesh.py
  Sec. 3.1 (product basis, Zernike, orthogonality)         -> basis.py
  Sec. 3.3 (point P, point O, seven regions, L_max,
            analytic spatial integral, five steps)         -> geometry.py
  Sec. 3.4 (seven sub-regions, bilinear patch map,
            radial projection, Jacobian)                   -> quadrature.py
  Sec. 3.2 (Galerkin matrix entries, Eq. Bapprox/B4DInt)   -> assemble.py
  Sec. 2 (Neumann series, Eq. NSum/GovIE)                  -> solve.py
  Sec. 4 (sources projected onto the basis)                -> sources.py

Precision is FP64 throughout.  Where the paper is silent the reading taken is
stated in the function that needs it.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or Monte Carlo ray tracing,
except where a docstring says "parity unpinned".
"""

from . import mesh, basis, quadrature, geometry, assemble, solve, sources  # noqa: F401
