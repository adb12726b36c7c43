"""FP64 CPU oracle for the nodal DG Maxwell right-hand side and its LSERK driver.

TEST INFRASTRUCTURE ONLY.  Nothing in the library path may import, call or
execute this package: only the tests, the smoke check of the entry module and
the CPU-baseline leg of the benchmark use it.  It shares no code with the HIP
library; only the seeded input generators in ``dg_inputs`` serve both.

It computes, plainly and slowly, the semi-discrete operator of the paper's
Section 2 (strong DG form, the matrices M, S, D = M^-1 S, the face mass
matrices and the lifting matrix L of the figure on its construction), for
Maxwell's equations with the upwind flux of the results section, on affine
tetrahedra (Section 2.1), and the five-stage low-storage RK4 used to step it.

Modules
  refelem   reference tetrahedron: nodes, basis, Vandermonde, Dr/Ds/Dt, Fmask,
            face mass matrices, LIFT, quadrature mass/stiffness
  mesh      affine geometry (rx..tz, J, normals, sJ, Fscale) and connectivity
            by coordinate matching
  maxwell   the right-hand side
  lserk     the 5-stage 4th-order low-storage Runge-Kutta scheme
  diag      energy, dissipation form, error norms, operator assembly

Parity status per function is given in each module header; every function is
pinned by the CPU tests under tests/ (test_oracle_*.py).
"""
from . import refelem, mesh, maxwell, lserk, diag  # noqa: F401
