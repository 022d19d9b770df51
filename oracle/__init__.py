"""Plain FP64 CPU oracle for BDDC-preconditioned CG on unfitted Q1 meshes.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
run this package: only the tests, the package smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path;
the only common module is `workloads`, which draws seeded inputs and holds
none of the method's arithmetic.

Source: S. Badia and F. Verdugo, "Robust and scalable domain decomposition
solvers for unfitted finite element methods" (arXiv:1703.06323).  Each
function cites the section / equation it follows.  Where the paper is silent
the reading taken is stated in the function's docstring.

Modules
  geometry   sub-cell Gauss points, kept-point test, cell classification (Sect. 2.1)
  integrate  cut-cell element stiffness / mass (Sect. 2.2, A_e with Gamma_D = 0)
  surface    Nitsche terms on the ball surfaces and beta_e (Sect. 2.2, eq. local-eigenvals)
  assemble   DOF numbering, global operator and load (Sect. 2.2)
  topology   subdomains, node subdomain sets, objects, variant-1 splitting,
             coarse numbering (Sects. 3.1, 3.2, 4.4)
  bddc       weighting (eq. weighting / eq. alge-weighting), local Dirichlet
             and constrained Neumann problems, coarse space, M r (eq. bddc)
  pcg        preconditioned conjugate gradients with the stopping test of Sect. 5.1
  adjoint    adjoint gradient of J = 0.5 |u - u_t|^2 w.r.t. per-cell
             log-conductivity and nodal source

Parity pins for each function live in tests/test_oracle_*.py.
"""
from . import geometry, integrate, surface, assemble, topology, bddc, pcg, adjoint  # noqa: F401
from .driver import OracleSolver  # noqa: F401
