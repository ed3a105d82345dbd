"""Plain FP64 CPU oracle for the matrix-free phase-field Jacobian path.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or links
this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do. It shares no code, tables or constants with the HIP
library: mesh, constraints, finite elements, assembly and the solvers are
written here again, slowly and plainly, from the paper (Kolditz & Wick,
"Matrix-Free Geometric Multigrid Preconditioning of Combined Newton-GMRES for
Solving Phase-Field Fracture with Local Mesh Refinement"):

* mesh.py      quadtree, nodes, hanging-node / Dirichlet constraints (Sec. 4, Table 1)
* fe.py        Q1/Q2 Lagrange elements and Gauss quadrature (Sec. 3)
* assemble.py  residual (Problem 2), Jacobian (Sec. 3.1), masked operator,
               diagonal, transpose, crack volume and parameter derivatives
* mg.py        level meshes, transfers, level block operators, Chebyshev-Jacobi,
               eigenvalue estimate, local-smoothing V-cycle (Sec. 3.2)
* krylov.py    left-preconditioned restarted GMRES (Sec. 3.2)
* newton.py    one primal-dual active set / line-search Newton iteration (Alg. 2)

Every function states the passage it follows; readings of passages that are
silent or ambiguous are listed in the repository's design notes.
"""
