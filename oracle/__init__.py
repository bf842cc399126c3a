"""FP64 CPU oracle for the Bernstein-Bezier DG acoustic solver.

TEST INFRASTRUCTURE ONLY.  Nothing on the solver's product path may import,
call or link anything in this package; only the test suite, the smoke check
and the CPU-baseline leg of the benchmark use it.

It evaluates the semi-discrete DG operator of the first-order acoustic system
(Section 2 and the strong-form ODE system of Section 3) with *dense* reference
operators: barycentric derivative matrices obtained by evaluating the scaled
barycentric monomials B_alpha (Section 3.1) and their derivatives at the
equispaced lattice and solving with the Bernstein-Vandermonde matrix, and the
face lift matrices L^f = M^{-1} M^f from the exact simplex integrals of
barycentric monomials.  Both are computed exactly in rational arithmetic and
rounded once to float64.  Time integration is the five-stage, fourth-order
low-storage Runge-Kutta method of Carpenter and Kennedy cited in Section 4.2.

Modules:
  bernstein  multi-indices and dense exact operators (M, M^f, D^i, L^f)
  mesh       affine geometry and face matching from vertices and topology
  dg         right-hand side, LSRK4, energy, projection, quadrature errors
"""
