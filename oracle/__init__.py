"""Plain CPU FP64 oracle for the mobility MVP and the PQN / Bi-PQN LCP solvers.

This package is TEST INFRASTRUCTURE. Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import it. The product path (the HIP
library and its Python binding) never calls it, and it shares no code with that
path: every routine here is written from the paper's statement (Rummel, Jensen,
Becker, Corona, "A Bifidelity Proximal Quasi-Newton Method for Dense Rigid Body
Suspension Collision Resolution") or from the textbook definition it relies on,
in plain numpy/scipy FP64, slow and straightforward.

Modules
-------
grid      Gauss-Legendre x trapezoid sphere grids and the degree-p spherical
          harmonic projection (Sec. 5.1, "coarseness of discretization").
bie       The completed double-layer boundary integral equation, its discrete
          operator (self block, off-particle pair sums, near pairs, rigid
          projection, Stokeslet/rotlet completion), GMRES and the mobility
          MVP U = M F (Sec. 2, eq. (mobility), Fig. 1).
lcp       Contact Jacobian, the LCP operator A = D^T M D and b (eq. (LCP),
          eq. (defAandb)), the KKT error (eq. (kkt-error)), the weighted prox
          (Prop. 1, Alg. 3), the optimal over-relaxation (Alg. 2), BFGS, BB-PGD
          (eq. (spectralStepSize)), Mono-PQN (Alg. 1), Bi-PQN (Alg. 4) and a
          brute-force LCP solver.
dynamics  Contact detection (eq. (collisional-set)) and one forward-Euler step
          of the linearised DVI (eq. (dvi)).

Parity status of each function is stated in its docstring ("pinned by ..." or
"parity unpinned").
"""
