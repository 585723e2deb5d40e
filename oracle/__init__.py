"""Plain FP64 CPU oracle for the fully dissipative 2D ultra-relativistic lattice
Boltzmann method (Coelho, Mendoza, Doria, Herrmann, arXiv:1709.09073).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test suite, the smoke entry and the
benchmark's CPU-baseline leg may import it.  The product path (the HIP library and
its Python binding) never calls it, and it never calls the product path.

Every function follows the paper's definitions step by step, in double precision
(mpmath at 50 digits for the constant tables and the special functions):

* ``quadrature``   - radial Gauss rules of the d2v72 lattice (Sec. 2.4,
                     Eq. quadrature-eq) by Gram-Schmidt, root finding and the
                     moment equations.
* ``gfunc``        - the generalised EDF integral g_nu(z) (Eq. gz-eq) and the
                     (n, eps) -> (theta, z) inversion (Eqs. theta-eq, n-eps-eq).
* ``closed_forms`` - the 56 monomial integrals I_2^{mnq} of the appendix.
* ``equilibrium``  - the N-th order expansion of f^eq as the orthogonal projection
                     onto the span of the relativistic polynomials (Eqs.
                     expansion-eq, projections-eq, ortho-eq), sampled on the lattice.
* ``lattice``      - the time step: bilinear pull streaming (Sec. 2.4), moments,
                     Landau frame by the power method (Eq. eigen-eq), density
                     (Eq. density-eq), inversion, relaxation time, equilibrium and
                     Anderson-Witting relaxation (discrete Boltzmann equation,
                     Sec. 2.1), boundary rules and output fields (Eq. heat-eq2).
* ``bruteforce``   - a second, slower checker on tiny grids built from other
                     routes (numerical angular integration, dense interpolation
                     matrices, library eigen-solver).

Parity status: every function here is pinned by a test under ``tests/`` against
values printed in the paper, closed forms, invariants or brute force; none is
"parity unpinned".
"""
