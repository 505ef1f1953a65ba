"""FP64 CPU oracle for the coupled poroelasticity / elasticity solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` use it.  It shares no code with the HIP path.

What it computes is the plain definition of one backward-Euler time step of
the paper's fully discrete problem: the global block system of eq.
(linalg-system) in Section 2.5, assembled from the bilinear forms (aD), (bD),
(af) of Section 2.3 on the P_k-P1-P1-P1 / P_k-P1 spaces of Section 2.4, with
the Lagrange multiplier gluing the displacement on the interface.  Theorem 3.1
and the equivalence stated for system (sim-feti) in Section 3.2 say that the
FETI interface solve reaches exactly this discrete solution, so the oracle
solves the same system monolithically with a sparse direct factorisation
(SciPy SuperLU) instead of reproducing the FETI algorithm.

Modules
-------
fem         P1/P2 Lagrange elements, the 7-point degree-5 quadrature rule,
            element matrices of the forms (aD), (bD), (af), the L2 mass and
            the closed-form edge masses of the boundary terms.
mesh        structured right-triangle mesh of the unit square and regions.
problem     material constants (Section 2.2 kappas, Table 3 Lame formulas)
            and closed-form loads derived symbolically from eqs. (2.1)-(2.3).
monolithic  global assembly of eq. (linalg-system), Dirichlet lifting,
            SuperLU, time stepping, L-infinity(L2) errors; loads given as
            nodal data (body force, source, traction and flux on boundary
            edges, eqs. (vf1), (vf3), (vf4)) through element and edge masses.
indexing    an independent statement of the subdomain numbering and the
            signed Boolean jump maps used by the FETI path (bit-exact checks).
local       the torn per-subdomain matrices and right-hand sides, and the
            plain-definition references the unit tests compare with: the
            interface Schur complement of eq. (reduced-system) and the
            generalised inverse of a floating subdomain.
dual_primal the dual-primal gluing (primal xi / p and corner DOFs, multipliers on the
            other u / eta DOFs): partially assembled matrix, interface operator and
            right-hand side, solution and primal coarse matrix, by sparse direct solves.
decoupled   the explicit fluid step of the decoupled mass balance (Remark after eq.
            (linalg-system)) and the momentum balance alone.
mlp         FP64 forward/backward of the warm-start MLP (BF16 weights, the
            specification's reference) and Adam, for the gradient checks.
"""
