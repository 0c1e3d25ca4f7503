"""Plain FP64 CPU oracle for the additive Schwarz / SIPG / multigrid hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code,
tables or constants with the HIP library; the only thing both sides consume is
the seeded input generator in ``synthetic/`` (which holds none of the method's
arithmetic).

What it computes is the plain definition of the method (Witte, Arndt,
Kanschat, "Fast tensor product Schwarz smoothers for high-order discontinuous
Galerkin methods"):

* ``basis``     Gauss-Lobatto Lagrange basis and Gauss quadrature (Sec. 3 intro).
* ``mesh``      rectilinear Cartesian meshes, cell-major lexicographic DoFs
                (Sec. 2.1, eq. multiindex).
* ``sipg``      the global SIPG matrix assembled by d-dimensional quadrature
                directly from eq. (bfsipg) with the 1/sqrt(2) average
                (eq. jumpavgscalar, avgbdry) and penalty eq. (penalty).
* ``schwarz``   cell and vertex-patch subspaces, exact local solvers
                A_j = R_j A R_j^T factored by dense LU (eq. ritzproj), the
                additive smoother (eq. additiveschwarz, Alg. addsmoother).
* ``multigrid`` embedding prolongation / transpose restriction and the V-cycle
                (Alg. gmg, Sec. 2.2) with a dense-LU coarse solve.
* ``krylov``    textbook preconditioned CG.
* ``onedim``    a separate 1-D path (Sec. 3.2 formulas) used only by tests to
                pin the separability identity and to build exact full-size
                solutions by global fast diagonalisation (Lynch et al.).
* ``sampled``   the same definitions restricted to a few cells of a large mesh
                (residual and one smoothing step need only a bounded
                neighbourhood), for parity checks at full problem size.
* ``tangent``   forward-mode derivatives of the V-cycle iteration with respect
                to the right-hand side, the damping and the penalty factor of
                every level, propagated step by step.
* ``mapped``    SIPG on multilinearly mapped cells (Sec. 4): the assembled
                matrix, load and boundary terms by quadrature, the Cartesian
                surrogate cell solvers (eq. avglength), the surrogate
                additive smoother and the mapped-mesh V-cycle.

Functions with no independent pin say "parity unpinned" in their docstring.
"""
