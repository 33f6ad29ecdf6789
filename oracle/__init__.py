"""Plain, slow, FP64 CPU oracle for the cell-wise Q_p Laplacian hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP path: the 1D rules, the
element matrices, the patch operators and the solver are written here from
their definitions.

What it computes, each from its plain definition:

* ``basis``   -- Gauss-Lobatto-Legendre nodes, Gauss-Legendre rule, Lagrange
  basis values and derivatives (textbook definitions).
* ``mesh``    -- graded Cartesian hexahedral mesh, global node numbering and
  the cell-to-global node map (the gather operator G of Section 2.1).
* ``element`` -- element stiffness and mass matrices by plain 3D quadrature
  (not by Kronecker factorisation).
* ``operators`` -- G, G^T, the direct stiffness summation S = G G^T
  (Eq. of Section 3.3), the Dirichlet-masked global and cell-wise operator
  apply, sparse global assembly for small meshes.
* ``patches`` -- vertex-patch (2x2x2 cells) operators assembled from the
  eight element matrices, inverted by dense LU, and the additive Schwarz
  preconditioner built from them (the overlapping Schwarz patch smoother the
  paper names in its Remark "Beyond DSS").
* ``twolevel`` -- the Schwarz smoother plus an exact coarse correction on the
  Q_1 space of the same mesh (prolongation by interpolation, Galerkin coarse
  operator, sparse LU): the two-level member of the multigrid family the
  paper's solver is built for (Remark after the equivalence theorem).
* ``multiblock`` -- multi-block meshes (blocks glued along whole faces in any
  orientation, Section 4.2): nodes identified geometrically, DSS = G G^T.
* ``solver``  -- damped Richardson smoothing on additive Schwarz and the
  (flexible) preconditioned conjugate gradient of the paper's Algorithm
  "Communication-Free (F)PCG", run on assembled global vectors, which the
  equivalence theorem of Section 3.2 says the cell-wise solve reproduces.

Readings where the paper is silent (node set, quadrature, Dirichlet
treatment, damping) are listed in the repository's design notes; the oracle
follows exactly those readings.
"""
from . import basis, mesh, element, multiblock, operators, patches, solver, twolevel  # noqa: F401
