"""FP64 CPU oracle for the spectral-element Poisson operator path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
CPU-baseline leg of the benchmark may import anything from here.  The GPU
library never calls it, and this package imports nothing from the GPU library.

Every routine is a plain, slow, checkable statement of what the method
computes, in float64 (unless a routine emulates a reduced precision on purpose),
citing the passage of the paper (arXiv 2506.20994, "Portable High-Performance
Kernel Generation for a CFD Code with DaCe") it follows.  Where the paper is
silent the docstring names the reading taken.

Modules
  gll       GLL nodes, weights, Lagrange basis and derivative matrix (Sec. 3, Eq. 2)
  mesh      periodic box mesh: node positions, deformation, global numbering (Sec. 3, Eq. 3)
  geometry  isoparametric Jacobian, geometric factors G_ab, mass weights (Sec. 3, Eq. 1)
  ax        the element operator: node-by-node quadrature form, einsum form, dense Kronecker form
  gs        gather-scatter via bincount, multiplicity (Sec. 2.1)
  assemble  dense assembled matrix, Jacobi diagonal
  solve     textbook Jacobi-PCG, mixed-precision refinement, flexible CG
  quant     round-to-nearest-even float32 / bfloat16 emulation
  mlp       per-element MLP forward/backward and Adam, and their bfloat16-storage emulation
  mg        multigrid V-cycle: p- and h-transfers, Chebyshev-Jacobi smoothing, dense coarsest solve
  cref      ctypes loader for sem_ref.c: the path in plain C (CPU baseline, 32^3 reference solutions)

Parity status of each function is stated in its docstring; anything without
an independent pin says "parity unpinned".
"""
