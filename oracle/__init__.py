"""FP64 CPU oracle of the Chebyshev black-box FMM matvec phi = K sigma.

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, obviously checkable
restatement of the method (octree and lists of Section 2.1 / Definition 2.1,
Lagrange interpolation of Section 2.2, the four stages of Section 2.3, the
homogeneity and SVD compression of Section 2.5) plus the exact direct sum of
eq. (1)-(2).  It shares no code with the HIP library: only ``tests/``, the
smoke check and the CPU-baseline leg of the benchmark may import it.

Modules
  tree       octree, binning, Morton order, neighbour / interaction lists
  cheb       Chebyshev nodes, 1D/3D Lagrange bases, dense M2M operators
  operators  M2L operator sampling and SVD compression
  fmm        the matvec stages and the direct sum
  _native    plain C pair loops (kernel evaluation and summation)

Parity unpinned (no value in the paper to check against, see the tests for
the properties that are pinned): the absolute error per interpolation order
for each workload, and the exact weighting used by the cited SVD compression.
"""
from . import cheb, fmm, operators, tree  # noqa: F401
from ._native import build as build_native  # noqa: F401
