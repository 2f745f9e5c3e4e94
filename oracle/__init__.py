"""Plain FP64 CPU oracle for additive-multigrid MPCG (test infrastructure).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it.  It
shares no code with the HIP path: it builds its own operators, transfers,
Galerkin hierarchy, smoother, pseudo-inverse and Krylov loop with numpy and
scipy.sparse, in float64, slowly and step by step in the paper's order.

Modules
  operators  finite-difference operator, 1-D/tensor linear interpolation,
             full-weighting restriction, Galerkin products (Sec. 2.1)
  hierarchy  the nested level list V_0 c ... c V_L (Sec. 2.1)
  smoother   damped-Jacobi smoothing iteration, eq. (2)
  mpcg       additive-MG corrections as a direction block, the pseudo-inverse
             step, eq. (4) and Algorithm 1 (Sec. 2.2)
  pcg        textbook preconditioned CG (a pin, and the outer loop of the
             comparators)
  comparators  the comparison methods of Sec. 3: additive MG-PCG and
             MG(V)-PCG (one V-cycle as preconditioner)
  cnn        FP64 U-Net forward/backward for the learned direction

Every function is pinned by the tests against closed forms, invariants, dense
brute force or textbook routines; anything unpinned says so in its docstring.
"""
from . import operators, hierarchy, smoother, mpcg, pcg, comparators  # noqa: F401
