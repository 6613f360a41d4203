"""CPU FP64 oracle for the mixed-precision Newton refinement of large sparse
CAREs  A^T X + X A - X B B^T X + C^T C = 0,  X ~ Z Z^T  (eq. (1.1)).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy/SciPy implementation used to check the HIP library.  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it;
the product path (the C-ABI library and its Python binding) never does, and
the two share no code.  Every function cites the passage of the paper it
follows.

Modules
  riccati  - Riccati operator, dense Schur and dense Newton-Kleinman solvers
  lowrank  - Algorithm 1 (residual factor decomposition), Algorithm 2
             (solution factor decomposition), factored X-differences
  adi      - shifted solves with SMW (Sec. 4) and residual-based LR-ADI
  care     - NLR-ADI initial solve and Framework 1 (mixed-precision Newton IR)
  shifts   - Penzl-style heuristic shift selection from Ritz values
  ilu      - multicolour ILU(0) of A^T + p I (the GMRES preconditioner of Sec. 5)
"""
from . import riccati, lowrank, adi, care, ilu  # noqa: F401
