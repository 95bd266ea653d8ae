"""CPU oracle for the robust LOBPCG path (Duersch, Shao, Yang, Gu, arXiv 1704.07458).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, FP64 NumPy/SciPy
restatement of the paper's algorithms, used to check the HIP path.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  The product path never calls it and shares no code with it.

Modules:
  lobpcg         Algorithms 2, 3, 4, 5, 6, 7, 8 and criterion (9).
  adjoint        dense reference gradient of eigenpairs and the block projected
                 solve for eigenvector adjoints.
  brute          cyclic Jacobi eigensolver for small dense matrices.
  closed_forms   closed-form spectra of the synthetic pencils.
"""
