"""FP64 CPU oracle for PowerLU and PowerLU_FP (Zhang & Mascagni, "Pass-Efficient
Randomized LU Algorithms for Computing Low-Rank Matrix Approximation",
arXiv:2002.07138).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the paper's algorithms in NumPy float64.  It exists to check the
HIP library against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path (the C-ABI
library and its Python binding) never imports, calls or links it, and it shares
no code with that path.

Modules
-------
powerlu   GETRF with partial pivoting, the LU reorthogonalization, thin QR,
          the generalized power iteration (Alg. 7), PowerLU (Alg. 5),
          the error indicator and rank rules (Thm 4.3, Alg. 8, Alg. 11),
          PowerLU_FP (Alg. 9) and the relative residual (eq. "error", Sec. 6.2).
lowp      bfloat16 and block-scaled FP8 E4M3 operand rounding for the
          precision form of the passes.
philox    Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
          Box-Muller transform, for the seeded Gaussian test matrix.
baselines RandLU (Alg. 3 with Alg. 4) and RandSVD (Alg. 1 with Alg. 2), the
          paper's fixed-rank comparison algorithms.

Every function states the passage it follows.  Parity status of each function
is listed in the module docstrings; none is "parity unpinned" except where a
docstring says so.
"""
