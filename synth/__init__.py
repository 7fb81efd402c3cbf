"""Seeded synthetic inputs for PowerLU / PowerLU_FP.

This module holds input generators only: it contains none of the method's
arithmetic, and both the oracle checks and the HIP library's callers draw
their matrices from here.  Everything is NumPy on the host, float64, rounded
to float32 where a device-shaped input is wanted.

Matrix families
---------------
* ``paper_type(t, n, seed)``: the three accuracy-test families of Sec. 6.2:
  A = U Sigma V^T with random orthonormal U, V and
  Type 1 (slow decay)      sigma_k = k^-2,
  Type 2 (fast decay)      sigma_k = exp(-k/7),
  Type 3 (S-shaped decay)  sigma_k = 1e-4 + 1/(1 + exp(k - 30)).
  ``paper_type_family(n, seed)`` builds several types on one pair of
  factors (Table 1's size, n = 8000, without three pairs of n x n QRs).
* ``lowrank_plus_noise``: X diag(sigma) Y^T + noise with X, Y the Q factors
  of seeded Gaussian matrices, the workload shapes used for measurement
  (square 2000, 20000, 32768; 30000 x 20000; mixed request sizes).
* ``gaussian_omega``: the N(0,1) test matrix (Sec. 1, Alg. 7).
* ``sprand_csr``: sparse matrices like MATLAB's sprand (uniform values at
  random positions, Sec. 6.1's sparse experiment), in compressed rows;
  ``csr_dense`` expands them.
* ``crafted_tie_matrix``: tall matrices on which partial pivoting meets exact
  ties at every step while float32 elimination stays exact (pivot tie-break
  tests).

Seed scheme: ``seed = 1000 * workload + role`` with role 0 the left factor,
1 the right factor, 2 the noise, 3 + s the Gaussian test matrix of run s.
"""

from .generators import (  # noqa: F401
    spectrum,
    orthonormal,
    paper_type,
    paper_type_family,
    lowrank_factors,
    lowrank_plus_noise,
    gaussian_omega,
    sprand_csr,
    csr_dense,
    crafted_tie_matrix,
    WORKLOADS,
    workload_matrix_factors,
    workload_matrix,
    workload_slice,
    request_stream,
)
