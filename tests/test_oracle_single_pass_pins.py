"""Pins of the oracle's single-pass randomized LU (Alg. 10, Sec. 5).  CPU only.

What fixes the result independently of the oracle's code:
  * exact recovery: a matrix of rank k is reproduced, A[p][:, q] = L U;
  * the plain definition: L U equals (A V V^T)[p][:, q] for V an orthonormal
    basis of Range(A^T Omega) (G pinv(G) is the projector onto Range(G));
  * so its residual equals PowerLU's with v = 2 and no oversampling on the
    same Omega (Alg. 7 with v = 2 gives V = qr(A^T Omega));
  * structure: U unit upper trapezoidal with |u| <= 1, L lower trapezoidal;
  * a planted mistake (U = L^T read literally from the listing's last line)
    breaks the reconstruction.
"""

import numpy as np
import pytest

from oracle import powerlu as O
from synth import lowrank_plus_noise, spectrum


def _exact_rank(m, n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((m, k)) @ rng.standard_normal((k, n))


def test_exact_recovery():
    A = _exact_rank(90, 70, 12, 1)
    Om = np.random.default_rng(2).standard_normal((90, 12))
    f = O.single_pass_lu(A, 12, Om)
    assert np.max(np.abs(A[f.p][:, f.q] - f.L @ f.U)) <= 1e-10 * np.max(np.abs(A))


@pytest.mark.parametrize("m,n,k", [(120, 100, 10), (80, 150, 25)])
def test_equals_projection_onto_range_of_AtOmega(m, n, k):
    A = lowrank_plus_noise(m, n, spectrum("exp", min(m, n) - 1, tau=8.0), 3, 4, 1e-3, 5,
                           dtype=np.float64)
    Om = np.random.default_rng(6).standard_normal((m, k))
    f = O.single_pass_lu(A, k, Om)
    V, _ = np.linalg.qr(A.T @ Om)
    approx = A @ V @ V.T
    assert np.max(np.abs(approx[f.p][:, f.q] - f.L @ f.U)) <= 1e-9 * np.max(np.abs(A))
    # the same approximation as PowerLU with v = 2, l = k (Alg. 7: V = qr(A^T Omega))
    g = O.powerlu(A, k, Om, 2)
    r1 = O.relative_residual(A, f.p, f.q, f.L, f.U)
    r2 = O.relative_residual(A, g.p, g.q, g.L, g.U)
    assert abs(r1 - r2) <= 1e-10 * r2
    # structure (Alg. 10's ENSURE, reading R10)
    U = f.U
    assert np.allclose(np.diag(U[:, :k]), 1.0) and np.all(np.tril(U[:, :k], -1) == 0.0)
    assert np.max(np.abs(U)) <= 1.0 + 1e-12
    assert np.all(np.triu(f.L[:k], 1) == 0.0)


def test_planted_listing_reading_fails():
    A = _exact_rank(60, 50, 8, 7)
    Om = np.random.default_rng(8).standard_normal((60, 8))
    f = O.single_pass_lu(A, 8, Om)
    wrong_U = f.L.T                     # "U = L^T" taken literally
    assert np.max(np.abs(A[f.p][:, f.q] - f.L @ wrong_U[:, :50])) > 1e-3 * np.max(np.abs(A))
