"""RandLU and RandSVD, the paper's fixed-rank comparison algorithms, in plain
NumPy float64 (test infrastructure only: nothing outside tests/, the smoke
check and the benchmark's CPU leg may import it).

Follows arXiv:2002.07138, Sec. 2:
  * RandLU: Alg. 3 with its steps 1-3 replaced by Alg. 4 (LU power iteration
    reorthogonalization), as Sec. 2.2 and Sec. 6 run it;
  * RandSVD: Alg. 1 with the power iteration of Alg. 2 (QR after every
    product).

Readings (each also listed in the design notes of the repository):
  R17 Alg. 4: the three-output ``[L, U, P] = lu(X)`` is getrf's P X = L U
      (L unit lower in pivot order); ``L = P^T L`` and the two-output
      ``[L, ~] = lu(X)`` are the row-permuted factor in X's own row order
      (reading R1 of the PowerLU oracle).  With p = 0 the algorithm is the
      single LU of A Omega.
  R18 Alg. 3 step 6, ``B Q = L_b U_b`` with column pivoting, is partial
      (row) pivoting of B^T: [L2, U2, Q] = lu(B^T), so L_b = U2^T and
      U_b = L2^T -- PowerLU's last step -- and A[p][:, q] ~ L U as in R5.
  R19 Alg. 3 step 5 forms the pseudo-inverse of L_y by the normal equations
      L_y^+ = (L_y^T L_y)^{-1} L_y^T, as the Remark after Alg. 4 states.
  R20 Alg. 1 returns a rank-l SVD; at target rank k the k leading singular
      triplets of B are kept (the rank-k comparisons of Sec. 6).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .powerlu import Factorization, LUResult, getrf, lur, thin_qr


# ----------------------------------------------------------------------------
# RandLU: Alg. 4 (power iteration with LU reorthogonalization) and Alg. 3.
# ----------------------------------------------------------------------------
@dataclass
class PowerLURecord:
    passes: int = 0
    lu_steps: list | None = None     # LUResult of every LU, in order


def lu_power(A: np.ndarray, Omega: np.ndarray, p: int,
             record: PowerLURecord | None = None) -> LUResult:
    """Alg. 4.  Returns the three-output LU of the last product (reading
    R17).  In exact arithmetic that product is Y T with Y = A (A^T A)^p Omega
    and T upper triangular and invertible, so its P and L are those of lu(Y)
    (its U is U_Y T).

    [L, U, P] = lu(A Omega); for p > 0: L = P^T L, then for i = 1..p:
    L = lu2(A^T L); then L = lu2(A L), except that the last product's LU
    keeps all three outputs."""
    A = np.asarray(A, dtype=np.float64)
    Omega = np.asarray(Omega, dtype=np.float64)
    m, n = A.shape
    if Omega.shape[0] != n:
        raise ValueError("Omega is n x l")
    rec = record if record is not None else PowerLURecord()
    rec.lu_steps = []
    f = getrf(A @ Omega)
    rec.passes = 1
    rec.lu_steps.append(f)
    if p == 0:
        return f
    V = np.empty_like(f.L)
    V[f.perm] = f.L                               # L = P^T L
    for i in range(1, p + 1):
        V, g = lur(A.T @ V)
        rec.passes += 1
        rec.lu_steps.append(g)
        Y = A @ V
        rec.passes += 1
        if i == p:
            f = getrf(Y)
            rec.lu_steps.append(f)
        else:
            V, g = lur(Y)
            rec.lu_steps.append(g)
    return f


def randlu(A: np.ndarray, k: int, Omega: np.ndarray, p: int) -> Factorization:
    """RandLU (Alg. 3 with Alg. 4 in place of its steps 1-3).  Omega is the
    caller's n x l Gaussian matrix, l = k + oversampling.  Makes 2p + 2 passes
    over A.

    Steps: P Y = L_y U_y (Alg. 4); L_y = L_y(:, :k); B = L_y^+ P A with
    L_y^+ = (L_y^T L_y)^{-1} L_y^T (reading R19); [L2, U2, Q] = lu(B^T)
    (reading R18); L = L_y U2^T, U = L2^T.  Returns the row order p (P's),
    the column order q and L, U with A[p][:, q] ~ L U."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = Omega.shape[1]
    if not (1 <= k <= l < min(m, n)):
        raise ValueError("need 1 <= k <= l < min(m, n)")
    rec = PowerLURecord()
    f = lu_power(A, Omega, p, rec)
    Ly = f.L[:, :k]                               # m x k, rows in P's order
    PA = A[f.perm]
    W = Ly.T @ Ly                                 # L_y^T L_y (k x k)
    B = np.linalg.solve(W, Ly.T @ PA)             # k x n
    f2 = getrf(B.T)
    L = Ly @ f2.U.T
    U = f2.L.T
    fac = Factorization(p=f.perm, q=f2.perm, L=L, U=U, rank=k, lu1=f, lu2=f2,
                        V=None, Y=None, Bt=B.T)
    fac.passes = rec.passes + 1
    fac.normA2 = float(np.sum(A * A))
    return fac


# ----------------------------------------------------------------------------
# RandSVD: Alg. 2 (power iteration with QR after every product) and Alg. 1.
# ----------------------------------------------------------------------------
def qr_power(A: np.ndarray, Omega: np.ndarray, p: int) -> np.ndarray:
    """Alg. 2: Q = qr(A Omega); for i = 1..p: Q = qr(A^T Q); Q = qr(A Q).
    An orthonormal m x l basis of Range(A (A^T A)^p Omega) in exact
    arithmetic; 2p + 1 passes over A."""
    A = np.asarray(A, dtype=np.float64)
    Q = thin_qr(A @ np.asarray(Omega, dtype=np.float64))
    for _ in range(p):
        Q = thin_qr(A.T @ Q)
        Q = thin_qr(A @ Q)
    return Q


@dataclass
class SVDResult:
    U: np.ndarray          # (m, k) orthonormal columns
    s: np.ndarray          # (k,) singular values, non-increasing
    V: np.ndarray          # (n, k) orthonormal columns
    U_all: np.ndarray      # the rank-l factors before truncation (reading R20)
    s_all: np.ndarray
    V_all: np.ndarray
    Q: np.ndarray          # the basis of Alg. 2
    passes: int = 0


def randsvd(A: np.ndarray, k: int, Omega: np.ndarray, p: int) -> SVDResult:
    """RandSVD (Alg. 1 with Alg. 2): B = Q^T A (l x n); B = U_hat S V^T (the
    library SVD serves as that step); U = Q U_hat; the k leading triplets
    are kept (reading R20).  2p + 2 passes over A."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = Omega.shape[1]
    if not (1 <= k <= l < min(m, n)):
        raise ValueError("need 1 <= k <= l < min(m, n)")
    Q = qr_power(A, Omega, p)
    B = Q.T @ A
    Uh, s, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ Uh
    V = Vt.T
    return SVDResult(U=U[:, :k], s=s[:k], V=V[:, :k], U_all=U, s_all=s, V_all=V, Q=Q,
                     passes=2 * p + 2)


def svd_relative_residual(A: np.ndarray, U: np.ndarray, s: np.ndarray, V: np.ndarray) -> float:
    """||A - U diag(s) V^T||_F / ||A||_F in float64 (eq. (error), Sec. 6.2)."""
    A = np.asarray(A, dtype=np.float64)
    R = A - (np.asarray(U, np.float64) * np.asarray(s, np.float64)) @ np.asarray(V, np.float64).T
    return float(np.sqrt(np.sum(R * R)) / np.sqrt(np.sum(A * A)))
