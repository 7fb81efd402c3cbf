"""PowerLU / PowerLU_FP in plain NumPy float64 (test infrastructure only).

Follows arXiv:2002.07138:
  * Alg. 5 (PowerLU) with steps 1-2 replaced by Alg. 7 (generalized power
    iteration reorthogonalization, any pass count v >= 2), Sec. 3;
  * Thm 4.2 / Thm 4.3 (error indicator without updating A), Alg. 8 (blocked
    adaptive rank determination), Alg. 11 (per-column refinement) and
    Alg. 9 (PowerLU_FP), Sec. 4 and Sec. 6.4;
  * relative Frobenius error, eq. (error), Sec. 6.2.

Readings of passages that are silent or garbled (each is also listed in the
design notes of the repository):
  R1  ``[V, ~] = lu(X)`` (MATLAB two-output form) returns the row-permuted unit
      lower factor P^T L in X's own row order (Alg. 4 writes L = P^T L
      explicitly).  -> ``lur``.
  R2  ``[V, ~] = qr(X)`` is the thin (economy) QR: Alg. 7's ENSURE line gives
      V as n x l.  -> ``thin_qr``.
  R3  For even v the first Gaussian matrix is m x l (Sec. 3.4 item 1 and
      Alg. 7), whatever Thm 3.3's statement of its size says.
  R4  Partial pivoting picks the first maximum in the current (already
      swapped) row order, as LAPACK's getrf does; a zero pivot column is left
      unscaled and the first such step is reported.
  R5  ``PAQ ~ LU`` with Q from ``[L2, U2, Q] = lu(B^T)`` means, in index form,
      A[p][:, q] ~ L @ U with p, q the row orders of the two LU steps.
  R6  The stopping test is E <= eps^2 ||A||_F^2 everywhere (Alg. 8's form).
  R7  Alg. 11's column loop is read as: k = the first column j (1-based) whose
      running indicator E_j = ||A||^2 - sum_{i<=j} ||G(:,i)||^2 meets R6.
  R8  When l columns are not enough, the rank-l result is returned with
      ``tol_reached = False`` (the Remark after Alg. 8 suggests a restart; that
      is not part of this oracle).
  R15 Restart (the Remark after Alg. 8): when a round's l columns miss the
      tolerance, a fresh Gaussian matrix is drawn and Alg. 7 runs on the
      remainder A - A V V^T; the new block is projected out of V twice and
      re-orthonormalized, and the indicator continues over all columns.
  R16 Single-pass LU (Alg. 10): Omega is m x k as the listing sizes it (the
      text's n x k does not conform with A^T Omega); U = L2^T as the text
      derives (the listing's last line reads L^T); pinv(G^T) is the
      Moore-Penrose inverse of the full-row-rank k x n matrix G^T.
  R13 Precision form (not in the paper, which computes in float64): the v - 1
      passes of Alg. 7 take operands rounded to a narrower format (module
      ``lowp``) and accumulate exactly; the final product with A, the LU and
      QR steps and the indicator stay exact.  With exact_last, the last of
      the v - 1 passes (the one feeding the final QR) is exact too: a
      refinement pass that re-projects the rounded iterate with the exact A.
  R22 Two exact closing passes (exact_tail = 2): the last two of the v - 1
      passes of Alg. 7 -- the A X and A^T Y of the loop's final iteration --
      are exact, one exact power step applied to the basis the rounded
      passes found.  This is the stronger refinement taken when one exact
      pass leaves the rounded form's residual above 1.05x the exact one's
      (the E4M3 form at rank 200 of the 32768^2 workload).

Pins: see tests/test_oracle_pins.py (GETRF against LAPACK and the textbook
definition, crafted ties, zero columns; thin QR against exact arithmetic;
Alg. 7 against the explicit Krylov basis at 60 digits; the assembly identity;
exact recovery; Eckart-Young; Thm 3.2; Thm 4.1/4.3 by brute force; Table 1's
truncated-SVD ranks through the rank rule).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


# ----------------------------------------------------------------------------
# LU with partial pivoting (the paper's lu(.), Sec. 2 notation; Golub & Van
# Loan, Matrix Computations, Alg. 3.4.1 "outer product LU with partial
# pivoting").
# ----------------------------------------------------------------------------
@dataclass
class LUResult:
    perm: np.ndarray      # (m,) int: X[perm] == L @ U  (row order after pivoting)
    L: np.ndarray         # (m, c) unit lower trapezoidal
    U: np.ndarray         # (c, c) upper triangular
    ipiv: np.ndarray      # (c,) int: at step j, rows j and ipiv[j] were swapped
    gaps: np.ndarray      # (c,) relative gap between the two largest |candidates|
    zero_step: int        # first step with an exactly zero pivot column, or -1


def getrf(X: np.ndarray) -> LUResult:
    """Unblocked right-looking LU with partial pivoting of an m x c matrix
    (m >= c), in float64.

    Step j (0-based): pick r = j + (first index of max |W[j:, j]|) in the
    current row order (reading R4), swap rows j and r, divide the column below
    the pivot by the pivot and subtract the outer product from the trailing
    block.  A zero pivot column is neither swapped nor scaled.
    """
    W = np.array(X, dtype=np.float64, copy=True)
    m, c = W.shape
    if m < c:
        raise ValueError("getrf oracle expects m >= c")
    perm = np.arange(m)
    ipiv = np.zeros(c, dtype=np.int64)
    gaps = np.zeros(c, dtype=np.float64)
    zero_step = -1
    for j in range(c):
        cand = np.abs(W[j:, j])
        r_rel = int(np.argmax(cand))          # first maximum in current order
        top = cand[r_rel]
        if cand.size > 1:
            rest = np.delete(cand, r_rel)
            second = rest.max()
            gaps[j] = (top - second) / top if top > 0 else 0.0
        else:
            gaps[j] = 1.0
        r = j + r_rel
        ipiv[j] = r
        if r != j:
            W[[j, r], :] = W[[r, j], :]
            perm[[j, r]] = perm[[r, j]]
        piv = W[j, j]
        if piv != 0.0:
            W[j + 1:, j] /= piv
            W[j + 1:, j + 1:] -= np.outer(W[j + 1:, j], W[j, j + 1:])
        elif zero_step < 0:
            zero_step = j
    L = np.tril(W, -1)
    L[np.arange(c), np.arange(c)] = 1.0
    U = np.triu(W[:c, :c])
    return LUResult(perm, L, U, ipiv, gaps, zero_step)


def lur(X: np.ndarray) -> tuple[np.ndarray, LUResult]:
    """The paper's ``[V, ~] = lu(X)``: V = P^T L, the unit lower factor placed
    back in X's own row order (reading R1; Alg. 4 states L = P^T L)."""
    f = getrf(X)
    V = np.empty_like(f.L)
    V[f.perm] = f.L
    return V, f


def thin_qr(X: np.ndarray) -> np.ndarray:
    """The paper's ``[V, ~] = qr(X)`` read as the thin QR (reading R2).
    Householder QR (LAPACK geqrf + orgqr) serves as the library step; the
    column signs are immaterial to everything downstream (PowerLU's output is
    invariant under V -> V D with D = diag(+-1))."""
    Q, _ = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    return Q


# ----------------------------------------------------------------------------
# Alg. 7: generalized power iteration reorthogonalization (Sec. 3.4).
# ----------------------------------------------------------------------------
@dataclass
class RangeRecord:
    passes: int = 0
    lu_steps: list = field(default_factory=list)   # LUResult of each LU reorth
    v_final: np.ndarray | None = None


def range_basis(A: np.ndarray, Omega: np.ndarray, v: int,
                record: RangeRecord | None = None, pass_round=None,
                exact_last: bool = False, exact_tail: int = 0) -> np.ndarray:
    """Alg. 7.  Returns an orthonormal n x l basis V of (A^T A)^P A^T Omega
    (v even, Omega m x l) or (A^T A)^P Omega (v odd, Omega n x l), with
    P = floor((v - 1) / 2).  Makes v - 1 passes over A; the caller's final
    product with A is the v-th.

    v even: X = A^T Omega, then LU reorth if v > 2 else QR.
    v odd:  V = Omega.
    Loop i = 1..P: V = lur(A V); V = qr(A^T V) if i == P else lur(A^T V).

    pass_round (precision form, reading R13): when given, every one of these
    v - 1 products takes rounded operands, pass_round(A, axis) and
    pass_round(X, 0), with axis the contraction axis of A (1 for A X, 0 for
    A^T X), and is accumulated exactly.  Nothing else is rounded.
    exact_last: the last of the v - 1 products (the one whose result the
    final QR orthonormalizes) is exact even when pass_round is given.
    exact_tail: the last exact_tail of the v - 1 products are exact
    (exact_last is exact_tail = 1; 2 makes the closing A X, A^T Y pair one
    exact power step on the rounded iterate, reading R22).
    """
    if v < 2:
        raise ValueError("v >= 2 (Alg. 7 REQUIRE)")
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    P = (v - 1) // 2
    rec = record if record is not None else RangeRecord()
    tail = max(int(exact_tail), 1 if exact_last else 0)

    def rounded():         # is the product about to be taken a rounded one?
        if pass_round is None:
            return False
        return rec.passes - start < v - 1 - tail

    def times(X):          # A X, the products of the loop
        if not rounded():
            return A @ X
        return pass_round(A, 1) @ pass_round(X, 0)

    def times_t(X):        # A^T X
        if not rounded():
            return A.T @ X
        return pass_round(A, 0).T @ pass_round(X, 0)

    start = rec.passes

    if v % 2 == 0:
        if Omega.shape[0] != m:
            raise ValueError("even v needs an m x l Gaussian matrix (reading R3)")
        X = times_t(Omega)
        rec.passes += 1
        if v > 2:
            V, f = lur(X)
            rec.lu_steps.append(f)
        else:
            V = thin_qr(X)
    else:
        if Omega.shape[0] != n:
            raise ValueError("odd v needs an n x l Gaussian matrix")
        V = np.array(Omega, dtype=np.float64, copy=True)
    for i in range(1, P + 1):
        Y = times(V)
        rec.passes += 1
        V, f = lur(Y)
        rec.lu_steps.append(f)
        X = times_t(V)
        rec.passes += 1
        if i == P:
            V = thin_qr(X)
        else:
            V, f = lur(X)
            rec.lu_steps.append(f)
    assert rec.passes == v - 1
    rec.v_final = V
    return V


# ----------------------------------------------------------------------------
# Alg. 5 steps 3-8 (shared with Alg. 9 steps 2-6).
# ----------------------------------------------------------------------------
@dataclass
class Factorization:
    p: np.ndarray          # (m,) row order:    A[p][:, q] ~ L @ U   (reading R5)
    q: np.ndarray          # (n,) column order
    L: np.ndarray          # (m, k) lower trapezoidal (diag = diag(U2), not unit)
    U: np.ndarray          # (k, n) unit upper trapezoidal, |u_ij| <= 1
    rank: int
    lu1: LUResult | None = None
    lu2: LUResult | None = None
    V: np.ndarray | None = None
    Y: np.ndarray | None = None
    Bt: np.ndarray | None = None
    G: np.ndarray | None = None        # A V over all kept columns (fixed precision)
    normA2: float = 0.0
    E: np.ndarray | None = None        # running indicator E_j (fixed precision)
    tol_reached: bool = True
    passes: int = 0


def assemble(A: np.ndarray, Vk: np.ndarray, Y: np.ndarray | None = None) -> Factorization:
    """Alg. 5 steps 3-8 (eq. plu, firstlu, secondlu, powerlufinal):
    Y = A Vk; [L1, U1, P] = lu(Y); B = U1 Vk^T; [L2, U2, Q] = lu(B^T);
    L = L1 U2^T; U = L2^T."""
    A = np.asarray(A, dtype=np.float64)
    k = Vk.shape[1]
    if Y is None:
        Y = A @ Vk
    f1 = getrf(Y)
    Bt = Vk @ f1.U.T                    # B^T = Vk U1^T  (n x k)
    f2 = getrf(Bt)
    L = f1.L @ f2.U.T                   # m x k
    U = f2.L.T                          # k x n
    return Factorization(p=f1.perm, q=f2.perm, L=L, U=U, rank=k, lu1=f1,
                         lu2=f2, V=Vk, Y=Y, Bt=Bt)


def powerlu(A: np.ndarray, k: int, Omega: np.ndarray, v: int,
            pass_round=None, exact_last: bool = False, exact_tail: int = 0) -> Factorization:
    """PowerLU (Alg. 5 with Alg. 7 in place of steps 1-2).  Omega is the
    caller's Gaussian matrix: m x l for even v, n x l for odd v, l = k + q.
    pass_round, exact_last: precision form of the v - 1 range passes (see
    range_basis); the final product Y = A V_k is always exact."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = Omega.shape[1]
    if not (1 <= k <= l < min(m, n)):
        raise ValueError("need 1 <= k <= l < min(m, n)")
    rec = RangeRecord()
    V = range_basis(A, Omega, v, rec, pass_round, exact_last, exact_tail)
    fac = assemble(A, V[:, :k])
    fac.passes = rec.passes + 1
    fac.normA2 = float(np.sum(A * A))
    return fac


# ----------------------------------------------------------------------------
# Sec. 4: error indicator, Alg. 8, Alg. 11, Alg. 9.
# ----------------------------------------------------------------------------
def indicator(normA2: float, colnorm2: np.ndarray) -> np.ndarray:
    """Thm 4.3: E_j = ||A||_F^2 - sum_{i<=j} ||A v_i||^2, accumulated in
    column order (returned for j = 1..l)."""
    E = np.empty(len(colnorm2), dtype=np.float64)
    acc = float(normA2)
    for j, c in enumerate(colnorm2):
        acc -= float(c)
        E[j] = acc
    return E


def rank_rule(normA2: float, colnorm2: np.ndarray, eps: float, b: int,
              column_mode: bool) -> tuple[int, bool]:
    """Alg. 8 (blocks of b columns) or Alg. 11 (per column) stopping rule on
    the indicator of Thm 4.3, with the test E <= eps^2 ||A||^2 (reading R6/R7).
    Returns (k, tol_reached).  normA2 == 0 gives k = 0."""
    if normA2 == 0.0:
        return 0, True
    acc = eps * eps * normA2
    l = len(colnorm2)
    E = float(normA2)
    for t1 in range(0, l, b):
        block = colnorm2[t1:t1 + b]
        if column_mode:
            for jj, c in enumerate(block):
                E -= float(c)
                if E <= acc:
                    return t1 + jj + 1, True
        else:
            s = 0.0
            for c in block:
                s += float(c)
            E -= s
            if E <= acc:
                return t1 + len(block), True
    return l, False


def powerlu_fp(A: np.ndarray, eps: float, b: int, Omega: np.ndarray, v: int,
               column_mode: bool = True, pass_round=None,
               exact_last: bool = False, restart_omegas=(), exact_tail: int = 0) -> Factorization:
    """PowerLU_FP (Alg. 9) on top of Alg. 8 (block rule) or Alg. 11 (column
    rule).  l = Omega.shape[1] must be a multiple of b (Sec. 4.1, l = s b).
    pass_round: precision form of the v - 1 range passes; G = A V is exact.

    restart_omegas (reading R15 of the Remark after Alg. 8): when the l
    columns of a round do not reach the tolerance, the next round draws a
    fresh Gaussian matrix (the next entry, same shape as Omega) and runs
    Alg. 7 on the remainder R = A - A V V^T of the columns found so far.
    The new block is orthogonalized against V (Range(R^T) is orthogonal to
    V in exact arithmetic; projecting twice, then a thin QR, keeps that in
    floating point), its G block is A times it, and the indicator of
    Thm 4.3 continues over the concatenated columns, blocks of b included.
    The rounds stop when the tolerance is met or the entries run out."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    l = Omega.shape[1]
    rounds = 1 + len(restart_omegas)
    if l % b != 0 or not (l * rounds < min(m, n)):
        raise ValueError("need b | l and (rounds * l) < min(m, n)")
    normA2 = float(np.sum(A * A))
    rec = RangeRecord()
    V = range_basis(A, Omega, v, rec, pass_round, exact_last, exact_tail)
    G = A @ V
    colnorm2 = np.sum(G * G, axis=0)
    k, ok = rank_rule(normA2, colnorm2, eps, b, column_mode)
    used = 1
    for Om in restart_omegas:
        if ok:
            break
        used += 1
        R = A - G @ V.T                                  # remainder A (I - V V^T)
        Vr = range_basis(R, np.asarray(Om, dtype=np.float64), v, RangeRecord(),
                         pass_round, exact_last, exact_tail)
        for _ in range(2):                               # against the columns kept so far
            Vr = Vr - V @ (V.T @ Vr)
        Vr = thin_qr(Vr)
        Gr = A @ Vr
        V = np.concatenate([V, Vr], axis=1)
        G = np.concatenate([G, Gr], axis=1)
        colnorm2 = np.sum(G * G, axis=0)
        k, ok = rank_rule(normA2, colnorm2, eps, b, column_mode)
    E = indicator(normA2, colnorm2)
    if k == 0:
        fac = Factorization(p=np.arange(m), q=np.arange(n), L=np.zeros((m, 0)),
                            U=np.zeros((0, n)), rank=0)
    else:
        fac = assemble(A, V[:, :k], Y=G[:, :k])
    fac.normA2 = normA2
    fac.E = E
    fac.tol_reached = ok
    fac.passes = (rec.passes + 1) * used       # v passes over A (or its remainder) per round
    fac.V = V
    fac.G = G
    return fac


# ----------------------------------------------------------------------------
# Sec. 5: single-pass randomized LU (Alg. 10).
# ----------------------------------------------------------------------------
def single_pass_lu(A: np.ndarray, k: int, Omega: np.ndarray) -> Factorization:
    """Alg. 10.  Omega is m x k (the listing's size; reading R16).  G = A^T Omega
    and H = A G are the two products the one pass over A yields (the Remark
    after the derivation streams the columns of A once, forming G(i,:) and
    the outer product A(:,i) G(i,:) together); here they are plain products.
    [L1, U1, P] = lu(H); the pseudo-inverse of G^T (n x k, G of full column
    rank) times U1^T is factored as [L2, U2, Q] = lu(.); L = L1 U2^T and
    U = L2^T (the listing's last line reads U = L^T; the text's derivation
    gives L2^T).  That is Alg. 5's assembly with V := pinv(G^T) and Y := H,
    so the approximation L U equals A G pinv(G) = A V V^T for V an
    orthonormal basis of Range(A^T Omega), in the row and column orders p, q."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    Omega = np.asarray(Omega, dtype=np.float64)
    if Omega.shape != (m, k) or not (1 <= k < min(m, n)):
        raise ValueError("need Omega m x k and 1 <= k < min(m, n)")
    G = A.T @ Omega                      # n x k
    H = A @ G                            # m x k
    Gt_pinv = np.linalg.pinv(G.T)        # n x k
    fac = assemble(A, Gt_pinv, Y=H)
    fac.normA2 = float(np.sum(A * A))
    fac.passes = 1
    fac.V = Gt_pinv
    fac.G = G
    return fac


# ----------------------------------------------------------------------------
# Accuracy measure, eq. (error) in Sec. 6.2.
# ----------------------------------------------------------------------------
def relative_residual(A: np.ndarray, p: np.ndarray, q: np.ndarray,
                      L: np.ndarray, U: np.ndarray) -> float:
    """||A[p][:, q] - L U||_F / ||A||_F in float64."""
    A = np.asarray(A, dtype=np.float64)
    R = A[np.ix_(p, q)] - np.asarray(L, np.float64) @ np.asarray(U, np.float64)
    return float(np.sqrt(np.sum(R * R)) / np.sqrt(np.sum(A * A)))
