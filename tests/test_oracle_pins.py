"""Pins for the FP64 oracle: each check ties the oracle to something other than
itself (LAPACK, exact arithmetic, closed forms, theorems of the paper, values
the paper prints).  CPU only."""

import json
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg
import scipy.linalg.lapack as lapack

from oracle import powerlu as O
from oracle import philox as PH
from synth import spectrum, paper_type, gaussian_omega, lowrank_plus_noise

mpmath.mp.dps = 60


def _rand(m, n, seed):
    return np.random.default_rng(seed).standard_normal((m, n))


# ----------------------------------------------------------------------------
# GETRF (the paper's lu(.))
# ----------------------------------------------------------------------------
def test_getrf_textbook_definition():
    X = _rand(300, 40, 1)
    f = O.getrf(X)
    u = np.finfo(np.float64).eps
    # P X = L U with a backward error of order m u ||X||
    R = X[f.perm] - f.L @ f.U
    assert np.max(np.abs(R)) <= 10 * 300 * u * np.max(np.abs(X))
    # L unit lower trapezoidal with |l_ij| <= 1 (partial pivoting), U upper
    assert np.allclose(np.diag(f.L[:40]), 1.0)
    assert np.all(np.triu(f.L[:40], 1) == 0.0)
    assert np.max(np.abs(f.L)) <= 1.0
    assert np.all(np.tril(f.U, -1) == 0.0)
    # perm is a permutation
    assert sorted(f.perm.tolist()) == list(range(300))


@pytest.mark.parametrize("shape,seed", [((500, 40), 2), ((64, 64), 3), ((1000, 7), 4)])
def test_getrf_pivots_equal_lapack(shape, seed):
    """Special case that reduces to a library routine: on Gaussian inputs
    (gaps far above rounding) the pivot sequence equals LAPACK dgetrf's."""
    X = _rand(*shape, seed)
    f = O.getrf(X)
    lu, piv, info = lapack.dgetrf(X)
    assert info == 0
    assert np.array_equal(f.ipiv, piv)
    c = shape[1]
    assert np.allclose(np.triu(lu[:c, :c]), f.U, rtol=1e-12, atol=1e-12)
    assert np.min(f.gaps) > 1e-8


def test_getrf_crafted_tie_picks_first_current_row():
    """Equal |values| at rows j+2 and j+5: the first one in current order wins
    (LAPACK's idamax rule)."""
    X = np.zeros((8, 2))
    X[:, 0] = [1.0, 0.5, 3.0, 0.25, -0.5, -3.0, 2.0, 0.125]
    X[:, 1] = np.arange(8) + 1.0
    f = O.getrf(X)
    assert f.ipiv[0] == 2
    assert f.gaps[0] == 0.0
    lu, piv, info = lapack.dgetrf(X)
    assert np.array_equal(f.ipiv, piv)


def test_getrf_tie_after_swap_uses_current_order():
    """After the first swap the row that was at position 0 sits at position r;
    a later tie between it and a row below it must follow the current order."""
    X = np.array([[1.0, 2.0],
                  [4.0, 1.0],
                  [0.5, 3.0],
                  [2.0, 3.0]])
    # step 0 picks row 1 (|4|) and moves old row 0 to position 1.
    f = O.getrf(X)
    lu, piv, info = lapack.dgetrf(X)
    assert np.array_equal(f.ipiv, piv)
    assert np.allclose(f.L @ f.U, X[f.perm])


def test_getrf_zero_column():
    """A zero pivot column is not swapped or scaled; the first zero step is
    reported (LAPACK getrf INFO > 0 semantics)."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((10, 4))
    X[:, 2] = 0.0
    X[:, 3] = 2.0 * X[:, 0]          # exactly dependent after the zero column
    f = O.getrf(X)
    lu, piv, info = lapack.dgetrf(X)
    assert info == 3                 # 1-based first zero pivot
    assert f.zero_step == 2
    assert np.array_equal(f.ipiv[:3], piv[:3])
    assert f.ipiv[2] == 2
    assert np.allclose(X[f.perm], f.L @ f.U, atol=1e-12)


def test_lur_is_permuted_unit_lower():
    X = _rand(50, 6, 7)
    V, f = O.lur(X)
    # V[perm] = L  ->  V = P^T L, and V spans the same space as X
    assert np.allclose(V[f.perm], f.L)
    Qx = np.linalg.qr(X)[0]
    Qv = np.linalg.qr(V)[0]
    s = scipy.linalg.subspace_angles(Qx, Qv)
    assert np.max(s) < 1e-12


# ----------------------------------------------------------------------------
# thin QR against exact arithmetic
# ----------------------------------------------------------------------------
def _mp_thin_q(M):
    """Thin Q of a numpy matrix by Gram-Schmidt with reorthogonalization at
    60 significant digits."""
    rows, cols = M.shape
    A = mpmath.matrix(M.tolist())
    Q = mpmath.matrix(rows, cols)
    for j in range(cols):
        v = A[:, j]
        for _ in range(2):
            for i in range(j):
                d = sum(Q[t, i] * v[t] for t in range(rows))
                v = v - d * Q[:, i]
        nv = mpmath.sqrt(sum(v[t] ** 2 for t in range(rows)))
        Q[:, j] = v / nv
    return np.array(Q.tolist(), dtype=np.float64)


def _equal_up_to_signs(V, Q, tol):
    for j in range(V.shape[1]):
        s = np.sign(V[:, j] @ Q[:, j])
        if np.max(np.abs(V[:, j] - s * Q[:, j])) > tol:
            return False
    return True


def test_thin_qr_against_exact():
    X = _rand(9, 4, 11)
    V = O.thin_qr(X)
    assert V.shape == (9, 4)
    assert np.max(np.abs(V.T @ V - np.eye(4))) < 1e-14
    Q = _mp_thin_q(X)
    assert _equal_up_to_signs(V, Q, 1e-13)


# ----------------------------------------------------------------------------
# Alg. 7 against the explicit Krylov basis at 60 digits (F1: the LU
# reorthogonalizations only change the basis by an upper-triangular factor)
# ----------------------------------------------------------------------------
def _tiny_problem(m, n, seed):
    rng = np.random.default_rng(seed)
    U = np.linalg.qr(rng.standard_normal((m, m)))[0]
    W = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.linspace(1.0, 0.3, min(m, n))
    S = np.zeros((m, n))
    S[np.arange(len(s)), np.arange(len(s))] = s
    return U @ S @ W.T


def _mp_krylov_q(A, Omega, v):
    P = (v - 1) // 2
    Am = mpmath.matrix(A.tolist())
    K = mpmath.matrix(Omega.tolist())
    if v % 2 == 0:
        K = Am.T * K
    for _ in range(P):
        K = Am.T * (Am * K)
    return _mp_q_of(K)


def _mp_q_of(K):
    rows, cols = K.rows, K.cols
    Q = mpmath.matrix(rows, cols)
    for j in range(cols):
        v = K[:, j]
        for _ in range(2):
            for i in range(j):
                d = sum(Q[t, i] * v[t] for t in range(rows))
                v = v - d * Q[:, i]
        nv = mpmath.sqrt(sum(v[t] ** 2 for t in range(rows)))
        Q[:, j] = v / nv
    return np.array(Q.tolist(), dtype=np.float64)


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_range_basis_equals_krylov_q(v):
    m, n, l = 12, 10, 4
    A = _tiny_problem(m, n, 20 + v)
    Omega = _rand(m if v % 2 == 0 else n, l, 30 + v)
    rec = O.RangeRecord()
    V = O.range_basis(A, Omega, v, rec)
    assert rec.passes == v - 1
    Q = _mp_krylov_q(A, Omega, v)
    assert _equal_up_to_signs(V, Q, 1e-12)


def test_planted_mistake_lur_without_permutation_is_caught(monkeypatch):
    """If the LU reorthogonalization returned L in pivoted row order (instead
    of P^T L), the Krylov pin above fails: the pin does catch reading R1."""
    def bad_lur(X):
        f = O.getrf(X)
        return f.L.copy(), f
    monkeypatch.setattr(O, "lur", bad_lur)
    m, n, l, v = 12, 10, 4, 4
    A = _tiny_problem(m, n, 24)
    Omega = _rand(m, l, 34)
    V = O.range_basis(A, Omega, v)
    Q = _mp_krylov_q(A, Omega, v)
    assert not _equal_up_to_signs(V, Q, 1e-6)


# ----------------------------------------------------------------------------
# Assembly (Alg. 5 steps 3-8)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_assembly_identity_and_shapes(v):
    m, n, k, l = 60, 50, 6, 10
    rng = np.random.default_rng(40 + v)
    U0 = np.linalg.qr(rng.standard_normal((m, m)))[0]
    W0 = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = np.exp(-np.arange(n) / 5.0)
    A = (U0[:, :n] * s) @ W0.T
    Omega = rng.standard_normal((m if v % 2 == 0 else n, l))
    f = O.powerlu(A, k, Omega, v)
    assert f.L.shape == (m, k) and f.U.shape == (k, n)
    # L U equals (A Vk Vk^T)[p][:, q]  (eq. firstlu / secondlu / powerlufinal)
    Vk = f.V
    proj = (A @ Vk @ Vk.T)[np.ix_(f.p, f.q)]
    assert np.max(np.abs(f.L @ f.U - proj)) < 1e-12
    # residual^2 = ||A||^2 - ||A Vk||^2  (Thm 4.2 applied to Vk)
    r = O.relative_residual(A, f.p, f.q, f.L, f.U)
    nA2 = np.sum(A * A)
    ind = (nA2 - np.sum((A @ Vk) ** 2)) / nA2
    assert abs(r * r - ind) <= 1e-12 * max(ind, 1e-300) + 1e-15
    # U unit upper trapezoidal with |u| <= 1 ; L lower trapezoidal
    assert np.allclose(np.diag(f.U[:, :k]), 1.0)
    assert np.all(np.tril(f.U[:, :k], -1) == 0.0)
    assert np.max(np.abs(f.U)) <= 1.0 + 1e-15
    assert np.all(np.triu(f.L[:k], 1) == 0.0)
    # L1 (the first LU's factor) is unit lower with |l| <= 1
    assert np.allclose(np.diag(f.lu1.L[:k]), 1.0)
    assert np.max(np.abs(f.lu1.L)) <= 1.0


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_exact_recovery_of_rank_k(v):
    """Thm 3.1 with sigma_{k+1} = 0: an exactly rank-k matrix is recovered to
    rounding (relative residual < 1e-12)."""
    m, n, k, l = 200, 150, 8, 13
    rng = np.random.default_rng(50 + v)
    A = rng.standard_normal((m, k)) @ rng.standard_normal((k, n))
    Omega = rng.standard_normal((m if v % 2 == 0 else n, l))
    f = O.powerlu(A, k, Omega, v)
    assert O.relative_residual(A, f.p, f.q, f.L, f.U) < 1e-12


@pytest.mark.parametrize("t", [1, 2, 3])
def test_eckart_young_lower_bounds(t):
    """eq. (ey): no rank-k approximation beats the truncated SVD, in both the
    spectral and the Frobenius norm."""
    n, k, l = 300, 15, 25
    A = paper_type(t, n, seed=t)
    sv = np.linalg.svd(A, compute_uv=False)
    for v in (2, 3, 4):
        Omega = gaussian_omega(n, l, seed=100 + v).astype(np.float64)
        f = O.powerlu(A, k, Omega, v)
        R = A[np.ix_(f.p, f.q)] - f.L @ f.U
        assert np.linalg.norm(R, 2) >= sv[k] * (1 - 1e-10)
        assert np.linalg.norm(R, "fro") >= np.sqrt(np.sum(sv[k:] ** 2)) * (1 - 1e-10)


def test_thm32_range_equals_randlu_range():
    """Thm 3.2 (odd v = 2p+1): Range(P^T L) of PowerLU equals the range of
    Y = A (A^T A)^p Omega (RandLU's L_y), here truncated to the first k
    columns, which both sides span."""
    m, n, k = 80, 60, 6
    A = _tiny_problem(m, n, 60)
    rng = np.random.default_rng(61)
    for p_exp in (1, 2):
        v = 2 * p_exp + 1
        Omega = rng.standard_normal((n, k))
        # l = k here so that the truncation keeps the whole Krylov block
        rec = O.RangeRecord()
        V = O.range_basis(A, Omega, v, rec)
        fac = O.assemble(A, V[:, :k])
        PL = np.empty_like(fac.L)
        PL[fac.p] = fac.L
        Y = Omega
        for _ in range(p_exp):
            Y = A.T @ (A @ Y)
        Y = A @ Y
        ang = scipy.linalg.subspace_angles(np.linalg.qr(PL)[0], np.linalg.qr(Y[:, :k])[0])
        assert np.max(ang) < 1e-9


def _thm31_bound(s, k, q, p):
    """Thm 3.1's expectation bound on ||A - A V V^T|| (spectral norm)."""
    t = s[k] ** (2 * p)
    tail = np.sqrt(np.sum(s[k:] ** (4 * p)))
    return ((1 + np.sqrt(k / (q - 1)) * t) * t + np.e * np.sqrt(k + q) / q * tail) ** (1.0 / (2 * p))


def _thm33_bound(s, k, q, p):
    e = 2 * p + 1
    t = s[k] ** e
    tail = np.sqrt(np.sum(s[k:] ** (2 * e)))
    return ((1 + np.sqrt(k / (q - 1)) * t) * t + np.e * np.sqrt(k + q) / q * tail) ** (1.0 / e)


@pytest.mark.parametrize("t", [1, 2, 3])
def test_thm31_thm33_mean_error_below_bound(t):
    """Statistical pin: the mean over 20 Gaussian draws (the paper averages 20
    runs, Sec. 6) of ||A - A V V^T||_2 stays below Thm 3.1 (odd v) and
    Thm 3.3 (even v); the mean error does not grow with v."""
    n, k, q = 200, 10, 5
    A = paper_type(t, n, seed=10 + t)
    s = np.linalg.svd(A, compute_uv=False)
    means = {}
    for v in (3, 4, 5):
        errs = []
        for run in range(20):
            Om = np.random.default_rng(1000 * v + run).standard_normal((n, k + q))
            V = O.range_basis(A, Om, v)
            errs.append(np.linalg.norm(A - A @ V @ V.T, 2))
        means[v] = np.mean(errs)
        p = (v - 1) // 2
        bound = _thm31_bound(s, k, q, p) if v % 2 == 1 else _thm33_bound(s, k, q, p)
        assert means[v] <= bound
    assert means[5] <= means[3] * (1 + 1e-6)


# ----------------------------------------------------------------------------
# Sec. 4: block update, Thm 4.1, Thm 4.3 by brute force
# ----------------------------------------------------------------------------
def test_indicator_equals_explicit_block_update():
    m, n, b, s_blocks = 70, 60, 4, 5
    A = _tiny_problem(m, n, 70)
    l = b * s_blocks
    Om = _rand(m, l, 71)
    V = O.range_basis(A, Om, 4)
    nA2 = float(np.sum(A * A))
    E = O.indicator(nA2, np.sum((A @ V) ** 2, axis=0))
    Ai = A.copy()
    for i in range(s_blocks):
        Vi = V[:, i * b:(i + 1) * b]
        Ai = Ai - Ai @ Vi @ Vi.T                # eq. (b2)
        # Thm 4.1(b): A^(i) = A (I - P_i)
        Pi = V[:, :(i + 1) * b] @ V[:, :(i + 1) * b].T
        assert np.max(np.abs(Ai - A @ (np.eye(n) - Pi))) < 1e-12
        # Thm 4.3: ||A^(i)||^2 = ||A||^2 - sum_j ||A V_j||^2
        exact = float(np.sum(Ai * Ai))
        assert abs(E[(i + 1) * b - 1] - exact) <= 1e-10 * nA2


def test_table1_truncated_svd_ranks(golden_dir):
    """Table 1's truncated-SVD ranks are reproduced by the rank rule when the
    indicator is fed the exact singular directions (||A v_j||^2 = sigma_j^2):
    this pins the prefix sums, the stopping test and the column indexing."""
    rows = []
    with open(os.path.join(golden_dir, "table1_tsvd_ranks.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    assert len(rows) == 6
    for t, eps, n, k_tsvd, _k_fp, b in rows:
        s = spectrum(f"type{t}", int(n))
        c = s * s
        k_col, ok = O.rank_rule(float(np.sum(c)), c, float(eps), int(b), True)
        assert ok and k_col == int(k_tsvd)
        k_blk, ok = O.rank_rule(float(np.sum(c)), c, float(eps), int(b), False)
        assert ok and k_blk == int(b) * -(-int(k_tsvd) // int(b))


def test_table1_oracle_ranks_soft_pin(golden_dir):
    """Table 1's PowerLU_FP ranks (averages of 20 MATLAB runs) against the
    oracle's on the same setting: Matrix Types 1-3 at n = 8000, v = 4,
    l = 50 b, column rule, 20 Gaussian test matrices per row (5 for the
    l = 2000 row), stored by tests/golden/make_table1_oracle.py.  Soft: the
    mean within 3% or one column of the printed average.  Hard: every rank
    at least the truncated-SVD rank (Eckart-Young), the stored indicator
    values on either side of eps^2, and at s = 0 the column rule applied to
    the stored indicator curve gives the stored rank and the residual of the
    assembled factorization meets eps."""
    with open(os.path.join(golden_dir, "table1_oracle.json")) as fh:
        g = json.load(fh)
    assert g["n"] == 8000 and len(g["rows"]) == 6
    printed = {(1, 1e-2): (15, 15), (1, 1e-4): (313, 328), (2, 1e-4): (65, 66),
               (2, 1e-5): (81, 82), (3, 1e-2): (32, 32), (3, 1.5e-3): (1587, 1588)}
    for row in g["rows"]:
        k_tsvd, k_fp = printed[(row["type"], row["eps"])]
        assert (row["k_tsvd"], row["k_fp_printed"]) == (k_tsvd, k_fp)
        eps2 = row["eps"] ** 2
        ranks = [x["rank"] for x in row["runs"]]
        assert len(ranks) == (5 if row["l"] > 1000 else 20)
        for x in row["runs"]:
            assert x["tol_reached"] and x["rank"] >= k_tsvd
            assert x["e_at"] <= eps2 < x["e_prev"]
        mean = float(np.mean(ranks))
        assert abs(mean - k_fp) <= max(1.0, 0.03 * k_fp), (row["type"], row["eps"], mean, k_fp)
        E = np.asarray(row["E_s0"])
        k0 = int(np.argmax(E <= eps2)) + 1
        assert E[k0 - 1] <= eps2 and (k0 == 1 or E[k0 - 2] > eps2)
        assert k0 == row["runs"][0]["rank"]
        assert row["residual_s0"] <= row["eps"] * (1 + 1e-9)


def test_rank_rule_edge_cases():
    assert O.rank_rule(0.0, np.zeros(8), 1e-3, 2, True) == (0, True)
    c = np.array([1.0, 1.0, 1.0, 1.0])
    # ||A||^2 = 8: never reaches eps^2 * 8 with these four columns
    assert O.rank_rule(8.0, c, 1e-3, 2, True) == (4, False)
    # exactly reaching the threshold counts (E <= acc)
    assert O.rank_rule(4.0, c, 0.5, 1, True) == (3, True)


@pytest.mark.parametrize("t,eps,k_tsvd", [(2, 1e-4, 65), (3, 1e-2, 32)])
def test_powerlu_fp_rank_near_tsvd(t, eps, k_tsvd):
    """Table 1 setting at a reduced size (n = 1000, v = 4, b = 10, l = 50 b):
    PowerLU_FP's rank is at least the truncated-SVD rank (Eckart-Young) and
    within a few columns of it; the returned factorization meets the
    tolerance and its residual^2 equals the stopping indicator E_k."""
    n, b = 1000, 10
    l = 50 * b if 50 * b < n else 40 * b
    A = paper_type(t, n, seed=200 + t)
    Om = np.random.default_rng(300 + t).standard_normal((n, l))
    f = O.powerlu_fp(A, eps, b, Om, 4, column_mode=True)
    assert f.tol_reached
    assert k_tsvd <= f.rank <= k_tsvd + 3
    r = O.relative_residual(A, f.p, f.q, f.L, f.U)
    assert r <= eps * (1 + 1e-9)
    assert abs(r * r * f.normA2 - f.E[f.rank - 1]) <= 1e-9 * f.normA2
    fb = O.powerlu_fp(A, eps, b, Om, 4, column_mode=False)
    assert fb.rank == b * -(-f.rank // b)


def test_powerlu_fp_zero_matrix():
    A = np.zeros((40, 30))
    f = O.powerlu_fp(A, 1e-3, 2, _rand(40, 10, 1), 4)
    assert f.rank == 0 and f.tol_reached


# ----------------------------------------------------------------------------
# Philox4x32-10 and the Gaussian draw
# ----------------------------------------------------------------------------
def test_philox_known_answers(golden_dir):
    with open(os.path.join(golden_dir, "philox4x32_10_kat.txt")) as fh:
        rows = [l.split() for l in fh if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        out = PH.philox4x32_10(np.array([w[0:4]]), np.array(w[4:6]))[0]
        assert [int(x) for x in out] == w[6:10]


def test_philox_gaussian_moments_and_layout():
    z = PH.gaussian(1000, 250, seed=12345)
    assert z.shape == (1000, 250)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.01
    # layout: element e of the flattened matrix is word e % 4 of block e // 4
    w = PH.gaussian_words(3, 5, seed=7)
    blk = PH.philox4x32_10(np.array([[3, 0, 0, 0]]), np.array([7, 0]))[0]
    assert np.array_equal(w[12:15], blk[:3])
    # a different seed gives a different draw
    assert not np.allclose(PH.gaussian(4, 4, 1), PH.gaussian(4, 4, 2))


# ----------------------------------------------------------------------------
# Generators
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("t", [1, 2, 3])
def test_paper_type_spectrum(t):
    A = paper_type(t, 120, seed=9)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(sv, spectrum(f"type{t}", 120), rtol=1e-10, atol=1e-14)


def test_lowrank_plus_noise_is_seeded():
    s = spectrum("exp", 20, tau=4.0)
    A1 = lowrank_plus_noise(100, 80, s, 1, 2, 1e-3, 3)
    A2 = lowrank_plus_noise(100, 80, s, 1, 2, 1e-3, 3)
    assert A1.dtype == np.float32 and np.array_equal(A1, A2)
    A0 = lowrank_plus_noise(100, 80, s, 1, 2, 0.0, 3, dtype=np.float64)
    sv = np.linalg.svd(A0, compute_uv=False)
    assert np.allclose(sv[:20], s, rtol=1e-10)
    assert sv[20] < 1e-12
