"""Pins of the RandLU (Alg. 3 + Alg. 4) and RandSVD (Alg. 1 + Alg. 2) oracle.
CPU only.

What fixes the results independently of the oracle's own code:
  * RandLU is a projection: P A Q - L U = (I - Pi) P A Q with Pi the
    orthogonal projector onto Range(L_y(:, :k)), computed here from an
    independent QR -- a dropped (L_y^T L_y)^{-1} or a wrong transpose or
    permutation in the assembly breaks it (a planted mistake shows it does);
  * Alg. 4 and Alg. 2 span Range(A (A^T A)^p Omega) restricted to the leading
    columns, checked against the explicit power product on well-conditioned
    inputs, and against each other;
  * Thm 3.2: RandLU at p and PowerLU at v = 2p + 1 on the same Omega give the
    same Range(P^T L);
  * exact recovery of a matrix of rank <= k; Eckart-Young lower bounds;
  * RandSVD: singular values interlace those of A (any orthonormal Q), the
    rank-k residual obeys Pythagoras ||A||^2 - sum s_i^2, exact rank is
    recovered with the true singular values, and the rank-l factors rebuild
    Q Q^T A.
"""

import numpy as np
import pytest

from oracle import baselines as Bo
from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, spectrum


def _mat(m=300, n=240, r=120, tau=12.0, seed=3):
    return lowrank_plus_noise(m, n, spectrum("exp", r, tau=tau), seed, seed + 1, 1e-6, seed + 2,
                              dtype=np.float64)


def _proj(X):
    Q, _ = np.linalg.qr(X)
    return Q @ Q.T


def _tail(A, k):
    s = np.linalg.svd(A, compute_uv=False)
    return float(np.sqrt(np.sum(s[k:] ** 2)) / np.sqrt(np.sum(s ** 2)))


# ---------------------------------------------------------------- RandLU
@pytest.mark.parametrize("p", [0, 1, 2])
def test_randlu_is_the_projection_onto_Ly(p):
    A = _mat()
    m, n = A.shape
    k, l = 20, 30
    Om = gaussian_omega(n, l, seed=10 + p).astype(np.float64)
    f = Bo.randlu(A, k, Om, p)
    assert f.passes == 2 * p + 2
    Ly = f.lu1.L[:, :k]
    PA = A[f.p]
    R = PA - _proj(Ly) @ PA
    expect = float(np.sqrt(np.sum(R * R)) / np.sqrt(np.sum(A * A)))
    got = O.relative_residual(A, f.p, f.q, f.L, f.U)
    assert abs(got - expect) <= 1e-10 * expect
    assert got >= _tail(A, k) * (1 - 1e-12)           # Eckart-Young
    # L lower trapezoidal in pivot order, U unit upper trapezoidal, |u| <= 1
    assert np.allclose(np.triu(f.L, 1)[:k], 0.0)
    assert np.allclose(np.diag(f.U[:, :k]), 1.0) and np.max(np.abs(f.U)) <= 1 + 1e-12


def test_randlu_pin_catches_a_dropped_gram_inverse():
    """Planted mistake: B = L_y^T P A (the (L_y^T L_y)^{-1} dropped)."""
    A = _mat()
    m, n = A.shape
    k, l = 20, 30
    Om = gaussian_omega(n, l, seed=7).astype(np.float64)
    f = Bo.randlu(A, k, Om, 1)
    Ly = f.lu1.L[:, :k]
    PA = A[f.p]
    Bw = Ly.T @ PA
    g = O.getrf(Bw.T)
    Lw, Uw = Ly @ g.U.T, g.L.T
    wrong = O.relative_residual(A, f.p, g.perm, Lw, Uw)
    R = PA - _proj(Ly) @ PA
    expect = float(np.sqrt(np.sum(R * R)) / np.sqrt(np.sum(A * A)))
    assert abs(wrong - expect) > 1e-3 * expect


@pytest.mark.parametrize("p", [0, 1])
def test_lu_power_spans_the_power_product(p):
    """Range(P^T L_y(:, :k)) = Range(Y(:, :k)), Y = A (A^T A)^p Omega, on a
    mildly decaying spectrum where Y is well conditioned; Alg. 2's basis spans
    the full Range(Y)."""
    A = _mat(r=200, tau=150.0, seed=5)
    m, n = A.shape
    k, l = 12, 16
    Om = gaussian_omega(n, l, seed=20 + p).astype(np.float64)
    f = Bo.lu_power(A, Om, p)
    V = np.empty_like(f.L)
    V[f.perm] = f.L
    Y = A @ np.linalg.matrix_power(A.T @ A, p) @ Om
    assert np.linalg.norm(_proj(V[:, :k]) - _proj(Y[:, :k]), 2) < 1e-8
    Q = Bo.qr_power(A, Om, p)
    assert np.linalg.norm(Q @ Q.T - _proj(Y), 2) < 1e-8
    assert np.linalg.norm(Q @ Q.T - _proj(V), 2) < 1e-8
    # the three-output form: P and L are those of lu(Y) (the last product is
    # Y times an upper triangular matrix)
    g = O.getrf(Y)
    assert np.array_equal(g.perm[:l], f.perm[:l])
    assert np.max(np.abs(g.L - f.L)) < 1e-8


@pytest.mark.parametrize("p", [1, 2])
def test_thm32_randlu_and_powerlu_share_the_range(p):
    """Thm 3.2: Range(P_r^T L_r) = Range(P_p^T L_p) for RandLU at p and
    PowerLU at v = 2p + 1 on the same n x l Omega."""
    A = _mat(r=200, tau=60.0, seed=8)
    m, n = A.shape
    k, l = 15, 20
    Om = gaussian_omega(n, l, seed=30 + p).astype(np.float64)
    fr = Bo.randlu(A, k, Om, p)
    fp = O.powerlu(A, k, Om, 2 * p + 1)
    Lr = np.empty_like(fr.L)
    Lr[fr.p] = fr.L
    Lp = np.empty_like(fp.L)
    Lp[fp.p] = fp.L
    assert np.linalg.norm(_proj(Lr) - _proj(Lp), 2) < 1e-7


def test_randlu_exact_rank():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((250, 18)) @ rng.standard_normal((18, 200))
    Om = gaussian_omega(200, 25, seed=9).astype(np.float64)
    f = Bo.randlu(A, 18, Om, 1)
    assert O.relative_residual(A, f.p, f.q, f.L, f.U) < 1e-12


# ---------------------------------------------------------------- RandSVD
@pytest.mark.parametrize("p", [0, 1])
def test_randsvd_interlacing_and_pythagoras(p):
    A = _mat(seed=11)
    m, n = A.shape
    k, l = 20, 30
    Om = gaussian_omega(n, l, seed=40 + p).astype(np.float64)
    r = Bo.randsvd(A, k, Om, p)
    assert r.passes == 2 * p + 2
    sig = np.linalg.svd(A, compute_uv=False)
    assert np.all(r.s_all <= sig[:l] * (1 + 1e-12))
    assert np.all(np.diff(r.s) <= 0)
    assert np.max(np.abs(r.U.T @ r.U - np.eye(k))) < 1e-12
    assert np.max(np.abs(r.V.T @ r.V - np.eye(k))) < 1e-12
    nA2 = float(np.sum(A * A))
    res = Bo.svd_relative_residual(A, r.U, r.s, r.V)
    assert abs(res ** 2 - (nA2 - float(np.sum(r.s ** 2))) / nA2) < 1e-12
    assert res >= _tail(A, k) * (1 - 1e-12)
    # the rank-l factors rebuild Q Q^T A
    QQA = r.Q @ (r.Q.T @ A)
    assert np.max(np.abs((r.U_all * r.s_all) @ r.V_all.T - QQA)) < 1e-12 * np.max(np.abs(A))


def test_randsvd_exact_rank_gives_the_true_svd():
    rng = np.random.default_rng(6)
    U0, _ = np.linalg.qr(rng.standard_normal((220, 10)))
    V0, _ = np.linalg.qr(rng.standard_normal((180, 10)))
    s0 = np.linspace(5.0, 0.5, 10)
    A = (U0 * s0) @ V0.T
    Om = gaussian_omega(180, 14, seed=2).astype(np.float64)
    r = Bo.randsvd(A, 10, Om, 0)
    assert np.max(np.abs(r.s - s0)) < 1e-12
    # singular vectors up to sign
    sg = np.sign(np.sum(r.U * U0, axis=0))
    assert np.max(np.abs(r.U * sg - U0)) < 1e-10
    assert np.max(np.abs(r.V * sg - V0)) < 1e-10
