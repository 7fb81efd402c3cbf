"""Pins of the oracle's restart rounds for PowerLU_FP (the Remark after
Alg. 8: when l columns miss the tolerance, draw a fresh Gaussian matrix and
run Alg. 7 on the remainder A - A V V^T).  CPU only.

What fixes the result independently of the oracle's own code:
  * without restart entries the function is the single-round Alg. 9;
  * the kept basis is orthonormal and the indicator at the returned rank
    equals the brute-force remainder energy ||A - A V_k V_k^T||_F^2
    (Thm 4.3 for an orthonormal basis);
  * Eckart-Young: no rank below the truncated-SVD rank meets the tolerance;
  * Ky Fan: the two rounds together capture nearly the energy of the 2l
    largest singular values (power iteration on the remainder finds its
    dominant subspace), never more;
  * a planted mistake (the second round's indicator restarted from
    ||A||^2) is caught by the brute-force energy pin.
"""

import numpy as np
import pytest

from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, spectrum


def _case(seed=3, m=320, n=280, r=150, tau=18.0):
    sig = spectrum("exp", r, tau=tau)
    A = lowrank_plus_noise(m, n, sig, seed, seed + 1, 1e-7, seed + 2, dtype=np.float64)
    return A


def _tsvd_rank(s, eps):
    tail = np.cumsum((s ** 2)[::-1])[::-1]            # tail[i] = sum_{j >= i} s_j^2
    total = tail[0]
    for k in range(len(s) + 1):
        rest = tail[k] if k < len(s) else 0.0
        if rest <= eps * eps * total:
            return k
    return len(s)


def test_no_restart_entries_is_single_round():
    A = _case()
    Om = gaussian_omega(A.shape[0], 40, seed=5).astype(np.float64)
    f1 = O.powerlu_fp(A, 1e-3, 8, Om, 4)
    f2 = O.powerlu_fp(A, 1e-3, 8, Om, 4, restart_omegas=())
    assert f1.rank == f2.rank and np.array_equal(f1.p, f2.p) and np.array_equal(f1.L, f2.L)
    assert not f1.tol_reached and f1.rank == 40


@pytest.mark.parametrize("column_mode", [True, False])
def test_restart_reaches_tolerance_with_exact_indicator(column_mode):
    A = _case()
    m, n = A.shape
    l, b, eps, v = 40, 8, 1e-3, 4
    oms = [gaussian_omega(m, l, seed=10 + i).astype(np.float64) for i in range(4)]
    f = O.powerlu_fp(A, eps, b, oms[0], v, column_mode, restart_omegas=oms[1:])
    s = np.linalg.svd(A, compute_uv=False)
    k_tsvd = _tsvd_rank(s, eps)
    assert k_tsvd > l                                   # one round cannot do it
    assert f.tol_reached
    assert k_tsvd <= f.rank <= k_tsvd + 2 * b
    V = f.V
    assert np.max(np.abs(V.T @ V - np.eye(V.shape[1]))) < 1e-12
    k = f.rank
    Vk = V[:, :k]
    R = A - (A @ Vk) @ Vk.T
    normA2 = float(np.sum(A * A))
    assert abs(f.E[k - 1] - float(np.sum(R * R))) <= 1e-10 * normA2
    assert f.E[k - 1] <= eps * eps * normA2
    r = O.relative_residual(A, f.p, f.q, f.L, f.U)
    assert r <= eps * (1 + 1e-9)


def _two_round_energy(A, l, v, om1, om2):
    """Energy ||A V||_F^2 captured by the two rounds' bases."""
    V1 = O.range_basis(A, om1, v)
    G1 = A @ V1
    B = A - G1 @ V1.T
    V2 = O.range_basis(B, om2, v)
    for _ in range(2):
        V2 = V2 - V1 @ (V1.T @ V2)
    V2 = O.thin_qr(V2)
    G2 = A @ V2
    return float(np.sum(G1 * G1)), float(np.sum(G2 * G2))


def test_second_round_captures_the_next_singular_values():
    """Ky Fan: no 2l-column orthonormal basis captures more than the sum of
    the 2l largest sigma_i^2; power iteration on the remainder gets within
    a small fraction of it, the rerun on A itself does not."""
    A = _case()
    l, v = 40, 4
    om1 = gaussian_omega(A.shape[0], l, seed=21).astype(np.float64)
    om2 = gaussian_omega(A.shape[0], l, seed=22).astype(np.float64)
    s = np.linalg.svd(A, compute_uv=False)
    top = float(np.sum(s[:2 * l] ** 2))
    second = float(np.sum(s[l:2 * l] ** 2))
    e1, e2 = _two_round_energy(A, l, v, om1, om2)
    assert e1 + e2 <= top * (1 + 1e-9)
    assert top - (e1 + e2) <= 0.1 * second
    # the oracle's own second round captures the same energy as this restatement
    f = O.powerlu_fp(A, 1e-9, 8, om1, v, restart_omegas=[om2])
    assert abs(float(np.sum(f.G[:, l:2 * l] ** 2)) - e2) <= 1e-9 * second


def test_indicator_pin_catches_a_restarted_indicator():
    """Planted mistake: the indicator of the second round restarted from
    ||A||^2 instead of continuing; the brute-force remainder energy of the
    pin above tells it apart from the oracle's."""
    A = _case()
    m = A.shape[0]
    l, b, eps, v = 40, 8, 1e-3, 4
    oms = [gaussian_omega(m, l, seed=30 + i).astype(np.float64) for i in range(3)]
    f = O.powerlu_fp(A, eps, b, oms[0], v, restart_omegas=oms[1:])
    normA2 = float(np.sum(A * A))
    j = 2 * l - 1                                       # last column of round two
    Vj = f.V[:, :j + 1]
    R = A - (A @ Vj) @ Vj.T
    truth = float(np.sum(R * R))
    assert abs(f.E[j] - truth) <= 1e-10 * normA2
    wrong = normA2 - float(np.sum(f.G[:, l:j + 1] ** 2))
    assert abs(wrong - truth) > 1e-3 * normA2
