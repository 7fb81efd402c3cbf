"""Step-level parity of the HIP path against the FP64 oracle, through the C ABI.
Each test names the step of the path it covers."""

import numpy as np
import pytest

from tests.gpu_common import torch, have_gpu, handle, dev, host, equal_up_to_signs, assert_pivots
from tests.test_crafted_ties import TIE_CASES
from oracle import powerlu as O
from oracle import philox as PH
from synth import crafted_tie_matrix, gaussian_omega, lowrank_plus_noise, spectrum

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


# ---------------------------------------------------------------- a1: Gaussian draw
@pytest.mark.parametrize("rows,cols,seed", [(1001, 37, 5), (64, 4, 0), (3, 5, 2**40 + 7)])
def test_gaussian_matches_philox_oracle(h, rows, cols, seed):
    z = host(h.gaussian(rows, cols, seed))
    ref = PH.gaussian(rows, cols, seed)
    # Philox words are integers (exact); only log/sqrt/sin/cos differ (fp32 vs fp64)
    assert np.max(np.abs(z - ref) / (1.0 + np.abs(ref))) < 2e-6


# ---------------------------------------------------------------- a2/a4/a6: passes
@pytest.mark.parametrize("m,n,l", [(1000, 777, 30), (3001, 2500, 110), (517, 4133, 13),
                                   (256, 256, 16), (9000, 300, 133), (300, 9000, 250)])
@pytest.mark.parametrize("trans", [False, True])
def test_pass_matches_fp64(h, m, n, l, trans):
    rng = np.random.default_rng(m * 7 + n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((m if trans else n, l)).astype(np.float32)
    nA2 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    out = host(h.pass_(dev(A), dev(X), trans=trans, normA2=nA2))
    ref = (A.astype(np.float64).T if trans else A.astype(np.float64)) @ X.astype(np.float64)
    K = m if trans else n
    # fp32 accumulation of K products of N(0,1) entries: error ~ sqrt(K) u per term scale
    tol = 8.0 * np.sqrt(K) * 6e-8 * np.sqrt(K)
    assert np.max(np.abs(out - ref)) < tol
    assert abs(float(nA2.cpu()) - np.sum(A.astype(np.float64) ** 2)) <= 1e-12 * np.sum(A.astype(np.float64) ** 2)


# ---------------------------------------------------------------- a3/a7/a9: LU
@pytest.mark.parametrize("M,c,seed", [(2000, 30, 1), (5000, 110, 2), (300, 64, 3), (129, 128, 4),
                                      (1000, 1, 5), (4096, 200, 6), (777, 65, 7)])
def test_getrf_matches_oracle(h, M, c, seed):
    X = np.random.default_rng(seed).standard_normal((M, c)).astype(np.float32)
    F = dev(X)
    perm, U, info = h.getrf(F)
    ref = O.getrf(X.astype(np.float64))
    V_ref, _ = O.lur(X.astype(np.float64))
    # these Gaussian inputs have every oracle gap above 1e-4: compared in full
    assert_pivots(host(perm)[:c], ref.perm[:c], ref.gaps, 1e-4)
    assert np.array_equal(host(perm), ref.perm)
    assert np.max(np.abs(host(F) - V_ref)) < 1e-3
    assert np.max(np.abs(host(U) - ref.U)) <= 1e-4 * np.max(np.abs(ref.U)) * np.sqrt(c) + 1e-5
    assert info["zero_pivot_step"] == -1


@pytest.mark.parametrize("M,c,seed", TIE_CASES)
def test_getrf_crafted_ties_follow_lapack_order(h, M, c, seed):
    """Exact ties at every step, on inputs whose elimination is exact in
    float32 (checked on the CPU by tests/test_crafted_ties.py): the first
    maximum in the current row order wins at every one of the c steps, as in
    the oracle, and the factors are bit-identical."""
    X = crafted_tie_matrix(M, c, seed)
    F = dev(X.astype(np.float32))
    perm, U, info = h.getrf(F)
    ref = O.getrf(X)
    V_ref, _ = O.lur(X)
    assert int(np.sum(np.asarray(ref.gaps[:c]) == 0.0)) == c
    assert np.array_equal(host(perm), ref.perm)
    assert np.array_equal(host(U).astype(np.float64), ref.U)
    assert np.array_equal(host(F).astype(np.float64), V_ref)


def test_getrf_zero_column_reports_step(h):
    rng = np.random.default_rng(10)
    X = rng.standard_normal((400, 8)).astype(np.float32)
    X[:, 3] = 0.0
    F = dev(X)
    perm, U, info = h.getrf(F)
    ref = O.getrf(X.astype(np.float64))
    assert info["zero_pivot_step"] == 3 == ref.zero_step
    assert np.array_equal(host(perm)[:4], ref.perm[:4])


# ---------------------------------------------------------------- a5: thin QR
@pytest.mark.parametrize("M,c,seed,tau", [(2000, 30, 1, 40.0), (5000, 110, 2, 40.0),
                                          (3000, 200, 3, 40.0), (600, 300, 4, 40.0),
                                          # column scales down to e^-25 and e^-32: the
                                          # float64 Gram of every block is far beyond
                                          # the probe's limit, so each block takes the LU
                                          (3000, 200, 5, 8.0), (2500, 260, 6, 8.0)])
def test_thin_qr_orthonormal_and_same_range(h, M, c, seed, tau):
    rng = np.random.default_rng(seed)
    X = (rng.standard_normal((M, c)) @ np.diag(np.exp(-np.arange(c) / tau))).astype(np.float32)
    Q = host(h.thin_qr(dev(X)))
    eta = np.max(np.abs(Q.T.astype(np.float64) @ Q - np.eye(c)))
    print(f"M {M} c {c}: max |Q^T Q - I| = {eta:.2e}")
    # one Gram-Schmidt block (c <= 128): final product in fp64, so only the
    # fp32 rounding of Q remains: off-diagonal ~u32/sqrt(M), diagonal up to
    # ~u32 max|q_ij|^2 <= u32; several blocks: fp32 projections between
    # blocks -> ~u32 * sqrt(c)
    assert eta < (1e-7 if c <= 128 else 2e-6)
    Qr = O.thin_qr(X.astype(np.float64))
    ok, worst = equal_up_to_signs(Q.astype(np.float64), Qr, 2e-3)
    assert ok, worst


# ---------------------------------------------------------------- Alg. 7
@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_range_basis_matches_oracle(h, v):
    m, n, l = 1500, 1200, 30
    A = lowrank_plus_noise(m, n, spectrum("exp", 200, tau=15.0), 21, 22, 1e-6, 23)
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=24 + v)
    V = host(h.range_basis(dev(A), l, v, Omega=dev(Om))).astype(np.float64)
    Vr = O.range_basis(A.astype(np.float64), Om.astype(np.float64), v)
    assert np.max(np.abs(V.T @ V - np.eye(l))) < 2e-5
    # leading columns carry the dominant directions and must agree closely
    ok, worst = equal_up_to_signs(V[:, :20], Vr[:, :20], 2e-3)
    assert ok, worst


# ---------------------------------------------------------------- a12: rank rule
def test_rank_rule_matches_oracle(h):
    rng = np.random.default_rng(3)
    G = (rng.standard_normal((5000, 96)) * np.exp(-np.arange(96) / 10.0)).astype(np.float32)
    c = np.sum(G.astype(np.float64) ** 2, axis=0)
    nA2 = float(np.sum(c)) * (1 + 1e-7)
    for col in (True, False):
        k, E, cn, ok = h.rank_rule(dev(G), nA2, 1e-3, 8, column_exact=col)
        kr, okr = O.rank_rule(nA2, c, 1e-3, 8, col)
        assert (k, ok) == (kr, okr)
        assert np.allclose(cn, c, rtol=1e-12)
