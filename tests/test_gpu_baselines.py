"""RandLU (Alg. 3 + Alg. 4) and RandSVD (Alg. 1 + Alg. 2) on the GPU against
the FP64 oracle, through the C ABI, in both storage orders of A.

RandLU gates, as for PowerLU's end-to-end tests:
  * p and q bit-exact up to the first step whose oracle gap is below
    tau = 1e-4;
  * relative residual <= 1.05 x the oracle's + 64 u32 (u32 = 2^-24, a float32
    rounding allowance that matters only where the oracle's residual is
    near zero, as for a matrix of exact rank k);
  * where the pivots agree, L within 1e-3 (relative to max |L|) and U within
    1e-3 of the oracle's;
  * a matrix of rank k is recovered to float32 accuracy;
  * Thm 3.2 on the device: RandLU at p and PowerLU at v = 2p + 1 on the same
    Omega span the same Range(P^T L) (projector distance <= 1e-3 on spectra
    whose leading k directions are well separated).

RandSVD gates (float32 passes and QR: B carries an error of about l u32
relative to sigma_1, u32 = 2^-24):
  * singular values non-increasing and within 16 l u32 sigma_1 of the
    oracle's;
  * U and V orthonormal to 16 l u32;
  * relative rank-k residual <= 1.05 x the oracle's + 64 u32;
  * leading singular vectors whose relative gap g to their neighbours
    exceeds 1e-2 agree with the oracle's, up to sign, within 1e-5 / g;
  * a matrix of rank k gives its singular values and vectors.
"""

import numpy as np
import pytest

import paper_2002_07138_amd as plu
from tests.gpu_common import torch, have_gpu, handle, dev, host, assert_pivots, assert_factors_close
from oracle import baselines as Bo
from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, spectrum

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

TAU = 1e-4
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


def col_major(A):
    return torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda").t()


def _scatter(L, p):
    out = np.empty_like(L)
    out[p] = L
    return out


def _proj(X):
    Q, _ = np.linalg.qr(np.asarray(X, np.float64))
    return Q @ Q.T


def _check_randlu(h, A, k, p_over, pw, seed, col=False, expect=(None, None)):
    m, n = A.shape
    l = k + p_over
    Om = gaussian_omega(n, l, seed=seed)
    f = h.randlu(col_major(A) if col else dev(A), k, p_over, pw, Omega=dev(Om))
    ref = Bo.randlu(A.astype(np.float64), k, Om.astype(np.float64), pw)
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    assert sorted(p.tolist()) == list(range(m)) and sorted(q.tolist()) == list(range(n))
    assert f.info["passes"] == 2 * pw + 2
    r_gpu = O.relative_residual(A, p, q, L, U)
    r_ref = O.relative_residual(A, ref.p, ref.q, ref.L, ref.U)
    print(f"{m}x{n} k {k} l {l} p {pw} col {col}: residual gpu {r_gpu:.5g} oracle {r_ref:.5g}")
    assert r_gpu <= 1.05 * r_ref + 64 * U32, (r_gpu, r_ref)
    sp = assert_pivots(p[:k], ref.p[:k], ref.lu1.gaps, TAU, expect[0], "row pivots")
    sq = assert_pivots(q[:k], ref.q[:k], ref.lu2.gaps, TAU, expect[1], "column pivots")
    if sp == k and sq == k:
        assert_factors_close(L, U, ref.L, ref.U)
    assert np.allclose(np.diag(U[:, :k]), 1.0) and np.all(np.tril(U[:, :k], -1) == 0.0)
    assert np.max(np.abs(U)) <= 1.0 + 1e-6
    return f, ref, r_gpu


@pytest.mark.parametrize("pw", [0, 1, 2])
@pytest.mark.parametrize("m,n,k,p_over", [(1200, 900, 20, 10), (901, 1300, 64, 0),
                                          (2000, 1999, 100, 10)])
def test_randlu_against_oracle(h, m, n, k, p_over, pw):
    A = lowrank_plus_noise(m, n, spectrum("exp", min(m, n) // 2, tau=20.0), m + 3, n + 4, 1e-6, 5)
    # one input has an oracle row-pivot gap of 4.4e-5 (< tau) at step 95
    expect = (95, None) if (m, k, pw) == (2000, 100, 1) else (None, None)
    _check_randlu(h, A, k, p_over, pw, seed=m + 7 * pw, expect=expect)


@pytest.mark.parametrize("pw", [0, 1])
def test_randlu_column_major(h, pw):
    A = lowrank_plus_noise(1100, 800, spectrum("exp", 300, tau=15.0), 31, 32, 1e-6, 33)
    _check_randlu(h, A, 32, 8, pw, seed=40 + pw, col=True)


def test_randlu_k128_edge(h):
    A = lowrank_plus_noise(1500, 1400, spectrum("exp", 600, tau=60.0), 41, 42, 1e-6, 43)
    _check_randlu(h, A, 128, 4, 1, seed=44)


def test_randlu_exact_rank(h):
    rng = np.random.default_rng(4)
    A = (rng.standard_normal((800, 24)) @ rng.standard_normal((24, 700))).astype(np.float32)
    f, ref, r = _check_randlu(h, A, 24, 6, 1, seed=9)
    assert r < 1e-5


@pytest.mark.parametrize("pw", [1, 2])
def test_thm32_on_device(h, pw):
    """Range(P_r^T L_r) = Range(P_p^T L_p) for RandLU at p and PowerLU at
    v = 2p + 1 on the same Omega (Thm 3.2)."""
    A = lowrank_plus_noise(1500, 1200, spectrum("exp", 400, tau=8.0), 51, 52, 1e-7, 53)
    m, n = A.shape
    k, l = 20, 30
    Om = dev(gaussian_omega(n, l, seed=60 + pw))
    fr = h.randlu(dev(A), k, l - k, pw, Omega=Om)
    fp = h.fixed_rank(dev(A), k, l - k, 2 * pw + 1, Omega=Om)
    Pr = _proj(_scatter(host(fr.L), host(fr.p)))
    Pp = _proj(_scatter(host(fp.L), host(fp.p)))
    d = np.linalg.norm(Pr - Pp, 2)
    print(f"p {pw}: ||Pi_RandLU - Pi_PowerLU||_2 = {d:.3g}")
    assert d <= 1e-3


def test_randlu_argument_errors(h):
    A = dev(np.zeros((100, 80), np.float32))
    with pytest.raises(plu.PowerLUError):
        h.randlu(A, 0, 4, 1)
    with pytest.raises(plu.PowerLUError):
        h.randlu(A, 129, 0, 1)
    with pytest.raises(plu.PowerLUError):
        h.randlu(A, 70, 10, 1)          # l >= min(m, n)
    with pytest.raises(plu.PowerLUError):
        h.randlu(A, 10, 4, -1)
    torch.cuda.synchronize()


# ---------------------------------------------------------------- RandSVD
def _check_randsvd(h, A, k, p_over, pw, seed, col=False):
    m, n = A.shape
    l = k + p_over
    Om = gaussian_omega(n, l, seed=seed)
    U, S, V, info = h.randsvd(col_major(A) if col else dev(A), k, p_over, pw, Omega=dev(Om))
    ref = Bo.randsvd(A.astype(np.float64), k, Om.astype(np.float64), pw)
    U, S, V = (host(x).astype(np.float64) for x in (U, S, V))
    assert info["passes"] == 2 * pw + 2 and info["rank"] == k
    tol_s = 16 * l * U32
    ds = np.max(np.abs(S - ref.s)) / ref.s[0]
    ou = np.max(np.abs(U.T @ U - np.eye(k)))
    ov = np.max(np.abs(V.T @ V - np.eye(k)))
    r_gpu = Bo.svd_relative_residual(A, U, S, V)
    r_ref = Bo.svd_relative_residual(A, ref.U, ref.s, ref.V)
    print(f"{m}x{n} k {k} l {l} p {pw} col {col}: dS/s1 {ds:.2e} orth U {ou:.1e} V {ov:.1e} "
          f"residual gpu {r_gpu:.5g} oracle {r_ref:.5g}")
    assert np.all(np.diff(S) <= 0)
    assert ds <= tol_s
    assert ou <= tol_s and ov <= tol_s
    assert r_gpu <= 1.05 * r_ref + 64 * U32, (r_gpu, r_ref)
    sa = ref.s_all
    for j in range(min(k, 10)):
        gap = abs(sa[j] - sa[j + 1]) if j + 1 < len(sa) else sa[j]
        if j > 0:
            gap = min(gap, abs(sa[j - 1] - sa[j]))
        g = gap / sa[0]
        if g <= 1e-2:
            continue
        sg = np.sign(np.dot(U[:, j], ref.U[:, j]))
        assert np.max(np.abs(U[:, j] * sg - ref.U[:, j])) <= 1e-5 / g, j
        assert np.max(np.abs(V[:, j] * sg - ref.V[:, j])) <= 1e-5 / g, j
    return U, S, V, ref


@pytest.mark.parametrize("pw", [0, 1, 2])
@pytest.mark.parametrize("m,n,k,p_over", [(1200, 900, 20, 10), (901, 1300, 64, 0),
                                          (2000, 1999, 100, 10)])
def test_randsvd_against_oracle(h, m, n, k, p_over, pw):
    A = lowrank_plus_noise(m, n, spectrum("exp", min(m, n) // 2, tau=20.0), m + 5, n + 6, 1e-6, 7)
    _check_randsvd(h, A, k, p_over, pw, seed=m + 11 * pw)


def test_randsvd_column_major_and_l128(h):
    A = lowrank_plus_noise(1100, 1000, spectrum("exp", 400, tau=40.0), 61, 62, 1e-6, 63)
    _check_randsvd(h, A, 120, 8, 1, seed=64, col=True)


def test_randsvd_exact_rank(h):
    rng = np.random.default_rng(6)
    U0, _ = np.linalg.qr(rng.standard_normal((900, 10)))
    V0, _ = np.linalg.qr(rng.standard_normal((700, 10)))
    s0 = np.linspace(5.0, 0.5, 10)
    A = ((U0 * s0) @ V0.T).astype(np.float32)
    U, S, V, ref = _check_randsvd(h, A, 10, 4, 0, seed=2)
    assert np.max(np.abs(S - s0)) <= 1e-5 * s0[0]
    sg = np.sign(np.sum(U * U0, axis=0))
    assert np.max(np.abs(U * sg - U0)) <= 1e-4
    assert np.max(np.abs(V * sg - V0)) <= 1e-4


def test_randsvd_argument_errors(h):
    A = dev(np.zeros((400, 300), np.float32))
    with pytest.raises(plu.PowerLUError):
        h.randsvd(A, 0, 4, 1)
    with pytest.raises(plu.PowerLUError):
        h.randsvd(A, 120, 10, 1)        # l > 128
    with pytest.raises(plu.PowerLUError):
        h.randsvd(A, 10, 4, -1)
    torch.cuda.synchronize()
