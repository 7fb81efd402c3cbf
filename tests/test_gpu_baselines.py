"""RandLU (Alg. 3 + Alg. 4) on the GPU against the FP64 oracle, through the C
ABI, in both storage orders of A.

Gates, as for PowerLU's end-to-end tests:
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
"""

import numpy as np
import pytest

import paper_2002_07138_amd as plu
from tests.gpu_common import torch, have_gpu, handle, dev, host, pivot_prefix_ok
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


def _check_randlu(h, A, k, p_over, pw, seed, col=False):
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
    okp, stop_p = pivot_prefix_ok(p[:k], ref.p[:k], ref.lu1.gaps, TAU)
    assert okp, f"row pivots differ before step {stop_p}"
    if stop_p == k:
        okq, stop_q = pivot_prefix_ok(q[:k], ref.q[:k], ref.lu2.gaps, TAU)
        assert okq, f"column pivots differ before step {stop_q}"
        if stop_q == k:
            assert np.max(np.abs(L - ref.L)) <= 1e-3 * np.max(np.abs(ref.L))
            assert np.max(np.abs(U - ref.U)) <= 1e-3
    assert np.allclose(np.diag(U[:, :k]), 1.0) and np.all(np.tril(U[:, :k], -1) == 0.0)
    assert np.max(np.abs(U)) <= 1.0 + 1e-6
    return f, ref, r_gpu


@pytest.mark.parametrize("pw", [0, 1, 2])
@pytest.mark.parametrize("m,n,k,p_over", [(1200, 900, 20, 10), (901, 1300, 64, 0),
                                          (2000, 1999, 100, 10)])
def test_randlu_against_oracle(h, m, n, k, p_over, pw):
    A = lowrank_plus_noise(m, n, spectrum("exp", min(m, n) // 2, tau=20.0), m + 3, n + 4, 1e-6, 5)
    _check_randlu(h, A, k, p_over, pw, seed=m + 7 * pw)


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
