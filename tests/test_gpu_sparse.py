"""Sparse A (compressed rows; the sprand inputs of Sec. 6.1) through the C ABI.

The passes are the only part that changes, so the gates are:
  * plu_sparse_pass against the float64 product of the dense matrix, within
    the float32 accumulation bound c u32 (|A| |X|) elementwise, with c the
    longest row (or column) plus one; bitwise repeatable; A^T Y bitwise
    independent of the order of the entries within a row (the compressed
    columns are sorted by row on the device);
  * malformed compressed rows are refused with the argument's index (the
    structure is checked before any index is used);
  * PowerLU, PowerLU_FP, RandLU and RandSVD on the sparse form against the
    FP64 oracle on the same matrix made dense, under the dense path's gates
    (pivots up to the gap rule, residual within 1.05x + 64 u32, the
    indicator band, the singular values).
"""

import numpy as np
import pytest

import paper_2002_07138_amd as plu
from tests.gpu_common import torch, have_gpu, handle, dev, host, assert_pivots, assert_factors_close
from oracle import baselines as Bo
from oracle import powerlu as O
from synth import csr_dense, gaussian_omega, sprand_csr

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

TAU = 1e-4
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


def _bind(h, m, n, ip, ix, d):
    return h.sparse_matrix(torch.from_numpy(ip).cuda(), torch.from_numpy(ix).cuda(),
                           torch.from_numpy(d).cuda(), (m, n))


def _mat(h, m, n, density, seed):
    ip, ix, d = sprand_csr(m, n, density, seed)
    return _bind(h, m, n, ip, ix, d), csr_dense(m, n, ip, ix, d), (ip, ix, d)


@pytest.mark.parametrize("m,n,density,l", [(3000, 2000, 0.003, 110), (1500, 2500, 0.01, 37),
                                           (700, 900, 0.05, 300)])
def test_sparse_pass_against_dense_product(h, m, n, density, l):
    S, A, (ip, ix, d) = _mat(h, m, n, density, m + n)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((n, l)).astype(np.float32)
    Y = rng.standard_normal((m, l)).astype(np.float32)
    for trans, In, ref_of in ((False, X, lambda M: A @ M), (True, Y, lambda M: A.T @ M)):
        out = host(h.sparse_pass(S, dev(In), trans=trans)).astype(np.float64)
        ref = ref_of(In.astype(np.float64))
        bound_m = np.abs(A.T if trans else A) @ np.abs(In.astype(np.float64))
        c = int(np.max(np.count_nonzero(A, axis=0 if trans else 1))) + 1
        assert np.all(np.abs(out - ref) <= c * U32 * bound_m + 1e-30), trans
        again = host(h.sparse_pass(S, dev(In), trans=trans))
        assert np.array_equal(again, out.astype(np.float32)), "not repeatable"
    S.close()


def test_sparse_transpose_independent_of_row_order(h):
    m, n = 1200, 900
    ip, ix, d = sprand_csr(m, n, 0.01, 7)
    rng = np.random.default_rng(3)
    ix2, d2 = ix.copy(), d.copy()
    for i in range(m):                      # shuffle the entries within every row
        a, b = ip[i], ip[i + 1]
        perm = rng.permutation(b - a)
        ix2[a:b] = ix[a:b][perm]
        d2[a:b] = d[a:b][perm]
    S1 = _bind(h, m, n, ip, ix, d)
    S2 = _bind(h, m, n, ip, ix2, d2)
    Y = dev(rng.standard_normal((m, 50)).astype(np.float32))
    assert torch.equal(h.sparse_pass(S1, Y, trans=True), h.sparse_pass(S2, Y, trans=True))
    S1.close()
    S2.close()


def test_sparse_malformed_is_refused(h):
    m, n = 100, 80
    ip, ix, d = sprand_csr(m, n, 0.05, 9)
    bad_ptr = ip.copy()
    bad_ptr[50] = bad_ptr[51] + 1           # decreasing
    with pytest.raises(plu.PowerLUError) as ei:
        _bind(h, m, n, bad_ptr, ix, d)
    assert ei.value.code == -5
    bad_idx = ix.copy()
    bad_idx[3] = n                          # out of range
    with pytest.raises(plu.PowerLUError) as ei:
        _bind(h, m, n, ip, bad_idx, d)
    assert ei.value.code == -6
    short = ip.copy()
    short[-1] -= 1                          # rowptr[m] != nnz
    with pytest.raises(plu.PowerLUError) as ei:
        _bind(h, m, n, short, ix, d)
    assert ei.value.code == -5
    torch.cuda.synchronize()


def test_sparse_empty_matrix(h):
    m, n = 300, 200
    S = _bind(h, m, n, np.zeros(m + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.float32))
    X = dev(np.ones((n, 8), np.float32))
    assert float(h.sparse_pass(S, X).abs().max()) == 0.0
    S.close()


@pytest.mark.parametrize("v", [2, 3, 4, 5])
@pytest.mark.parametrize("m,n,density,k,p_over", [(1500, 1200, 0.01, 20, 10),
                                                  (2000, 2400, 0.004, 64, 8)])
def test_sparse_fixed_rank_against_oracle(h, m, n, density, k, p_over, v):
    S, A, _ = _mat(h, m, n, density, 11 * m + v)
    l = k + p_over
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=v + m)
    f = h.fixed_rank(S, k, p_over, v, Omega=dev(Om))
    ref = O.powerlu(A, k, Om.astype(np.float64), v)
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    r_gpu = O.relative_residual(A, p, q, L, U)
    r_ref = O.relative_residual(A, ref.p, ref.q, ref.L, ref.U)
    print(f"sparse {m}x{n} d {density} k {k} v {v}: residual gpu {r_gpu:.6g} oracle {r_ref:.6g}")
    assert abs(f.info["normA2"] - float(np.sum(A * A))) <= 1e-12 * float(np.sum(A * A))
    assert r_gpu <= 1.05 * r_ref + 64 * U32
    sp = assert_pivots(p[:k], ref.p[:k], ref.lu1.gaps, TAU, None, "row pivots")
    sq = assert_pivots(q[:k], ref.q[:k], ref.lu2.gaps, TAU, None, "column pivots")
    if sp == k and sq == k:
        assert_factors_close(L, U, ref.L, ref.U)
    S.close()


def test_sparse_fixed_precision_against_oracle(h):
    m, n = 1400, 1100
    S, A, _ = _mat(h, m, n, 0.02, 5)
    eps, b, l = 0.85, 8, 200          # truncated-SVD rank 98 for this matrix
    Om = gaussian_omega(m, l, seed=21)
    f = h.fixed_precision(S, eps, b, l=l, v=4, Omega=dev(Om))
    ref = O.powerlu_fp(A, eps, b, Om.astype(np.float64), 4, True)
    acc = eps * eps * ref.normA2
    delta = 2e-7 * ref.normA2
    k = f.rank
    print(f"sparse fp: k_gpu {k} k_oracle {ref.rank}")
    assert f.info["tol_reached"] == 1 and ref.tol_reached
    assert abs(f.info["E_final"] - ref.E[k - 1]) <= delta
    assert ref.E[k - 1] <= acc + delta and (k == 1 or ref.E[k - 2] >= acc - delta)
    r = O.relative_residual(A, host(f.p), host(f.q), host(f.L), host(f.U))
    assert r * r <= eps * eps + 2 * delta / ref.normA2
    S.close()


@pytest.mark.parametrize("pw", [0, 1])
def test_sparse_randlu_randsvd_against_oracle(h, pw):
    m, n = 1600, 1300
    S, A, _ = _mat(h, m, n, 0.01, 31 + pw)
    k, p_over = 30, 10
    Om = gaussian_omega(n, k + p_over, seed=40 + pw)
    f = h.randlu(S, k, p_over, pw, Omega=dev(Om))
    ref = Bo.randlu(A, k, Om.astype(np.float64), pw)
    r_gpu = O.relative_residual(A, host(f.p), host(f.q), host(f.L), host(f.U))
    r_ref = O.relative_residual(A, ref.p, ref.q, ref.L, ref.U)
    assert r_gpu <= 1.05 * r_ref + 64 * U32
    U, s, V, info = h.randsvd(S, k, p_over, pw, Omega=dev(Om))
    sref = Bo.randsvd(A, k, Om.astype(np.float64), pw)
    s = host(s).astype(np.float64)
    assert np.max(np.abs(s - sref.s)) <= 16 * (k + p_over) * U32 * sref.s[0]
    rs = Bo.svd_relative_residual(A, host(U), s, host(V))
    rs_ref = Bo.svd_relative_residual(A, sref.U, sref.s, sref.V)
    print(f"sparse p {pw}: RandLU {r_gpu:.6g} / {r_ref:.6g}, RandSVD {rs:.6g} / {rs_ref:.6g}")
    assert rs <= 1.05 * rs_ref + 64 * U32
    S.close()


def test_sparse_argument_errors(h):
    S, A, _ = _mat(h, 300, 250, 0.02, 3)
    with pytest.raises(plu.PowerLUError) as ei:
        h.fixed_rank(S, 10, 4, 3, prec=plu.PREC_BF16)
    assert ei.value.code == -6          # prec, index 6 in the sparse signature
    with pytest.raises(plu.PowerLUError) as ei:
        h.fixed_rank(S, 0, 4, 3)
    assert ei.value.code == -3          # k
    S.close()
    torch.cuda.synchronize()
