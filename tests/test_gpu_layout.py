"""Column-major A (plu_layout PLU_COL_MAJOR) through the C ABI.

A column-major A is the row-major storage of A^T, so the library runs the
same kernels with the two pass directions swapped.  Gates:
  * the fixed-rank and fixed-precision results against the FP64 oracle under
    the row-major path's gates (pivots up to the gap rule, residual within
    1.05x of the oracle's, the same rank band);
  * the bfloat16 range basis is bit-identical between the two storage orders
    (both round A to the same codes and multiply the same copies);
  * plu_residual on the same factors agrees between the storage orders;
  * batched and served problems with a column-major A equal the single call
    bit for bit.
"""

import numpy as np
import pytest

import paper_2002_07138_amd as plu
from tests.gpu_common import torch, have_gpu, handle, dev, host, assert_pivots, assert_factors_close
from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, paper_type, spectrum

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

TAU = 1e-4


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


def col_major(A, pad=0):
    """Device copy of A stored column-major with leading dimension m + pad."""
    m, n = A.shape
    buf = torch.full((n, m + pad), float("nan"), dtype=torch.float32, device="cuda")
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda")
    Ac = buf.t()[:m, :]
    assert Ac.stride() == (1, m + pad)
    return Ac


@pytest.mark.parametrize("m,n,k,p_over,v,pad", [(1200, 900, 20, 10, 3, 0), (901, 1300, 33, 0, 2, 5),
                                                (2000, 1999, 64, 16, 4, 3), (515, 700, 7, 5, 5, 0)])
def test_fixed_rank_column_major_against_oracle(h, m, n, k, p_over, v, pad):
    A = lowrank_plus_noise(m, n, spectrum("exp", min(m, n) // 2, tau=20.0), m + 1, n + 2, 1e-6, 9)
    l = k + p_over
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=m * 7 + n)
    f = h.fixed_rank(col_major(A, pad), k, p_over, v, Omega=dev(Om))
    ref = O.powerlu(A.astype(np.float64), k, Om.astype(np.float64), v)
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    assert sorted(p.tolist()) == list(range(m)) and sorted(q.tolist()) == list(range(n))
    r_gpu = O.relative_residual(A, p, q, L, U)
    r_ref = O.relative_residual(A, ref.p, ref.q, ref.L, ref.U)
    assert r_gpu <= 1.05 * r_ref + 1e-7, (r_gpu, r_ref)
    sp = assert_pivots(p[:k], ref.p[:k], ref.lu1.gaps, TAU, None, "row pivots")
    sq = assert_pivots(q[:k], ref.q[:k], ref.lu2.gaps, TAU, None, "column pivots")
    if sp == k and sq == k:
        assert_factors_close(L, U, ref.L, ref.U)
    # the same factors' residual on the GPU, from either storage order
    r_col = h.residual(col_major(A, pad), f)
    r_row = h.residual(dev(A), f)
    assert abs(r_col - r_row) <= 1e-9 * max(r_row, 1e-30)
    assert abs(r_col - r_gpu) <= 1e-4 * r_gpu + 1e-9


@pytest.mark.parametrize("typ,eps,l,b", [(1, 1e-3, 120, 10), (3, 1e-2, 120, 10), (2, 1e-3, 300, 10)])
def test_fixed_precision_column_major_against_oracle(h, typ, eps, l, b):
    """Matrix Types of Sec. 6.2 at n = 800, column rule, under the row-major
    path's indicator band."""
    n = 800
    A = paper_type(typ, n, seed=40 + typ).astype(np.float32)
    Om = gaussian_omega(n, l, seed=typ * 11)
    f = h.fixed_precision(col_major(A, 2), eps, b, l=l, v=4, Omega=dev(Om))
    ref = O.powerlu_fp(A.astype(np.float64), eps, b, Om.astype(np.float64), 4, True)
    acc = eps * eps * ref.normA2
    delta = (2e-8 if l <= 128 else 4e-7) * ref.normA2
    k = f.rank
    assert abs(f.info["E_final"] - ref.E[k - 1]) <= delta
    assert ref.E[k - 1] <= acc + delta
    assert k == 1 or ref.E[k - 2] >= acc - delta
    assert f.info["tol_reached"] == 1
    r = O.relative_residual(A, host(f.p), host(f.q), host(f.L), host(f.U))
    assert r * r <= eps * eps + 2 * delta / ref.normA2
    # the row-major call finds the same rank band
    fr = h.fixed_precision(dev(A), eps, b, l=l, v=4, Omega=dev(Om))
    assert abs(fr.rank - k) <= 1


def test_range_basis_bf16_bit_identical_across_layouts(h):
    m, n, l = 700, 520, 24
    A = lowrank_plus_noise(m, n, spectrum("exp", 100, tau=10.0), 3, 4, 1e-5, 5)
    for v in (2, 3, 4):
        Om = dev(gaussian_omega(m if v % 2 == 0 else n, l, seed=v))
        Vr = h.range_basis(dev(A), l, v, Omega=Om, prec=plu.PREC_BF16)
        Vc = h.range_basis(col_major(A, 7), l, v, Omega=Om, prec=plu.PREC_BF16)
        torch.cuda.synchronize()
        assert torch.equal(Vr, Vc), v


def test_range_basis_fp32_close_across_layouts(h):
    m, n, l = 640, 900, 30
    A = lowrank_plus_noise(m, n, spectrum("exp", 200, tau=8.0), 6, 7, 1e-5, 8)
    for v in (2, 3, 5):
        Om = dev(gaussian_omega(m if v % 2 == 0 else n, l, seed=10 + v))
        Vr = host(h.range_basis(dev(A), l, v, Omega=Om))
        Vc = host(h.range_basis(col_major(A), l, v, Omega=Om))
        # the passes differ only in summation order; compare the leading
        # (well-separated) columns up to sign
        s = np.sign(np.sum(Vr[:, :10] * Vc[:, :10], axis=0))
        assert np.max(np.abs(Vr[:, :10] - Vc[:, :10] * s)) <= 2e-3


def test_batched_column_major_equals_single(h):
    probs = []
    for i, (m, n) in enumerate([(700, 600), (512, 900), (1000, 1000)]):
        A = lowrank_plus_noise(m, n, spectrum("exp", 64, tau=12.0), 20 + i, 30 + i, 1e-5, 40 + i)
        Ac = col_major(A, i)
        if i % 2 == 0:
            probs.append(dict(A=Ac, mode=0, k=16, p_over=8, v=3, seed=100 + i))
        else:
            probs.append(dict(A=Ac, mode=1, eps=1e-3, b=8, l=96, v=4, seed=100 + i))
    out = h.batched(probs)
    for pr, fb in zip(probs, out):
        if pr["mode"] == 0:
            fs = h.fixed_rank(pr["A"], pr["k"], pr["p_over"], pr["v"], seed=pr["seed"])
        else:
            fs = h.fixed_precision(pr["A"], pr["eps"], pr["b"], l=pr["l"], v=pr["v"],
                                   seed=pr["seed"])
        assert fb.rank == fs.rank
        for a, b in ((fb.p, fs.p), (fb.q, fs.q), (fb.L, fs.L), (fb.U, fs.U)):
            assert torch.equal(a, b)


def test_server_column_major_host_input_equals_single(h):
    m, n = 800, 650
    A = lowrank_plus_noise(m, n, spectrum("exp", 64, tau=10.0), 61, 62, 1e-5, 63)
    A_f = np.asfortranarray(A)          # host, columns contiguous
    srv = plu.Server(0, hbm_budget_bytes=1 << 30, max_slots=4)
    try:
        t0 = srv.submit(A_f, mode=0, k=20, p_over=10, v=3, seed=5)
        t1 = srv.submit(A_f, mode=1, eps=1e-3, b=8, l=120, v=4, seed=6)
        r0, r1 = srv.wait(t0), srv.wait(t1)
    finally:
        srv.close()
    f0 = h.fixed_rank(col_major(A), 20, 10, 3, seed=5)
    f1 = h.fixed_precision(col_major(A), 1e-3, 8, l=120, v=4, seed=6)
    for r, f in ((r0, f0), (r1, f1)):
        k = r["rank"]
        assert k == f.rank
        assert np.array_equal(r["p"], host(f.p)) and np.array_equal(r["q"], host(f.q))
        assert np.array_equal(r["L"][:, :k], host(f.L)[:, :k])
        assert np.array_equal(r["U"][:k], host(f.U)[:k])
