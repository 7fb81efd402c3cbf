"""Full-size configurations.

* 32768 x 32768, rank 1000, sigma_i = i^-1.5, k = 200, p = 20, v = 4: the
  precision form (bfloat16 and block-scaled E4M3 passes, fp32 refinement).
  Error against the FP64 oracle on the 4096 x 4096 leading slice (both sides
  on the same slice and the same Omega); at full size the rounded forms'
  residuals against the fp32 path's and against the Eckart-Young optimum
  (closed form: the spectrum is known).
* 30000 x 20000, rank 2000, sigma_i = exp(-i/50), PowerLU_FP with eps = 1e-3,
  b = 32, l = 1600, v = 4: the rank against the truncated-SVD rank in closed
  form (Eckart-Young makes it a lower bound for any rank-k approximation;
  the indicator is Thm 4.3's exact error), the block rank, the residual.
"""

import numpy as np
import pytest

from tests.gpu_common import (torch, have_gpu, handle, dev, host, assert_pivots,
                               assert_pivots_measured, column_deviation)
from oracle import lowp as LP
from oracle import powerlu as O
from synth import WORKLOADS, gaussian_omega, workload_matrix

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

BF16, FP8, REFINE, REFINE_TWO = 1, 2, 16, 32


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


@pytest.fixture(scope="module")
def a32768():
    w = WORKLOADS["square32768_pow15"]
    return w, workload_matrix(w)


# (prec, rounding, exact closing passes, FP64 gate, pivot steps compared
# against the rounding-matched oracle (rows, columns; None = all k; the
# columns only when the rows agree in full), residual / FP64 oracle's on this
# slice as the oracle computes it)
SLICE_FORMS = [
    (BF16, LP.round_bf16, 0, True, (169, None), 1.0084),
    (BF16 | REFINE, LP.round_bf16, 1, True, (None, 11), 1.0009),
    (FP8 | REFINE, LP.round_mx_e4m3, 1, False, (17, None), 1.1788),
    (FP8 | REFINE_TWO, LP.round_mx_e4m3, 2, True, (34, None), 1.0295),
]


@pytest.mark.parametrize("prec,rnd,tail,gate_fp64,steps,ratio", SLICE_FORMS)
def test_precision_form_slice_4096_against_oracle(h, a32768, prec, rnd, tail, gate_fp64, steps,
                                                  ratio):
    """Every form matches the oracle's form of the same rounding (residual
    within 1.05x, pivots bit-exact up to the first step whose gap is below
    1e-3).  Against the FP64 oracle: the bfloat16 forms and the E4M3 form
    with two fp32 closing passes stay within 1.05x; the E4M3 form with one
    fp32 pass does not (1.18x: the E4M3 rounding error of A has spectral
    norm above sigma_201 here, so no rounded pass resolves the directions
    near k = 200; one exact power step does)."""
    w, A = a32768
    S = np.ascontiguousarray(A[:4096, :4096])
    k, p, v = 200, 20, 4
    Om = gaussian_omega(4096, k + p, seed=1000 * w.index + 3)
    f = h.fixed_rank(dev(S), k, p, v, Omega=dev(Om), prec=prec)
    S64, Om64 = S.astype(np.float64), Om.astype(np.float64)
    ref_f = O.powerlu(S64, k, Om64, v, pass_round=rnd, exact_tail=tail)
    ref_x = O.powerlu(S64, k, Om64, v)
    r_gpu = O.relative_residual(S, host(f.p), host(f.q), host(f.L), host(f.U))
    r_f = O.relative_residual(S, ref_f.p, ref_f.q, ref_f.L, ref_f.U)
    r_x = O.relative_residual(S, ref_x.p, ref_x.q, ref_x.L, ref_x.U)
    print(f"prec {prec}: slice residual gpu {r_gpu:.6e} oracle-form {r_f:.6e} oracle-fp64 "
          f"{r_x:.6e}; gpu / fp64 {r_gpu / r_x:.4f}")
    assert abs(r_f / r_x - ratio) <= 1e-3
    assert r_gpu <= 1.05 * r_f + 1e-7
    if gate_fp64:
        assert r_gpu <= 1.05 * r_x + 1e-7
    else:
        assert r_f > 1.05 * r_x
    sp = assert_pivots(host(f.p)[:k], ref_f.p[:k], ref_f.lu1.gaps, 1e-3, steps[0], "row pivots")
    if sp == k:
        assert_pivots(host(f.q)[:k], ref_f.q[:k], ref_f.lu2.gaps, 1e-3, steps[1], "column pivots")


def test_precision_form_full_size(h, a32768):
    w, A = a32768
    k, p, v = 200, 20, 4
    Ad = dev(A)
    sig = w.sigma()[:w.rank].astype(np.float64)
    optimal = np.sqrt(np.sum(sig[k:] ** 2) / np.sum(sig ** 2))
    res = {}
    for prec in (0, BF16, BF16 | REFINE, FP8, FP8 | REFINE, FP8 | REFINE_TWO):
        f = h.fixed_rank(Ad, k, p, v, seed=31, prec=prec)
        res[prec] = h.residual(Ad, f)
    print({p_: (r, r / optimal) for p_, r in res.items()})
    for prec, r in res.items():
        assert r >= optimal * (1 - 1e-4)            # Eckart-Young
    # at equal residual: the bfloat16 forms and the refined FP8 form within
    # 1.05 x the fp32 path's residual
    for prec in (BF16, BF16 | REFINE, FP8 | REFINE, FP8 | REFINE_TWO):
        assert res[prec] <= 1.05 * res[0], (prec, res[prec], res[0])


def _tsvd_rank(sig, eps, slack=0.0):
    """Smallest k with sum_{i>k} sigma_i^2 <= (eps^2 + slack) ||A||_F^2."""
    tail = np.cumsum((sig ** 2)[::-1])[::-1]          # tail[j] = sum_{i >= j} sigma_i^2
    total = np.sum(sig ** 2)
    for kk in range(len(sig) + 1):
        t = tail[kk] if kk < len(sig) else 0.0
        if t <= (eps * eps + slack) * total:
            return kk
    return len(sig)


@pytest.mark.parametrize("column_exact", [True, False])
def test_fixed_precision_30000x20000(h, column_exact):
    w = WORKLOADS["rect30000x20000_exp50"]
    A = workload_matrix(w)
    sig = w.sigma()[:w.rank].astype(np.float64)
    eps, b, l, v = 1e-3, 32, 1600, 4
    kstar = _tsvd_rank(sig, eps)
    # the fp32 indicator may sit below the exact one by about its measured
    # error (<= 3.6e-8 ||A||^2 in the n = 1000 parity runs): 5e-8 of slack
    klo = _tsvd_rank(sig, eps, slack=5e-8)
    Ad = dev(A)
    f = h.fixed_precision(Ad, eps, b, l=l, v=v, column_exact=column_exact, seed=41)
    r = h.residual(Ad, f)
    print(f"column {column_exact}: k_gpu {f.rank} k_tsvd {kstar} residual {r:.6e}")
    assert f.info["tol_reached"] == 1
    # the first k basis vectors capture less than the top-k singular
    # directions (Table 1 shows PowerLU_FP ranks a few above the truncated-SVD
    # ranks), so the column rank lies between the optimum and the block rank
    kblock = int(np.ceil(kstar / b) * b)
    if column_exact:
        assert klo <= f.rank <= kblock
    else:
        assert f.rank in (int(np.ceil(klo / b) * b), kblock)
    assert r * r <= eps * eps + 5e-8
    # L U is a rank-k factorization: the residual is at least the optimum
    assert r * r >= np.sum(sig[f.rank:] ** 2) / np.sum(sig ** 2) * (1 - 1e-3)


@pytest.mark.parametrize("column_exact", [True, False])
def test_fixed_precision_6000x4000_l1024_against_oracle(h, column_exact):
    """The 30000 x 20000 workload's recipe at 6000 x 4000 (same spectrum
    exp(-i/50), rank 2000 and seeds) with l = 1024 -- eight 128-column QR
    blocks and eight LU panels of l columns, the multi-block path of the
    l = 1600 configuration -- against the FP64 oracle (Alg. 9 on Alg. 8 /
    Alg. 11): the indicator within the fp32 basis' orthogonality band of the
    oracle's (4e-7 ||A||^2 for several blocks), the rank in the band it
    allows, pivots of both final LUs bit-exact over the steps decided above
    the measured deviation of the fp32 basis, residual within 1.05x of the
    oracle's at that rank and within eps."""
    w = WORKLOADS["rect30000x20000_exp50"]
    A = workload_matrix(w, 6000, 4000)
    eps, b, l, v = 1e-3, 32, 1024, 4
    Om = gaussian_omega(6000, l, seed=1000 * w.index + 3)
    f = h.fixed_precision(dev(A), eps, b, l=l, v=v, column_exact=column_exact, Omega=dev(Om))
    A64 = A.astype(np.float64)
    ref = O.powerlu_fp(A64, eps, b, Om.astype(np.float64), v, column_exact)
    acc = eps * eps * ref.normA2
    delta = 4e-7 * ref.normA2
    k = f.rank
    print(f"column {column_exact}: k_gpu {k} k_oracle {ref.rank} E_gpu/acc "
          f"{f.info['E_final'] / acc:.6f} E_oracle(k)/acc {ref.E[k - 1] / acc:.6f}")
    assert f.info["tol_reached"] == 1 and f.info["passes"] == v
    assert abs(f.info["E_final"] - ref.E[k - 1]) <= delta
    step = 1 if column_exact else b
    assert ref.E[k - 1] <= acc + delta and ref.E[k - 1 - step] >= acc - delta, (k, ref.rank)
    # the oracle's factorization at the GPU's rank (GETRF's first steps do not
    # depend on later columns, so p is the oracle's for any rank)
    fk = O.assemble(A64, ref.V[:, :k], ref.G[:, :k]) if k != ref.rank else ref
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    # The basis columns near k carry the largest fp32 deviation (sigma_k /
    # sigma_1 ~ 1e-3 here): measured on the same kernels' basis, up to 5e-3
    # per column, and the pivot steps are compared while the oracle's gap
    # stays 10x above the deviation of the columns that decide them.
    Vg = host(h.range_basis(dev(A), l, v, Omega=dev(Om)))[:, :k].astype(np.float64)
    cd = column_deviation(Vg, ref.V[:, :k])
    sp = assert_pivots_measured(p[:k], fk.p[:k], fk.lu1.gaps, cd, min_steps=k // 4,
                                what="row pivots")
    sq = assert_pivots_measured(q[:k], fk.q[:k], fk.lu2.gaps, cd, min_steps=k // 4,
                                what="column pivots")
    print(f"pivot steps compared: rows {sp}, columns {sq} of {k}; basis column deviation "
          f"max {cd.max():.2e}, median {np.median(cd):.2e}")
    r_gpu = O.relative_residual(A, p, q, L[:, :k], U[:k])
    r_ref = O.relative_residual(A, fk.p, fk.q, fk.L, fk.U)
    print(f"residual gpu {r_gpu:.6e} oracle {r_ref:.6e}")
    assert r_gpu <= 1.05 * r_ref + 1e-7
    assert r_gpu * r_gpu <= eps * eps + 2 * delta / ref.normA2
