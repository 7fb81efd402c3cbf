"""Precision form of the passes (bfloat16 operands, fp32 accumulation, fp32
refinement pass) on the GPU against the oracle's precision form and against
the plain FP64 oracle, through the C ABI.

Gates:
  * rounding of the operands: bit-exact against the oracle's bfloat16 rule;
  * one pass: within the fp32-accumulation bound of the exact product of the
    rounded operands;
  * PowerLU: pivots bit-exact up to the first final-LU step whose oracle gap
    is below TAU_BF16 = 1e-3 (the iterate is rounded to bfloat16 from fp32 on
    the GPU and from fp64 in the oracle, so a handful of entries sit on the
    other side of a bfloat16 rounding boundary: relative perturbations of
    about 2^-8 / sqrt(K) in the pass outputs); residual <= 1.05 x the
    oracle's precision form and <= 1.05 x the plain FP64 oracle's;
  * PowerLU_FP: the rank band and indicator gate of the fp32 path.
"""

import numpy as np
import pytest

from tests.gpu_common import torch, have_gpu, handle, dev, host, equal_up_to_signs, assert_pivots
from oracle import lowp as LP
from oracle import powerlu as O
from synth import WORKLOADS, gaussian_omega, lowrank_plus_noise, paper_type, spectrum, workload_matrix

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

TAU_BF16 = 1e-3

# Pivot steps compared against the rounding-matched oracle on the inputs whose
# oracle gap sequence falls below TAU_BF16 before step k (all others are
# compared in full): (form, m, n, k, v) -> (row steps, column steps); the
# column order is compared only when the row order agrees in full.
PIVOT_STEPS = {
    ("bf16", 2000, 2000, 20, 2): (None, 13), ("bf16", 2000, 2000, 20, 5): (7, None),
    ("bf16", 901, 1300, 33, 2): (None, 7), ("bf16", 3000, 2999, 100, 4): (11, None),
    ("fp8", 2000, 2000, 20, 3): (None, 0), ("fp8", 2000, 2000, 20, 4): (None, 0),
    ("bf16+r", 2000, 2000, 20, 5): (7, None), ("fp8+r", 2000, 2000, 20, 5): (11, None),
    ("fp8+r2", 2000, 2000, 20, 4): (4, None), ("bf16+r2", 2000, 2000, 20, 5): (7, None),
    ("fp8+r2", 2000, 2000, 20, 5): (11, None),
}


def _pivots_vs_form(p, q, ref, k, key):
    """Pivots against the rounding-matched oracle.  Reduced-precision forms are
    exempt from the bit-exact pivot gate; what is compared is a check beyond
    it.  E4M3: the row order only -- an fp32 iterate that differs from the
    oracle's float64 one in its last bits can round to a neighbouring E4M3
    code (a 2^-4 relative step of that entry), and the column gaps of
    lu(B^T) measured on the device move by up to 4e-3 against the oracle's,
    above TAU_BF16."""
    ep, eq = PIVOT_STEPS.get(key, (None, None))
    sp = assert_pivots(p[:k], ref.p[:k], ref.lu1.gaps, TAU_BF16, ep, "row pivots")
    if sp == k and not key[0].startswith("fp8"):
        assert_pivots(q[:k], ref.q[:k], ref.lu2.gaps, TAU_BF16, eq, "column pivots")
BF16 = 1

# Indicator gate of the rounded forms.  The GPU rounds its fp32 iterate and
# the oracle its fp64 iterate to the narrow format; the few entries whose two
# values straddle a rounding boundary differ by one ulp of that format
# (2^-8 relative for bfloat16, 2^-3 for E4M3), which moves the captured
# energy by far more than the fp32 rounding the fp32 path's band covers.
# Expected size ~ P(straddle) x ulp^2 ~ u32 x ulp; measured up to 2.5e-8 of
# ||A||^2 for bfloat16.  The band is 10x that for bfloat16, scaled by the
# ulp ratio (32x) for E4M3.
DELTA_FORM = {"bf16": 2e-7, "fp8": 6.4e-6}


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


def _reached_consistent(f, ref, k, acc, delta):
    """Where the oracle's indicator is clearly below the threshold the GPU
    must report the tolerance reached; within the band either report is
    right (when eps^2 ||A||^2 is below the band, the rounded forms cannot
    certify the tolerance, and report the rank-l result)."""
    if ref.tol_reached and ref.E[k - 1] <= acc - delta:
        assert f.info["tol_reached"] == 1


# ---------------------------------------------------------------- operand rounding
@pytest.mark.parametrize("rows,cols", [(333, 101), (64, 64), (1, 7), (700, 1)])
@pytest.mark.parametrize("transpose", [False, True])
def test_quantize_bf16_bit_exact(h, rows, cols, transpose):
    rng = np.random.default_rng(rows * 31 + cols)
    X = (rng.standard_normal((rows, cols)) * 10.0 ** rng.integers(-20, 20, (rows, cols))).astype(np.float32)
    # exact ties on the discarded half, signed zeros, subnormals, infinities
    flat = X.reshape(-1)
    specials = np.array([0.0, -0.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1e-40, -1e-42, np.inf, -np.inf,
                         3.3895e38], dtype=np.float32)
    flat[:min(len(flat), len(specials))] = specials[:min(len(flat), len(specials))]
    ties = rng.integers(0, len(flat), size=min(50, len(flat)))
    flat[ties] = (flat[ties].view(np.uint32) & np.uint32(0xFFFF0000) | np.uint32(0x8000)).view(np.float32)
    codes = host(h.quantize(dev(X), transpose=transpose)).view(np.uint16)
    ref = LP.bf16_bits(X.T if transpose else X)
    r, c = ref.shape
    assert np.array_equal(codes[:, :c], ref)
    assert np.all(codes[:, c:] == 0)
    assert codes.shape[1] % 64 == 0


# ---------------------------------------------------------------- one pass
@pytest.mark.parametrize("m,n,l", [(1000, 777, 30), (3001, 2500, 110), (517, 4133, 13),
                                   (256, 256, 16), (9000, 300, 133), (300, 9000, 250),
                                   (2001, 1500, 220), (70, 65, 1), (1, 700, 5), (700, 1, 5)])
@pytest.mark.parametrize("trans", [False, True])
def test_pass_bf16_matches_rounded_product(h, m, n, l, trans):
    rng = np.random.default_rng(m * 7 + n + l + 1)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((m if trans else n, l)).astype(np.float32)
    nA2 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    out = host(h.pass_(dev(A), dev(X), trans=trans, prec=BF16, normA2=nA2))
    Ar = LP.round_bf16(A)
    Xr = LP.round_bf16(X)
    ref = (Ar.T if trans else Ar) @ Xr
    K = m if trans else n
    # exact products of bfloat16 values, fp32 accumulation over K terms
    tol = 8.0 * np.sqrt(K) * 6e-8 * np.sqrt(K)
    assert np.max(np.abs(out - ref)) < tol
    nref = np.sum(A.astype(np.float64) ** 2)
    assert abs(float(nA2.cpu()) - nref) <= 1e-12 * nref
    # and the rounding is visible: the fp32 product differs at the bfloat16 level
    exact = (A.astype(np.float64).T if trans else A.astype(np.float64)) @ X.astype(np.float64)
    if K >= 64:
        assert np.max(np.abs(out - exact)) > 10 * tol


# ---------------------------------------------------------------- Alg. 7 in the precision form
@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_range_basis_bf16_matches_oracle(h, v):
    m, n, l = 1500, 1200, 30
    A = lowrank_plus_noise(m, n, spectrum("exp", 200, tau=15.0), 21, 22, 1e-6, 23)
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=24 + v)
    V = host(h.range_basis(dev(A), l, v, Omega=dev(Om), prec=BF16)).astype(np.float64)
    Vr = O.range_basis(A.astype(np.float64), Om.astype(np.float64), v, pass_round=LP.round_bf16)
    assert np.max(np.abs(V.T @ V - np.eye(l))) < 2e-5
    ok, worst = equal_up_to_signs(V[:, :20], Vr[:, :20], 2e-3)
    assert ok, worst


def _check_bf16_fixed_rank(h, A, k, p_over, v, seed):
    m, n = A.shape
    l = k + p_over
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=seed)
    f = h.fixed_rank(dev(A), k, p_over, v, Omega=dev(Om), prec=BF16)
    A64, Om64 = A.astype(np.float64), Om.astype(np.float64)
    ref_b = O.powerlu(A64, k, Om64, v, pass_round=LP.round_bf16)
    ref_x = O.powerlu(A64, k, Om64, v)
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    r_gpu = O.relative_residual(A, p, q, L, U)
    r_b = O.relative_residual(A, ref_b.p, ref_b.q, ref_b.L, ref_b.U)
    r_x = O.relative_residual(A, ref_x.p, ref_x.q, ref_x.L, ref_x.U)
    print(f"v {v}: residual gpu-bf16 {r_gpu:.6e} oracle-bf16 {r_b:.6e} oracle-fp64 {r_x:.6e}")
    assert r_gpu <= 1.05 * r_b + 1e-7, (r_gpu, r_b)
    assert r_gpu <= 1.05 * r_x + 1e-7, (r_gpu, r_x)
    _pivots_vs_form(p, q, ref_b, k, ("bf16", m, n, k, v))
    assert np.allclose(np.diag(U[:, :k]), 1.0) and np.max(np.abs(U)) <= 1.0 + 1e-6
    assert f.info["passes"] == v
    return r_gpu, r_b, r_x


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_fixed_rank_bf16_square2000_type1(h, v):
    w = WORKLOADS["square2000_type1"]
    A = workload_matrix(w)
    _check_bf16_fixed_rank(h, A, 20, 10, v, seed=1000 * w.index + 3)


@pytest.mark.parametrize("m,n,k,p_over,v", [(1200, 900, 7, 5, 3), (901, 1300, 33, 0, 2),
                                            (3000, 2999, 100, 10, 4), (515, 530, 1, 3, 5)])
def test_fixed_rank_bf16_shapes(h, m, n, k, p_over, v):
    A = lowrank_plus_noise(m, n, spectrum("exp", min(m, n) // 2, tau=20.0), m, n, 1e-6, 7)
    _check_bf16_fixed_rank(h, A, k, p_over, v, seed=m + n)


@pytest.mark.parametrize("t,eps,l,b", [(2, 1e-4, 120, 10), (2, 1e-3, 120, 10), (3, 1e-2, 120, 10),
                                       (1, 1e-3, 500, 10), (1, 1e-2, 120, 10)])
def test_fixed_precision_bf16_paper_types(h, t, eps, l, b):
    n = 1000
    A = paper_type(t, n, seed=300 + t).astype(np.float32)
    Om = gaussian_omega(n, l, seed=400 + t)
    f = h.fixed_precision(dev(A), eps, b, l=l, v=4, column_exact=True, Omega=dev(Om), prec=BF16)
    ref = O.powerlu_fp(A.astype(np.float64), eps, b, Om.astype(np.float64), 4, True,
                       pass_round=LP.round_bf16)
    acc = eps * eps * ref.normA2
    delta = DELTA_FORM["bf16"] * ref.normA2
    k = f.rank
    print(f"type {t} eps {eps}: k_gpu {k} k_oracle_bf16 {ref.rank} "
          f"indicator diff/nA2 {abs(f.info['E_final'] - ref.E[k - 1]) / ref.normA2:.2e}")
    assert abs(f.info["E_final"] - ref.E[k - 1]) <= delta
    E = ref.E
    if E[-1] > acc + delta:
        # the rounded passes cannot resolve eps^2 ||A||^2 (a basis built from
        # bfloat16 data misses about u_bf16^2 of the energy): both sides
        # report the rank-l result with the tolerance not reached
        assert not ref.tol_reached and k == l and f.info["tol_reached"] == 0
        return
    assert E[k - 1] <= acc + delta and (k < 2 or E[k - 2] >= acc - delta), (k, ref.rank)
    _reached_consistent(f, ref, k, acc, delta)
    if f.info["tol_reached"]:
        r = O.relative_residual(A, host(f.p), host(f.q), host(f.L), host(f.U))
        assert r * r <= eps * eps + 2 * delta / ref.normA2


# ---------------------------------------------------------------- FP8 E4M3 with block scales
FP8 = 2


@pytest.mark.parametrize("rows,cols", [(333, 101), (128, 128), (1, 7), (700, 1), (257, 300)])
@pytest.mark.parametrize("transpose", [False, True])
def test_quantize_fp8_bit_exact(h, rows, cols, transpose):
    rng = np.random.default_rng(rows * 17 + cols)
    X = (rng.standard_normal((rows, cols)) * 10.0 ** rng.integers(-12, 12, (rows, 1))).astype(np.float32)
    flat = X.reshape(-1)
    specials = np.array([0.0, -0.0, 448.0, -448.0, 1e-40, 2.0**-9, 3 * 2.0**-10], dtype=np.float32)
    flat[:min(len(flat), len(specials))] = specials[:min(len(flat), len(specials))]
    codes, sc = h.quantize(dev(X), fmt=FP8, transpose=transpose)
    codes, sc = host(codes), host(sc)
    Y = (X.T if transpose else X).astype(np.float64)          # blocks run along rows of Y
    e = LP.mx_exponents(Y, 1)
    K = Y.shape[1]
    scale = np.exp2(np.repeat(e, 32, axis=1)[:, :K].astype(np.float64))
    ref_codes = LP.e4m3_bits(LP.e4m3_round(Y / scale))
    assert np.array_equal(codes[:, :K], ref_codes)
    assert np.all(codes[:, K:] == 0)
    nb = (K + 31) // 32
    assert np.array_equal(sc[:, :nb].astype(np.int64), e + 127)
    assert np.all(sc[:, nb:] == 0)


@pytest.mark.parametrize("m,n,l", [(1000, 777, 30), (3001, 2500, 110), (517, 4133, 13),
                                   (300, 9000, 250), (9000, 300, 133), (2001, 1500, 220),
                                   (70, 65, 1), (1, 700, 5), (700, 1, 5)])
@pytest.mark.parametrize("trans", [False, True])
def test_pass_fp8_matches_rounded_product(h, m, n, l, trans):
    rng = np.random.default_rng(m * 5 + n + l + 2)
    A = (rng.standard_normal((m, n)) * np.exp(rng.uniform(-3, 3, (m, 1)))).astype(np.float32)
    X = rng.standard_normal((m if trans else n, l)).astype(np.float32)
    nA2 = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    out = host(h.pass_(dev(A), dev(X), trans=trans, prec=FP8, normA2=nA2))
    # ||A||_F^2 accumulated in float64 by the conversion kernel from the
    # float32 values it reads
    nref = np.sum(A.astype(np.float64) ** 2)
    assert abs(float(nA2.cpu()) - nref) <= 1e-12 * nref
    Ar = LP.round_mx_e4m3(A, 0 if trans else 1)
    Xr = LP.round_mx_e4m3(X, 0)
    ref = (Ar.T if trans else Ar) @ Xr
    K = m if trans else n
    scale = np.abs(Ar.T if trans else Ar) @ np.abs(Xr)
    # the products of scaled E4M3 values are exact (subnormal codes and
    # scales included, checked on the matrix core), but the 128 products of
    # one matrix-core step are not summed in fp32 arithmetic: on rows whose
    # entries span a wide range (here the transposed copy mixes row scales
    # of e^6) the step loses up to ~2^-14 of sum |a b| (measured 7.4e-5 at
    # K = 70).  Gate: the fp32-accumulation bound plus 2^-12 of sum |a b|.
    err = np.abs(out - ref)
    print(f"max |err| / sum|a b| = {np.max(err / np.maximum(scale, 1e-30)):.3e}")
    assert np.all(err <= (8.0 * K * 6e-8 + 2.0 ** -12) * scale + 1e-30)


def _check_fp8_fixed_rank(h, A, k, p_over, v, seed):
    m, n = A.shape
    l = k + p_over
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=seed)
    f = h.fixed_rank(dev(A), k, p_over, v, Omega=dev(Om), prec=FP8)
    A64, Om64 = A.astype(np.float64), Om.astype(np.float64)
    ref_8 = O.powerlu(A64, k, Om64, v, pass_round=LP.round_mx_e4m3)
    ref_x = O.powerlu(A64, k, Om64, v)
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    r_gpu = O.relative_residual(A, p, q, L, U)
    r_8 = O.relative_residual(A, ref_8.p, ref_8.q, ref_8.L, ref_8.U)
    r_x = O.relative_residual(A, ref_x.p, ref_x.q, ref_x.L, ref_x.U)
    print(f"v {v}: residual gpu-fp8 {r_gpu:.6e} oracle-fp8 {r_8:.6e} oracle-fp64 {r_x:.6e} "
          f"(fp8 form / fp64: {r_gpu / r_x:.4f})")
    assert r_gpu <= 1.05 * r_8 + 1e-7, (r_gpu, r_8)
    _pivots_vs_form(p, q, ref_8, k, ("fp8", m, n, k, v))
    assert f.info["passes"] == v
    return r_gpu, r_8, r_x


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_fixed_rank_fp8_square2000_type1(h, v):
    w = WORKLOADS["square2000_type1"]
    A = workload_matrix(w)
    _check_fp8_fixed_rank(h, A, 20, 10, v, seed=1000 * w.index + 3)


def test_fixed_rank_fp8_ragged(h):
    A = lowrank_plus_noise(1200, 901, spectrum("exp", 400, tau=20.0), 5, 6, 1e-6, 7)
    _check_fp8_fixed_rank(h, A, 33, 7, 4, seed=9)


# ---------------------------------------------------------------- refinement of the last range pass
REFINE = 16


REFINE_TWO = 32


def _check_form(h, A, k, p_over, v, seed, prec, rnd, exact_last, gate_fp64):
    m, n = A.shape
    l = k + p_over
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=seed)
    f = h.fixed_rank(dev(A), k, p_over, v, Omega=dev(Om), prec=prec)
    A64, Om64 = A.astype(np.float64), Om.astype(np.float64)
    ref_r = O.powerlu(A64, k, Om64, v, pass_round=rnd, exact_last=exact_last,
                      exact_tail=2 if prec & REFINE_TWO else 0)
    ref_x = O.powerlu(A64, k, Om64, v)
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    r_gpu = O.relative_residual(A, p, q, L, U)
    r_r = O.relative_residual(A, ref_r.p, ref_r.q, ref_r.L, ref_r.U)
    r_x = O.relative_residual(A, ref_x.p, ref_x.q, ref_x.L, ref_x.U)
    print(f"prec {prec} v {v}: residual gpu {r_gpu:.6e} oracle-form {r_r:.6e} oracle-fp64 {r_x:.6e}")
    assert r_gpu <= 1.05 * r_r + 1e-7, (r_gpu, r_r)
    if gate_fp64:
        assert r_gpu <= 1.05 * r_x + 1e-7, (r_gpu, r_x)
    tag = (("bf16" if (prec & 15) == BF16 else "fp8") + ("+r" if prec & REFINE else "")
           + ("+r2" if prec & REFINE_TWO else ""))
    _pivots_vs_form(p, q, ref_r, k, (tag, m, n, k, v))
    assert f.info["passes"] == v


@pytest.mark.parametrize("v", [3, 4, 5])
@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_fixed_rank_refined_square2000_type1(h, v, fmt):
    """With the last range pass on the fp32 A both forms stay within 1.05x of
    the FP64 oracle's residual (the FP8 form without it does not)."""
    w = WORKLOADS["square2000_type1"]
    A = workload_matrix(w)
    prec, rnd = (BF16, LP.round_bf16) if fmt == "bf16" else (FP8, LP.round_mx_e4m3)
    _check_form(h, A, 20, 10, v, 1000 * w.index + 3, prec | REFINE, rnd, True, True)


@pytest.mark.parametrize("v", [4, 5, 6])
@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_fixed_rank_refined_two_square2000_type1(h, v, fmt):
    """The last two range passes on the fp32 A (one exact power step on the
    rounded basis): against the rounding-matched oracle and within 1.05x of
    the FP64 oracle's residual."""
    w = WORKLOADS["square2000_type1"]
    A = workload_matrix(w)
    prec, rnd = (BF16, LP.round_bf16) if fmt == "bf16" else (FP8, LP.round_mx_e4m3)
    _check_form(h, A, 20, 10, v, 1000 * w.index + 3, prec | REFINE_TWO, rnd, False, True)


@pytest.mark.parametrize("t,eps,l,b", [(2, 1e-4, 120, 10), (2, 1e-3, 120, 10), (1, 1e-3, 500, 10)])
@pytest.mark.parametrize("fmt", ["bf16", "fp8"])
def test_fixed_precision_refined_paper_types(h, t, eps, l, b, fmt):
    n = 1000
    A = paper_type(t, n, seed=300 + t).astype(np.float32)
    Om = gaussian_omega(n, l, seed=400 + t)
    prec, rnd = (BF16, LP.round_bf16) if fmt == "bf16" else (FP8, LP.round_mx_e4m3)
    f = h.fixed_precision(dev(A), eps, b, l=l, v=4, column_exact=True, Omega=dev(Om),
                          prec=prec | REFINE)
    ref = O.powerlu_fp(A.astype(np.float64), eps, b, Om.astype(np.float64), 4, True,
                       pass_round=rnd, exact_last=True)
    ref_x = O.powerlu_fp(A.astype(np.float64), eps, b, Om.astype(np.float64), 4, True)
    acc = eps * eps * ref.normA2
    delta = DELTA_FORM[fmt] * ref.normA2
    k = f.rank
    print(f"{fmt}+refine type {t} eps {eps}: k_gpu {k} k_oracle_form {ref.rank} k_fp64 {ref_x.rank} "
          f"indicator diff/nA2 {abs(f.info['E_final'] - ref.E[k - 1]) / ref.normA2:.2e}")
    assert abs(f.info["E_final"] - ref.E[k - 1]) <= delta
    E = ref.E
    assert E[k - 1] <= acc + delta and (k < 2 or E[k - 2] >= acc - delta), (k, ref.rank)
    _reached_consistent(f, ref, k, acc, delta)
    if f.info["tol_reached"]:
        r = O.relative_residual(A, host(f.p), host(f.q), host(f.L), host(f.U))
        assert r * r <= eps * eps + 2 * delta / ref.normA2


# ---------------------------------------------------------------- rounded copies kept (A unchanged)
A_UNCHANGED = 64


@pytest.mark.parametrize("fmt", [BF16, FP8])
def test_rounded_copies_reused_when_a_is_unchanged(h, fmt):
    """PLU_PREC_A_UNCHANGED reuses the handle's rounded copies of A: the same
    factors as a call that rounds A again, for fixed rank, fixed precision and
    single passes; a call in another form or shape in between drops the
    copies (the flag then rounds A again), so a changed A is never served
    stale copies after such a call."""
    A1 = lowrank_plus_noise(1500, 1200, spectrum("exp", 200, tau=15.0), 31, 32, 1e-6, 33)
    A2 = lowrank_plus_noise(1500, 1200, spectrum("exp", 200, tau=9.0), 34, 35, 1e-6, 36)
    Ad = dev(A1)
    ref = h.fixed_rank(Ad, 20, 10, 4, seed=3, prec=fmt | REFINE)
    f = h.fixed_rank(Ad, 20, 10, 4, seed=3, prec=fmt | REFINE | A_UNCHANGED)
    for a, b in ((f.p, ref.p), (f.q, ref.q), (f.L, ref.L), (f.U, ref.U)):
        assert np.array_equal(host(a), host(b))
    g = h.fixed_precision(Ad, 1e-3, 10, l=100, v=4, seed=4, prec=fmt | A_UNCHANGED)
    g0 = h.fixed_precision(Ad, 1e-3, 10, l=100, v=4, seed=4, prec=fmt)
    assert g.rank == g0.rank
    for a, b in ((g.p, g0.p), (g.q, g0.q), (g.L, g0.L), (g.U, g0.U)):
        assert np.array_equal(host(a), host(b))
    X = dev(np.random.default_rng(5).standard_normal((1200, 40)).astype(np.float32))
    o1 = host(h.pass_(Ad, X, prec=fmt))
    o2 = host(h.pass_(Ad, X, prec=fmt | A_UNCHANGED))
    assert np.array_equal(o1, o2)
    # an fp32 call lays the workspace out differently: the copies are gone,
    # so the flag after it rounds the new contents of A
    h.fixed_rank(Ad, 20, 10, 4, seed=3)
    Ad.copy_(dev(A2))
    f2 = h.fixed_rank(Ad, 20, 10, 4, seed=3, prec=fmt | REFINE | A_UNCHANGED)
    r2 = h.fixed_rank(dev(A2), 20, 10, 4, seed=3, prec=fmt | REFINE)
    for a, b in ((f2.p, r2.p), (f2.L, r2.L), (f2.U, r2.U)):
        assert np.array_equal(host(a), host(b))
