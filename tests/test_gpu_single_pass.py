"""Single-pass randomized LU (Alg. 10) on the GPU against the FP64 oracle,
through the C ABI, in both storage orders of A (one pass over a column-major
A, two over a row-major one).

Alg. 10 multiplies by the pseudo-inverse of G^T, so in float32 its
reconstruction carries an error of about cond(G) u32 (u32 = 2^-24), which
PowerLU's QR-based path does not; and H = A G has singular values falling
like sigma_i^2, so H's late pivot columns sink into float32 rounding once
cond(G)^2 u32 nears 1.  The gates account for both:
  * p and q bit-exact up to the first step whose oracle gap is below
    tau = 1e-4 or below the float32 noise of that step's candidates,
    16 k u32 |u_11| / |u_jj| (the Schur complement entries carry an absolute
    error of about k u32 times the largest entry of the factored matrix), or
    whose oracle pivot is below 1e-4 of the first one;
  * relative residual <= 1.05 x the oracle's + 8 cond(G) u32;
  * where the pivots agree, L and U within 1e-3 + 32 k cond(G) u32 of the
    oracle's (U comes from the factorization of pinv(G^T) U1^T);
  * U unit upper trapezoidal with |u| <= 1;
  * a matrix of rank k is recovered to 8 cond(G) u32;
  * the approximation is PowerLU's at v = 2 without oversampling on the same
    Omega (residuals within 1e-3 relative plus the cond(G) term).
The test spectra keep cond(G) moderate (sigma_k / sigma_1 >= e^-4).
"""

import numpy as np
import pytest

from tests.gpu_common import torch, have_gpu, handle, dev, host, assert_pivots
from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, spectrum, workload_matrix, WORKLOADS

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

TAU = 1e-4
U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


def col_major(A):
    m, n = A.shape
    buf = torch.from_numpy(np.ascontiguousarray(A.T)).to("cuda")
    return buf.t()


# Row-pivot steps compared on the inputs whose oracle gap sequence reaches a
# cut step (pivot below 1e-4 of the first, or a gap within the float32 noise
# of its step) before step k: (m, n, k) -> steps.
SP_ROW_STEPS = {(901, 1300, 64): 46, (3000, 2500, 100): 77, (700, 650, 128): 105,
                (4000, 4000, 100): 86}


def _check(h, A, k, seed, col):
    m, n = A.shape
    Om = gaussian_omega(m, k, seed=seed)
    Ad = col_major(A) if col else dev(A)
    f = h.single_pass(Ad, k, Omega=dev(Om))
    ref = O.single_pass_lu(A.astype(np.float64), k, Om.astype(np.float64))
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    assert sorted(p.tolist()) == list(range(m)) and sorted(q.tolist()) == list(range(n))
    r_gpu = O.relative_residual(A, p, q, L, U)
    r_ref = O.relative_residual(A, ref.p, ref.q, ref.L, ref.U)
    cond = float(np.linalg.cond(ref.G))
    slack = 8 * cond * U32
    print(f"{m}x{n} k {k} col {col}: cond(G) {cond:.3g} residual gpu {r_gpu:.4g} oracle {r_ref:.4g}")
    assert r_gpu <= 1.05 * r_ref + slack, (r_gpu, r_ref, slack)

    def gaps_cut(f):
        d = np.abs(np.diag(f.U))
        g = np.array(f.gaps, dtype=np.float64)
        g[d < 1e-4 * d[0]] = 0.0        # pivots sunk toward float32 rounding
        noise = 16 * k * U32 * d[0] / np.maximum(d, 1e-300)
        g[g < noise] = 0.0              # gap within the float32 noise of the step
        return g

    # steps whose oracle gap is cut above are compared only up to the first
    # of them; the column order is compared when the row order agrees in full
    # (B^T depends on all of U1)
    sp = assert_pivots(p[:k], ref.p[:k], gaps_cut(ref.lu1), TAU, SP_ROW_STEPS.get((m, n, k)),
                       "row pivots")
    if sp == k:
        sq = assert_pivots(q[:k], ref.q[:k], gaps_cut(ref.lu2), TAU, None, "column pivots")
        if sq == k:
            tol = 1e-3 + 32 * k * cond * U32
            assert np.max(np.abs(L - ref.L)) <= tol * np.max(np.abs(ref.L))
            assert np.max(np.abs(U - ref.U)) <= tol
    assert np.allclose(np.diag(U[:, :k]), 1.0) and np.all(np.tril(U[:, :k], -1) == 0.0)
    assert np.max(np.abs(U)) <= 1.0 + 1e-6
    return f, r_gpu, Om, slack


@pytest.mark.parametrize("col", [False, True])
@pytest.mark.parametrize("m,n,k", [(1200, 900, 20), (901, 1300, 64), (3000, 2500, 100),
                                   (700, 650, 128)])
def test_single_pass_against_oracle(h, m, n, k, col):
    A = lowrank_plus_noise(m, n, spectrum("exp", min(m, n) // 2, tau=k / 4.0), m, n, 1e-6, 3)
    _check(h, A, k, seed=m + n + k, col=col)


@pytest.mark.parametrize("col", [False, True])
def test_single_pass_exact_rank(h, col):
    rng = np.random.default_rng(4)
    A = (rng.standard_normal((800, 24)) @ rng.standard_normal((24, 700))).astype(np.float32)
    f, r, _, slack = _check(h, A, 24, seed=9, col=col)
    assert r < slack


@pytest.mark.parametrize("col", [False, True])
def test_single_pass_equals_powerlu_v2(h, col):
    A = lowrank_plus_noise(2000, 1800, spectrum("exp", 600, tau=30.0), 5, 6, 1e-4, 7)
    f, r_sp, Om, slack = _check(h, A, 50, seed=11, col=col)
    g = h.fixed_rank(dev(A), 50, 0, 2, Omega=dev(Om))
    r_pl = O.relative_residual(A, host(g.p), host(g.q), host(g.L), host(g.U))
    assert abs(r_sp - r_pl) <= 1e-3 * r_pl + slack


def test_single_pass_workload_reduced(h):
    """The 20000^2 workload's recipe at 4000 x 4000 (same spectrum and seeds),
    k = 100, column-major."""
    w = WORKLOADS["square20000_exp40"]
    A = workload_matrix(w, 4000, 4000)
    _check(h, A, 100, seed=1000 * w.index + 7, col=True)
