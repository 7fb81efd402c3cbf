"""The benchmark's own workload at full size: A = 20000 x 20000 float32,
rank-500 signal with sigma_i = exp(-i/40) plus 1e-4 N(0,1)/sqrt(n) noise,
k = 100, l = 110 -- the shapes, tuned plans and kernels the benchmark times.

  * one pass over A in each direction, against float64 products of sampled
    rows (A X) and sampled columns (A^T Y) computed one by one on the host,
    within the float32 accumulation bound (R + 1) u32 (|A| |X|), and bitwise
    repeatable;
  * PowerLU at v = 3 on the same Omega as the FP64 oracle at full size: the
    pivot prefixes up to the oracle's first gap below tau = 1e-4 are equal,
    and the relative residual is within 1.05x + 64 u32 of the oracle's.
"""

import numpy as np
import pytest

from tests.gpu_common import torch, have_gpu, handle, dev, host, assert_pivots, assert_factors_close
from oracle import powerlu as O
from synth import WORKLOADS, gaussian_omega, workload_matrix

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

U32 = 2.0 ** -24
TAU = 1e-4
K, P_OVER = 100, 10


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


@pytest.fixture(scope="module")
def workload():
    w = WORKLOADS["square20000_exp40"]
    A = workload_matrix(w)
    assert A.shape == (20000, 20000) and A.dtype == np.float32
    return A


def test_full_size_passes_on_sampled_outputs(h, workload):
    A = workload
    m, n = A.shape
    l = K + P_OVER
    Ad = dev(A)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((n, l)).astype(np.float32)
    Y = rng.standard_normal((m, l)).astype(np.float32)
    rows = np.sort(rng.choice(m, 48, replace=False))
    cols = np.sort(rng.choice(n, 48, replace=False))
    Xd, Yd = dev(X), dev(Y)
    for trans, In, idx in ((False, X, rows), (True, Y, cols)):
        out = h.pass_(Ad, Yd if trans else Xd, trans=trans)
        again = h.pass_(Ad, Yd if trans else Xd, trans=trans)
        assert torch.equal(out, again), "not repeatable"
        got = host(out)[idx].astype(np.float64)
        sub = (A[:, idx].T if trans else A[idx]).astype(np.float64)   # rows of op(A)
        In64 = In.astype(np.float64)
        ref = sub @ In64
        bound = (In.shape[0] + 1) * U32 * (np.abs(sub) @ np.abs(In64))
        err = np.abs(got - ref)
        print(f"trans {trans}: max err {err.max():.3e}, max err / (|A||X|) "
              f"{np.max(err / (np.abs(sub) @ np.abs(In64))):.3e}")
        assert np.all(err <= bound)
    del Ad
    torch.cuda.empty_cache()


def test_full_size_fixed_rank_against_oracle(h, workload):
    A = workload
    m, n = A.shape
    v = 3
    Om = gaussian_omega(n, K + P_OVER, seed=77)      # v odd: Omega is n x l
    Ad = dev(A)
    f = h.fixed_rank(Ad, K, P_OVER, v, Omega=dev(Om))
    p, q, L, U = host(f.p), host(f.q), host(f.L), host(f.U)
    del Ad
    torch.cuda.empty_cache()
    A64 = A.astype(np.float64)
    ref = O.powerlu(A64, K, Om.astype(np.float64), v)
    assert sorted(p.tolist()) == list(range(m)) and sorted(q.tolist()) == list(range(n))
    # every oracle gap of both final LUs is above tau on this input (the
    # smallest are 1.4e-4 and 2.8e-4): both orders are compared in full
    stop_p = assert_pivots(p[:K], ref.p[:K], ref.lu1.gaps, TAU, None, "row pivots")
    assert_pivots(q[:K], ref.q[:K], ref.lu2.gaps, TAU, None, "column pivots")
    assert_factors_close(L, U, ref.L, ref.U)
    r_gpu = O.relative_residual(A64, p, q, L, U)
    r_ref = O.relative_residual(A64, ref.p, ref.q, ref.L, ref.U)
    print(f"20000^2 v {v}: residual gpu {r_gpu:.8g} oracle {r_ref:.8g}; pivots equal to "
          f"step {stop_p}")
    assert r_gpu <= 1.05 * r_ref + 64 * U32
