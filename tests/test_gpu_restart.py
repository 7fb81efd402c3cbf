"""PowerLU_FP with restart rounds (max_rounds > 1) on the GPU against the
FP64 oracle's restart (reading R15 of the Remark after Alg. 8), through the
C ABI.

Round 0 takes the caller's Omega; round r >= 1 draws its Gaussian matrix on
the device from seed + r, which the oracle regenerates with its own Philox
(the draws agree to about 2e-6 relative).  Gates, as for the single-round
path with several orthonormal blocks:
  * |E_gpu - E_oracle(k)| <= delta and the GPU rank lies where the oracle's
    indicator is within delta of eps^2 ||A||^2 (delta = 4e-7 ||A||^2: the
    blocks of different rounds are orthogonal to about u32 sqrt(l));
  * residual^2 <= eps^2 + 2 delta / ||A||^2;
  * max_rounds = 1 is the single-round call (bit-identical).
"""

import numpy as np
import pytest

from tests.gpu_common import torch, have_gpu, handle, dev, host
from oracle import philox as PH
from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, paper_type, spectrum

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

DELTA = 4e-7


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


def _band_ok(E, k, acc, delta, step):
    if k < step or k > len(E):
        return False
    return E[k - 1] <= acc + delta and (k - step < 1 or E[k - step - 1] >= acc - delta)


def _check(h, A, eps, b, l, v, rounds, seed, column_exact=True):
    m, n = A.shape
    rows = m if v % 2 == 0 else n
    Om = gaussian_omega(rows, l, seed=seed)
    f = h.fixed_precision(dev(A), eps, b, l=l, v=v, column_exact=column_exact, Omega=dev(Om),
                          seed=seed, max_rounds=rounds)
    extra = [PH.gaussian(rows, l, seed + r).astype(np.float64) for r in range(1, rounds)]
    ref = O.powerlu_fp(A.astype(np.float64), eps, b, Om.astype(np.float64), v, column_exact,
                       restart_omegas=extra)
    acc = eps * eps * ref.normA2
    delta = DELTA * ref.normA2
    k = f.rank
    print(f"{m}x{n} eps {eps} l {l} rounds {rounds}: k_gpu {k} k_oracle {ref.rank} "
          f"dE/nA2 {abs(f.info['E_final'] - ref.E[k - 1]) / ref.normA2:.2e}")
    assert ref.tol_reached and f.info["tol_reached"] == 1
    assert abs(f.info["E_final"] - ref.E[k - 1]) <= delta
    assert _band_ok(ref.E, k, acc, delta, 1 if column_exact else b), (k, ref.rank)
    r = O.relative_residual(A, host(f.p), host(f.q), host(f.L), host(f.U))
    assert r * r <= eps * eps + 2 * delta / ref.normA2
    return f, ref


@pytest.mark.parametrize("column_exact", [True, False])
@pytest.mark.parametrize("v", [3, 4])
def test_restart_reaches_tolerance(h, v, column_exact):
    A = lowrank_plus_noise(640, 560, spectrum("exp", 300, tau=18.0), 11, 12, 1e-7, 13)
    f, ref = _check(h, A, 1e-3, 8, 40, v, 4, seed=100 + v, column_exact=column_exact)
    assert f.rank > 40                                   # one round was not enough


def test_restart_paper_type2(h):
    """Matrix Type 2 (Sec. 6.2) at n = 1000: l = 60 per round, eps = 1e-4."""
    A = paper_type(2, 1000, seed=302).astype(np.float32)
    f, ref = _check(h, A, 1e-4, 10, 60, 4, 3, seed=7)
    assert f.rank > 60


def test_one_round_is_the_single_round_call(h):
    A = lowrank_plus_noise(500, 420, spectrum("exp", 200, tau=15.0), 21, 22, 1e-7, 23)
    Om = dev(gaussian_omega(500, 40, seed=3))
    f1 = h.fixed_precision(dev(A), 1e-3, 8, l=40, v=4, Omega=Om)
    f2 = h.fixed_precision(dev(A), 1e-3, 8, l=40, v=4, Omega=Om, max_rounds=1)
    assert f1.rank == f2.rank == 40 and f1.info["tol_reached"] == 0
    for a, b in ((f1.p, f2.p), (f1.q, f2.q), (f1.L, f2.L), (f1.U, f2.U)):
        assert torch.equal(a, b)


def test_rounds_run_out(h):
    """Not enough rounds: the l * max_rounds factorization, TOL_NOT_REACHED."""
    A = np.random.default_rng(4).standard_normal((400, 300)).astype(np.float32)
    f = h.fixed_precision(dev(A), 1e-6, 8, l=32, v=4, seed=9, max_rounds=3)
    assert f.rank == 96 and f.info["tol_reached"] == 0
