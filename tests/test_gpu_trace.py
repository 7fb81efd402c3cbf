"""Pivot trace (plu_set_pivot_trace / plu_pivot_trace) against the oracle.

The trace of a fixed-rank call holds, in order, the LU reorthogonalizations
of Alg. 7 (l steps each) and the two final LU steps of Alg. 5 (k steps each).
Each segment's pivot rows are compared with the oracle's under the gap rule
of the end-to-end tests (bit-exact up to the first step whose oracle gap is
below tau); once a segment diverges the later segments see different inputs
and are only checked for validity.
"""

import numpy as np
import pytest

import paper_2002_07138_amd as plu
from tests.gpu_common import have_gpu, handle, dev, pivot_prefix_ok, assert_pivots
from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, spectrum

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

TAU = 1e-4


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.set_pivot_trace(0)
    hh.close()


def _oracle_segments(A64, Om, k, v):
    rec = O.RangeRecord()
    O.range_basis(A64, Om, v, rec)
    ref = O.powerlu(A64, k, Om, v)
    segs = [(lu.perm, lu.gaps, lu.L.shape[1], lu.L.shape[0]) for lu in rec.lu_steps]
    segs.append((ref.lu1.perm, ref.lu1.gaps, k, ref.lu1.L.shape[0]))
    segs.append((ref.lu2.perm, ref.lu2.gaps, k, ref.lu2.L.shape[0]))
    return segs


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_pivot_trace_of_fixed_rank(h, v):
    m, n, k, p_over = 1500, 1100, 20, 10
    l = k + p_over
    A = lowrank_plus_noise(m, n, spectrum("exp", 300, tau=15.0), 71, 72, 1e-6, 73)
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=80 + v)
    h.set_pivot_trace(100000)
    h.fixed_rank(dev(A), k, p_over, v, Omega=dev(Om))
    piv, gaps = h.pivot_trace()
    segs = _oracle_segments(A.astype(np.float64), Om.astype(np.float64), k, v)
    assert len(piv) == sum(c for _, _, c, _ in segs)
    at, diverged = 0, False
    for perm, ref_gaps, c, rows in segs:
        pg, gg = piv[at:at + c], gaps[at:at + c]
        at += c
        assert len(set(pg.tolist())) == c and pg.min() >= 0 and pg.max() < rows
        assert np.all((gg >= 0) & (gg <= 1))
        if diverged:
            continue
        ok, stop = pivot_prefix_ok(pg, perm[:c], ref_gaps, TAU)
        assert ok, f"pivots differ before step {stop}"
        assert np.max(np.abs(gg[:stop] - ref_gaps[:stop]), initial=0.0) <= 1e-3
        diverged = stop < c


def test_pivot_trace_of_getrf_and_limits(h):
    import torch
    rng = np.random.default_rng(5)
    X = rng.standard_normal((700, 90)).astype(np.float32)
    h.set_pivot_trace(1000)
    h.getrf(dev(X))
    piv, gaps = h.pivot_trace()
    ref = O.getrf(X.astype(np.float64))
    assert len(piv) == 90
    assert_pivots(piv, ref.perm[:90], ref.gaps, TAU)      # every oracle gap >= 9e-4 here
    # too small a capacity is reported, not truncated silently
    h.set_pivot_trace(50)
    h.getrf(dev(X))
    with pytest.raises(plu.PowerLUError) as ei:
        h.pivot_trace()
    assert ei.value.code == plu.PLU_ERR_OOM
    # off: nothing recorded
    h.set_pivot_trace(0)
    h.getrf(dev(X))
    piv, gaps = h.pivot_trace()
    assert len(piv) == 0
    torch.cuda.synchronize()
