"""CPU checks of the crafted pivot-tie inputs (synth.crafted_tie_matrix) that
the GPU tie-break test runs: on each case every one of the c steps of partial
pivoting meets an exact tie in the oracle's GETRF, and a float32 elimination
of the same input -- dividing by the pivot or multiplying by its float32
reciprocal -- reproduces the float64 oracle bit for bit, so float32
arithmetic decides nothing on these inputs and any correct float32 GETRF must
return the oracle's pivot order, ties included (LAPACK's first-maximum rule,
the paper's lu(.) of Sec. 2)."""

import numpy as np
import pytest

from oracle import powerlu as O
from synth import crafted_tie_matrix

TIE_CASES = [(700, 40, 0), (1537, 128, 0), (5000, 110, 1)]


def _elim32(X, reciprocal):
    """Unblocked partial-pivoting elimination in float32 (first maximum)."""
    X = X.astype(np.float32)
    M, c = X.shape
    perm = np.arange(M)
    for j in range(c):
        r = j + int(np.argmax(np.abs(X[j:, j])))
        X[[j, r]] = X[[r, j]]
        perm[[j, r]] = perm[[r, j]]
        piv = X[j, j]
        if piv != 0:
            if reciprocal:
                X[j + 1:, j] *= np.float32(1.0) / piv
            else:
                X[j + 1:, j] /= piv
            X[j + 1:, j + 1:] -= np.outer(X[j + 1:, j], X[j, j + 1:])
    return X, perm


@pytest.mark.parametrize("M,c,seed", TIE_CASES)
def test_crafted_ties_are_exact_in_float32(M, c, seed):
    X = crafted_tie_matrix(M, c, seed)
    assert np.array_equal(X.astype(np.float32).astype(np.float64), X)
    ref = O.getrf(X)
    assert int(np.sum(np.asarray(ref.gaps[:c]) == 0.0)) == c       # a tie at every step
    assert ref.zero_step == -1
    for reciprocal in (False, True):
        F, perm = _elim32(X, reciprocal)
        assert np.array_equal(perm, ref.perm)
        assert np.array_equal(np.triu(F[:c]).astype(np.float64), ref.U)
        L = np.tril(F, -1)[:, :c].astype(np.float64)
        L[np.arange(c), np.arange(c)] = 1.0
        assert np.array_equal(L, ref.L)
