"""Shared helpers for the GPU tests (imported by test modules only)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def have_gpu():
    return torch.cuda.is_available()


def handle():
    import paper_2002_07138_amd as plu
    return plu.Handle(0)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def equal_up_to_signs(V, Q, tol):
    worst = 0.0
    for j in range(V.shape[1]):
        s = np.sign(V[:, j] @ Q[:, j]) or 1.0
        worst = max(worst, float(np.max(np.abs(V[:, j] - s * Q[:, j]))))
    return worst <= tol, worst


def pivot_prefix_ok(gpu_perm, ref_perm, gaps, tau):
    """Bit-exact pivot agreement up to the first step whose oracle gap is
    below tau (the comparison is only meaningful where the pivot choice is
    not decided by rounding)."""
    c = len(gaps)
    stop = c
    for j in range(c):
        if gaps[j] < tau:
            stop = j
            break
    return np.array_equal(np.asarray(gpu_perm)[:stop], np.asarray(ref_perm)[:stop]), stop
