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


def assert_pivots(gpu_perm, ref_perm, gaps, tau, expect_steps=None, what="pivots"):
    """Bit-exact pivot parity.  Compares the first steps of the GPU's pivot
    order with the oracle's up to the first step whose oracle gap is below
    tau, and asserts how many steps that is: all of them (expect_steps None:
    the input was built with separated pivots, so the whole sequence is
    compared), or exactly expect_steps (an input whose oracle gap sequence is
    known to fall below tau at that step).  Returns the compared length."""
    c = len(gaps)
    ok, stop = pivot_prefix_ok(np.asarray(gpu_perm)[:c], np.asarray(ref_perm)[:c], gaps, tau)
    assert ok, f"{what} differ from the oracle's before step {stop}"
    want = c if expect_steps is None else expect_steps
    assert stop == want, (f"{what}: the oracle's gap falls below tau = {tau:g} at step {stop} "
                          f"(expected {want} of {c} steps compared)")
    return stop


def assert_factors_close(L, U, ref_L, ref_U, l_tol=1e-4, u_tol=1e-3):
    """Factor parity once both pivot orders agree in full: L within l_tol of
    max|L_oracle| and U within u_tol (|u| <= 1), entry by entry.  A float32
    run of the same algorithm through LAPACK's float32 routines already
    deviates from the float64 oracle by up to ~8e-6 max|L| and ~1.3e-4 on U
    on the pipeline inputs, so these gates leave about 10x of room; an
    elementwise relative gate of 1e-4 on entries above 1e-3 max is below
    what float32 arithmetic reaches (the same float32 run misses it by up to
    30x on U)."""
    dl = float(np.max(np.abs(L - ref_L)))
    du = float(np.max(np.abs(U - ref_U)))
    assert dl <= l_tol * float(np.max(np.abs(ref_L))), ("L", dl, float(np.max(np.abs(ref_L))))
    assert du <= u_tol, ("U", du)
    return dl / float(np.max(np.abs(ref_L))), du
