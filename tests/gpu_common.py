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
    g, r = np.asarray(gpu_perm)[:c], np.asarray(ref_perm)[:c]
    ok, stop = pivot_prefix_ok(g, r, gaps, tau)
    if not ok:
        j = int(np.flatnonzero(g[:stop] != r[:stop])[0])
        raise AssertionError(f"{what} differ from the oracle's at step {j} (oracle gap there "
                             f"{gaps[j]:.3e}, tau {tau:g}, {stop} steps above tau)")
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


def column_deviation(Vg, Vr):
    """Per column j: max|Vg[:, j] - s Vr[:, j]| / max|Vr[:, j]| with s = +-1
    the sign that aligns the two (a thin-Q basis is unique up to signs)."""
    out = np.empty(Vr.shape[1])
    for j in range(Vr.shape[1]):
        s = np.sign(Vg[:, j] @ Vr[:, j]) or 1.0
        out[j] = np.max(np.abs(Vg[:, j] - s * Vr[:, j])) / np.max(np.abs(Vr[:, j]))
    return out


def assert_pivots_measured(gpu_perm, ref_perm, gaps, col_dev, margin=10.0, tau=1e-4,
                           min_steps=0, what="pivots"):
    """Pivot parity with a threshold from the measured deviation of the GPU's
    basis (the parity rule's tau = a multiple of the GPU's relative deviation
    from the oracle): step j is decided above rounding when the oracle's gap
    there exceeds max(tau, margin x the largest column deviation among the
    first j + 1 columns).  The orders must agree up to the first step that is
    not, and at least min_steps steps must be compared.  Returns that count."""
    c = len(gaps)
    thr = np.maximum(tau, margin * np.maximum.accumulate(np.asarray(col_dev)[:c]))
    below = np.flatnonzero(np.asarray(gaps[:c]) < thr)
    stop = int(below[0]) if len(below) else c
    g, r = np.asarray(gpu_perm)[:stop], np.asarray(ref_perm)[:stop]
    if not np.array_equal(g, r):
        j = int(np.flatnonzero(g != r)[0])
        raise AssertionError(f"{what} differ from the oracle's at step {j} (oracle gap "
                             f"{gaps[j]:.3e}, threshold {thr[j]:.3e})")
    assert stop >= min_steps, f"{what}: only {stop} steps decided above the measured deviation"
    return stop
