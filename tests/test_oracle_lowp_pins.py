"""Pins for the reduced-precision operand rounding of the oracle (the
precision form of the passes) and for how the precision form applies it.
CPU only."""

import numpy as np
import pytest
import torch

from oracle import lowp as LP
from oracle import powerlu as O
from synth import gaussian_omega, lowrank_plus_noise, spectrum


def _specials32():
    vals = [0.0, -0.0, 1.0, -1.0, 1.0 + 2**-8, 1.0 + 3 * 2**-8, 1.0 + 2**-9, 65504.0,
            3.3895313892515355e38, 1e-40, -1e-42, 2**-126, 2**-133, np.inf, -np.inf,
            1.00390625, 1.01171875, 0.1, 1 / 3]
    return np.array(vals, dtype=np.float32)


# ---------------------------------------------------------------- bfloat16
def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.standard_normal(200000).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 200000).astype(np.float32),
        # exact ties: the lower 16 bits are 0x8000
        (rng.integers(0, 2**31, 5000, dtype=np.uint64).astype(np.uint32) & np.uint32(0x7FFF0000) | np.uint32(0x8000)).view(np.float32),
        _specials32(),
    ])
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(LP.bf16_bits(x), ref)
    assert np.array_equal(LP.round_bf16(x), torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy())


def test_bf16_nonfinite():
    x = np.array([np.inf, -np.inf, np.nan], dtype=np.float32)
    r = LP.round_bf16(x)
    assert r[0] == np.inf and r[1] == -np.inf and np.isnan(r[2])


# ---------------------------------------------------------------- E4M3
def test_e4m3_grid_matches_torch():
    rng = np.random.default_rng(2)
    y = np.concatenate([
        rng.uniform(-448, 448, 100000),
        rng.standard_normal(100000) * 2.0 ** rng.integers(-12, 8, 100000),
        # every grid point and every midpoint between neighbours (ties to even)
        np.arange(256, dtype=np.float64),
    ])
    grid = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    grid = np.unique(np.abs(grid[np.isfinite(grid)]))
    mids = (grid[1:] + grid[:-1]) / 2
    y = np.concatenate([y, grid, -grid, mids, -mids]).astype(np.float32).astype(np.float64)
    y = y[np.abs(y) <= 448]
    q = LP.e4m3_round(y)
    ref = torch.from_numpy(y.astype(np.float32)).to(torch.float8_e4m3fn)
    assert np.array_equal(q, ref.to(torch.float64).numpy())
    # codes of the rounded values are the format's bit patterns
    codes = LP.e4m3_bits(q)
    assert np.array_equal(codes[q != 0], ref.view(torch.uint8).numpy()[q != 0])


def test_mx_exponent_is_minimal_and_error_is_half_spacing():
    rng = np.random.default_rng(3)
    X = (rng.standard_normal((70, 100)) * 10.0 ** rng.integers(-20, 20, (70, 1))).astype(np.float32)
    X[5, :] = 0.0
    X[6, 32:64] = 448.0 * 2.0**-3          # amax exactly on the boundary
    for axis in (0, 1):
        e = LP.mx_exponents(X, axis)
        Xm = np.moveaxis(X.astype(np.float64), axis, -1)
        K = Xm.shape[-1]
        for blk in range(e.shape[-1]):
            sl = Xm[..., blk * 32:min(K, blk * 32 + 32)]
            amax = np.max(np.abs(sl), axis=-1)
            eb = e[..., blk]
            nz = amax > 0
            assert np.all(amax[nz] / 2.0 ** eb[nz] <= 448.0)
            assert np.all((amax[nz] / 2.0 ** (eb[nz] - 1) > 448.0) | (eb[nz] == -127))
            assert np.all(eb[~nz] == -127)
        Q = LP.round_mx_e4m3(X, axis)
        # round to nearest: error <= half the spacing at each value, spacing
        # <= 2^(e - 3) * 2^floor(log2(448 / 256)) relative to the block scale
        scale = np.moveaxis(np.exp2(np.repeat(e, 32, axis=-1)[..., :K].astype(np.float64)), -1, axis)
        y = X / scale
        sp = np.exp2(np.maximum(np.floor(np.log2(np.maximum(np.abs(y), 1e-300))), -6) - 3)
        assert np.all(np.abs(Q - X) <= 0.5 * sp * scale * (1 + 1e-12))
    assert LP.mx_exponents(X, 1)[6, 1] == -3


# ---------------------------------------------------------------- precision form of Alg. 7
def test_precision_form_rounds_exactly_the_range_passes():
    """The v - 1 products of Alg. 7 take rounded operands; the final product
    with A (assembly) does not.  A recording rounding shows which operands
    are rounded and along which axis."""
    A = lowrank_plus_noise(120, 90, spectrum("exp", 20, tau=4.0), 1, 2, 1e-6, 3, dtype=np.float64)
    for v in (2, 3, 4, 5):
        calls = []

        def rec(X, axis):
            calls.append((X.shape, axis))
            return np.asarray(X, dtype=np.float64)

        Om = gaussian_omega(120 if v % 2 == 0 else 90, 12, seed=v).astype(np.float64)
        f = O.powerlu(A, 8, Om, v, pass_round=rec)
        f0 = O.powerlu(A, 8, Om, v)
        # identity rounding reproduces the exact algorithm
        assert np.array_equal(f.L, f0.L) and np.array_equal(f.U, f0.U)
        assert len(calls) == 2 * (v - 1)
        a_axes = [ax for (shape, ax) in calls[0::2]]
        # even v starts with A^T (contraction over rows), then alternates
        start = 0 if v % 2 == 0 else 1
        assert a_axes == [(start + i) % 2 for i in range(v - 1)]
        assert all(shape == (120, 90) for (shape, ax) in calls[0::2])
        assert all(ax == 0 for (shape, ax) in calls[1::2])
        # with exact_last the last range product is not rounded
        calls.clear()
        O.powerlu(A, 8, Om, v, pass_round=rec, exact_last=True)
        assert len(calls) == 2 * (v - 2)
        assert [ax for (shape, ax) in calls[0::2]] == a_axes[:v - 2]
        # with exact_tail = 2 the last two are not (none of them when v <= 3)
        calls.clear()
        O.powerlu(A, 8, Om, v, pass_round=rec, exact_tail=2)
        assert len(calls) == 2 * max(v - 3, 0)
        assert [ax for (shape, ax) in calls[0::2]] == a_axes[:max(v - 3, 0)]
        # exact_last is exact_tail = 1
        calls.clear()
        O.powerlu(A, 8, Om, v, pass_round=rec, exact_tail=1)
        assert len(calls) == 2 * (v - 2)


@pytest.mark.parametrize("v", [2, 3, 4, 5])
def test_exact_tail_covering_every_pass_is_the_exact_algorithm(v):
    """With exact_tail >= v - 1 no range product is rounded: the factors are
    the exact algorithm's bit for bit, under a real (E4M3) rounding; with
    fewer exact passes they differ."""
    A = lowrank_plus_noise(140, 100, spectrum("exp", 30, tau=5.0), 4, 5, 1e-6, 6, dtype=np.float64)
    Om = gaussian_omega(140 if v % 2 == 0 else 100, 12, seed=30 + v).astype(np.float64)
    f0 = O.powerlu(A, 8, Om, v)
    f1 = O.powerlu(A, 8, Om, v, pass_round=LP.round_mx_e4m3, exact_tail=v - 1)
    assert np.array_equal(f0.L, f1.L) and np.array_equal(f0.U, f1.U)
    assert np.array_equal(f0.p, f1.p) and np.array_equal(f0.q, f1.q)
    if v >= 3:
        f2 = O.powerlu(A, 8, Om, v, pass_round=LP.round_mx_e4m3, exact_tail=v - 2)
        assert not np.array_equal(f0.L, f2.L)


@pytest.mark.parametrize("v", [2, 3, 4])
def test_precision_form_depends_on_A_and_Omega_only_through_their_rounding(v):
    """Perturbing A and Omega by less than half a bfloat16 ulp leaves the
    bfloat16 form's basis unchanged: every product sees the rounded copies."""
    m, n, l = 150, 110, 14
    rng = np.random.default_rng(7)
    # bf16-exact values: integers below 2^7 times powers of two
    B = (rng.integers(-100, 100, (m, n)) * 2.0 ** rng.integers(-4, 4, (m, 1))).astype(np.float64)
    Om = rng.integers(-50, 50, (m if v % 2 == 0 else n, l)).astype(np.float64)
    dA = rng.uniform(-1, 1, (m, n)) * np.abs(B) * 2.0**-10      # < half ulp of bf16
    dO = rng.uniform(-1, 1, Om.shape) * np.abs(Om) * 2.0**-10
    A1 = (B + dA).astype(np.float32).astype(np.float64)
    O1 = (Om + dO).astype(np.float32).astype(np.float64)
    assert np.array_equal(LP.round_bf16(A1), B) and np.array_equal(LP.round_bf16(O1), Om)
    V0 = O.range_basis(B, Om, v, pass_round=LP.round_bf16)
    V1 = O.range_basis(A1, O1, v, pass_round=LP.round_bf16)
    assert np.array_equal(V0, V1)
    # while the exact form does see the perturbation
    assert not np.array_equal(O.range_basis(B, Om, v), O.range_basis(A1, O1, v))
