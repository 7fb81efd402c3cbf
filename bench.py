"""Benchmark: PowerLU on MI355X.

Workload (square20000_exp40): A = X diag(sigma) Y^T + 1e-4 N(0,1)/sqrt(n),
m = n = 20000, X, Y orthonormalized seeded Gaussian 20000 x 500,
sigma_i = exp(-i/40); k = 100, oversampling 10 (l = 110).  One step is the
whole fixed-rank path for every pass count v = 2, 3, 4, 5 (Alg. 5 with
Alg. 7): Gaussian draw, v passes over A, LU reorthogonalizations, thin QR,
the two final LU factorizations and the L/U assembly -- 14 passes over A.

Prints one JSON line (see the keys below).  GFLOP/s counts the algorithmic
work of the paper's cost model (C_mm = 2, LU m c^2 - c^3/3, QR 2 n c^2 -
2 c^3/3), not the extra work of the implementation.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
WORKLOAD = "square20000_exp40"
K_RANK, P_OVER = 100, 10
VS = (2, 3, 4, 5)


def flops_fixed_rank(m: int, n: int, k: int, l: int, v: int) -> float:
    """Algorithmic flops of PowerLU (Alg. 5 + Alg. 7), cost constants as in
    the paper's cost model with C_mm = 2, C_lu = 1 (m c^2 - c^3/3), C_qr = 2."""
    lu = lambda r, c: r * c * c - c ** 3 / 3.0
    qr = lambda r, c: 2.0 * r * c * c - 2.0 * c ** 3 / 3.0
    f = (v - 1) * 2.0 * m * n * l + 2.0 * m * n * k          # passes
    P = (v - 1) // 2
    # reorthogonalizations: v-2 LU + 1 QR (even v: first on n x l)
    n_lu_m = P                                  # lu(A V) on m x l
    n_lu_n = (v - 2) - P                        # lu(A^T V) on n x l
    f += n_lu_m * lu(m, l) + n_lu_n * lu(n, l) + qr(n, l)
    f += lu(m, k) + 2.0 * n * k * k + lu(n, k) + 2.0 * m * k * k   # Alg. 5 steps 4-7
    return f


def flops_fixed_precision(m: int, n: int, l: int, k: int, v: int) -> float:
    """Algorithmic flops of PowerLU_FP (Alg. 9 on Alg. 7): v passes with all
    l columns (the last is G = A V), the reorthogonalizations on l columns,
    the indicator (2 m l) and the assembly on the rank k."""
    lu = lambda r, c: r * c * c - c ** 3 / 3.0
    qr = lambda r, c: 2.0 * r * c * c - 2.0 * c ** 3 / 3.0
    f = v * 2.0 * m * n * l + 2.0 * m * l
    P = (v - 1) // 2
    f += P * lu(m, l) + ((v - 2) - P) * lu(n, l) + qr(n, l)
    if k > 0:
        f += lu(m, k) + 2.0 * n * k * k + lu(n, k) + 2.0 * m * k * k
    return f


FORMS = {"bf16": 1, "fp8_e4m3": 2, "bf16+refine_last": 1 | 16, "fp8_e4m3+refine_last": 2 | 16,
         "fp8_e4m3+refine_two": 2 | 32}
A_UNCHANGED = 64
FP64_INDICATOR = 128
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_FP8_MFMA_TFLOPS = 5000.0


def _event_times(fn, reps):
    """reps calls, each between two events on the current stream (no host
    synchronization between calls); per-call durations in ms."""
    import torch
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for e0, e1 in evs:
        e0.record()
        fn()
        e1.record()
    evs[-1][1].synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in evs]


def _stats(ts):
    import numpy as np
    a = np.asarray(ts, dtype=np.float64)
    return {"median": round(float(np.median(a)), 4), "p10": round(float(np.percentile(a, 10)), 4),
            "p90": round(float(np.percentile(a, 90)), 4), "n": int(a.size)}


def _sketch(rows, l, dev, gen=None, fill=True):
    """rows x l float32 with rows padded to a multiple of 4 floats (the
    layout of the library's own iterates and pass outputs)."""
    import torch
    lp = (l + 3) // 4 * 4
    t = (torch.randn((rows, lp), device=dev, generator=gen) if fill
         else torch.empty((rows, lp), device=dev))
    return t[:, :l]


def _pass_times(h, A, l, reps=10, prec=0):
    """Median time of one pass A X (N) and A^T X (T) with sketch width l."""
    import numpy as np
    import torch
    m, n = A.shape
    X_n = _sketch(n, l, A.device)
    X_m = _sketch(m, l, A.device)
    o_m = _sketch(m, l, A.device, fill=False)
    o_n = _sketch(n, l, A.device, fill=False)
    out = {}
    for name, X, o, tr in (("N", X_n, o_m, False), ("T", X_m, o_n, True)):
        h.pass_(A, X, trans=tr, out=o, prec=prec)                  # tuning / rounded copies
        torch.cuda.synchronize()
        keep = prec | (A_UNCHANGED if prec else 0)
        out[name] = float(np.median(_event_times(lambda: h.pass_(A, X, trans=tr, out=o, prec=keep),
                                                 reps)))
    return out


def _device_matrix(X, s, Y):
    """X diag(s) Y^T formed on the device in float32 from float64 factors."""
    import torch
    Xd = torch.from_numpy((X * s[None, :]).astype("float32")).cuda()
    Yd = torch.from_numpy(Y.astype("float32")).cuda()
    A = Xd @ Yd.t()
    del Xd, Yd
    torch.cuda.synchronize()
    return A


def square32768_section(h, reps=5, cpu=True):
    """The precision-form workload: A = X diag(i^-1.5) Y^T, 32768^2, rank 1000
    (X, Y the seeded Q factors; the product formed on the device in float32),
    k = 200, oversampling 20, v = 4.  Each form: call time (median, p10, p90
    of reps), GFLOP/s of the cost model, full-size residual; the rounded
    forms again with their copies of A kept (PLU_PREC_A_UNCHANGED).  Passes:
    the fp32 one against the FP32 MFMA peak, the rounded ones (copies kept:
    the pass alone) against HBM.  Error against the FP64 oracle: every form on
    the 4096^2 leading block (synth.workload_slice) with the same Gaussian
    matrix as the stored oracle residuals (tests/golden, written by a script
    that calls only the oracle)."""
    import numpy as np
    import torch
    from synth import WORKLOADS, gaussian_omega, workload_matrix_factors, workload_slice
    w = WORKLOADS["square32768_pow15"]
    k, p_over, v = 200, 20, 4
    l = k + p_over
    t0 = time.perf_counter()
    X, s, Y = workload_matrix_factors(w)
    A = _device_matrix(X, s, Y)
    del X, Y
    gen = time.perf_counter() - t0
    m, n = A.shape
    dev = A.device
    outs = (torch.empty(m, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty((m, k), device=dev), torch.empty((k, n), device=dev))
    flops = flops_fixed_rank(m, n, k, l, v)
    forms = {"fp32": 0, **{kk: vv for kk, vv in FORMS.items() if kk != "fp8_e4m3"}}
    res = {"workload": w.name, "m": m, "n": n, "k": k, "p_over": p_over, "v": v,
           "input_generation_s": round(gen, 2), "forms": {}}
    for name, prec in forms.items():
        f = h.fixed_rank(A, k, p_over, v, seed=31, prec=prec, out=outs)
        r = h.residual(A, f)
        ts = _event_times(lambda: h.fixed_rank(A, k, p_over, v, seed=31, prec=prec,
                                               sync_info=False, out=outs), reps)
        e = {"ms": _stats(ts), "gflops": round(flops / (np.median(ts) * 1e-3) / 1e9, 1),
             "residual_full_size": r}
        if prec:
            ts2 = _event_times(lambda: h.fixed_rank(A, k, p_over, v, seed=31,
                                                    prec=prec | A_UNCHANGED,
                                                    sync_info=False, out=outs), reps)
            e["ms_copies_kept"] = _stats(ts2)
            e["gflops_copies_kept"] = round(flops / (np.median(ts2) * 1e-3) / 1e9, 1)
        res["forms"][name] = e
    passes = {}
    fp32 = _pass_times(h, A, l)
    ms = 0.5 * (fp32["N"] + fp32["T"])
    passes["fp32"] = {"ms": fp32, "bound": "mfma", "achieved_tflops": round(2.0 * m * n * l / (ms * 1e-3) / 1e12, 2),
                      "frac": round(2.0 * m * n * l / (ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4)}
    for name, prec, bytes_a in (("bf16", 1, 2.0 * m * n), ("fp8_e4m3", 2, m * n * (1 + 1 / 32.0))):
        t = _pass_times(h, A, l, prec=prec)
        ms = 0.5 * (t["N"] + t["T"])
        passes[name] = {"ms": t, "bound": "hbm", "algorithmic_bytes": bytes_a,
                        "achieved_gbs": round(bytes_a / (ms * 1e-3) / 1e9, 1),
                        "frac": round(bytes_a / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    res["passes"] = passes
    del A
    torch.cuda.empty_cache()
    # error against the FP64 oracle on the leading 4096^2 block
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "square32768_slice4096_oracle.json")))
    S = torch.from_numpy(workload_slice(w, 4096, 4096)).to(dev)
    Om = torch.from_numpy(gaussian_omega(4096, l, seed=gold["omega_seed"])).to(dev)
    r64 = gold["residual"]["fp32"]
    sl = {}
    for name, prec in forms.items():
        f = h.fixed_rank(S, k, p_over, v, Omega=Om, prec=prec)
        r = h.residual(S, f)
        sl[name] = {"residual": r, "vs_fp64_oracle": round(r / r64, 5),
                    "form_oracle_vs_fp64_oracle": round(gold["residual"][name] / r64, 5)}
    res["slice4096_vs_fp64_oracle"] = sl
    if cpu:
        from oracle import powerlu as O
        S64 = S.cpu().numpy().astype(np.float64)
        Om64 = Om.cpu().numpy().astype(np.float64)
        t0 = time.perf_counter()
        O.powerlu(S64, k, Om64, v)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(flops_fixed_rank(4096, 4096, k, l, v) / dt / 1e9, 2),
                               "unit": "GFLOP/s", "cores": _oracle_threads(), "kind": "oracle",
                               "sample": f"one fixed-rank PowerLU (v={v}, k={k}, l={l}) of the "
                                         f"4096x4096 leading block in float64 NumPy, {dt:.2f} s"}
    del S
    torch.cuda.empty_cache()
    return res


def rect30000_section(h, reps=3, cpu=True):
    """The fixed-precision workload: A = X diag(exp(-i/50)) Y^T, 30000 x
    20000, rank 2000 (the product formed on the device in float32), eps =
    1e-3, b = 32, l = 1600, v = 4, both rank rules: call time (median, p10,
    p90), GFLOP/s of the cost model at the rank found, the rank and the
    residual; the l = 1600 pass against the FP32 MFMA peak.  CPU baseline: the
    oracle on the same recipe at 6000 x 4000 with l = 1024."""
    import numpy as np
    import torch
    from synth import WORKLOADS, gaussian_omega, workload_matrix, workload_matrix_factors
    w = WORKLOADS["rect30000x20000_exp50"]
    eps, b, l, v = 1e-3, 32, 1600, 4
    t0 = time.perf_counter()
    X, s, Y = workload_matrix_factors(w)
    A = _device_matrix(X, s, Y)
    del X, Y
    gen = time.perf_counter() - t0
    m, n = A.shape
    dev = A.device
    outs = (torch.empty(m, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.int32, device=dev),
            torch.empty((m, l), device=dev), torch.empty((l, n), device=dev),
            torch.zeros(1, dtype=torch.int32, device=dev))
    res = {"workload": w.name, "m": m, "n": n, "eps": eps, "b": b, "l": l, "v": v,
           "input_generation_s": round(gen, 2), "rules": {}}
    for name, col, prec in (("column", True, 0), ("block", False, 0),
                            ("column+fp64_indicator", True, FP64_INDICATOR)):
        f = h.fixed_precision(A, eps, b, l=l, v=v, column_exact=col, seed=41, prec=prec)
        r = h.residual(A, f)
        ts = _event_times(lambda: h.fixed_precision(A, eps, b, l=l, v=v, column_exact=col, seed=41,
                                                    prec=prec, sync_info=False, out=outs), reps)
        fl = flops_fixed_precision(m, n, l, f.rank, v)
        res["rules"][name] = {
            "rank": f.rank, "tol_reached": f.info["tol_reached"], "residual": r,
            "E_final_rel": f.info["E_final"] / f.info["normA2"],
            "ms": _stats(ts), "gflops": round(fl / (np.median(ts) * 1e-3) / 1e9, 1)}
        if prec:
            # its extra float64 work: G = A V (2 m n l) and the two Grams (l^2 (m + n))
            extra = 2.0 * m * n * l + 1.0 * l * l * (m + n)
            res["rules"][name]["fp64_extra_flops"] = extra
    t = _pass_times(h, A, l, reps=5)
    ms = 0.5 * (t["N"] + t["T"])
    res["pass"] = {"ms": t, "bound": "mfma",
                   "achieved_tflops": round(2.0 * m * n * l / (ms * 1e-3) / 1e12, 2),
                   "frac": round(2.0 * m * n * l / (ms * 1e-3) / 1e12 / PEAK_FP32_MFMA_TFLOPS, 4)}
    del A
    torch.cuda.empty_cache()
    if cpu:
        from oracle import powerlu as O
        Ar = workload_matrix(w, 6000, 4000).astype(np.float64)
        Om = gaussian_omega(6000, 1024, seed=1000 * w.index + 3).astype(np.float64)
        t0 = time.perf_counter()
        ref = O.powerlu_fp(Ar, eps, b, Om, v, True)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {
            "value": round(flops_fixed_precision(6000, 4000, 1024, ref.rank, v) / dt / 1e9, 2),
            "unit": "GFLOP/s", "cores": _oracle_threads(), "kind": "oracle",
            "sample": f"one PowerLU_FP (column rule, eps={eps}, b={b}, l=1024, v={v}, rank "
                      f"{ref.rank}) of the workload recipe at 6000x4000 in float64 NumPy, {dt:.2f} s"}
    return res


def _oracle_threads():
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        return max((i.get("num_threads", 0) for i in info), default=None) or os.cpu_count()
    except Exception:
        return os.cpu_count()


def single_pass_section(h, A, k, reps=5):
    """Single-pass randomized LU (Alg. 10) at the workload shape: one pass over
    a column-major copy of A (the storage order the paper's one-pass form
    needs), two over the row-major A, against PowerLU at v = 2 without
    oversampling (the same approximation); residuals from plu_residual."""
    import torch
    m, n = A.shape
    Ac = A.t().contiguous().t()          # same matrix, columns contiguous
    res = {}
    for name, M in (("column_major_one_pass", Ac), ("row_major_two_passes", A)):
        f = h.single_pass(M, k, seed=31, sync_info=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            h.single_pass(M, k, seed=31, sync_info=False)
        e1.record()
        e1.synchronize()
        res[name] = {"ms": round(e0.elapsed_time(e1) / reps, 3),
                     "residual": h.residual(M, f)}
    g = h.fixed_rank(A, k, 0, 2, seed=31, sync_info=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        h.fixed_rank(A, k, 0, 2, seed=31, sync_info=False)
    e1.record()
    e1.synchronize()
    res["powerlu_v2_p0"] = {"ms": round(e0.elapsed_time(e1) / reps, 3),
                            "residual": h.residual(A, g)}
    res["k"] = k
    del Ac
    torch.cuda.empty_cache()
    return res


def _time_calls(fn, reps):
    """One synchronized call (its result kept), then reps timed calls."""
    import torch
    f = fn(True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn(False)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps, f


def baselines_section(h, A, k, p_over, reps=3):
    """The paper's fixed-rank timing comparison (Sec. 6.1, Fig. 1) at the
    workload shape: PowerLU at v = 2p + 2 against RandLU (Alg. 3 + Alg. 4)
    and RandSVD (Alg. 1 + Alg. 2) at power exponent p -- the same 2p + 2
    passes over A -- for p = 0 and 1; milliseconds per call and relative
    residuals (plu_residual for the LU forms; the RandSVD residual is
    sqrt(1 - sum s_i^2 / ||A||_F^2), exact for its orthonormal factors)."""
    out = {}
    for pw in (0, 1):
        v = 2 * pw + 2
        t_pl, f_pl = _time_calls(
            lambda sync: h.fixed_rank(A, k, p_over, v, seed=71, sync_info=sync), reps)
        t_rl, f_rl = _time_calls(
            lambda sync: h.randlu(A, k, p_over, pw, seed=71, sync_info=sync), reps)
        t_sv, f_sv = _time_calls(
            lambda sync: h.randsvd(A, k, p_over, pw, seed=71, sync_info=sync), reps)
        s_sv = f_sv[1].double()
        nA2 = f_sv[3]["normA2"]
        r_sv = float(max(0.0, 1.0 - float((s_sv * s_sv).sum()) / nA2)) ** 0.5
        out[f"p{pw}"] = {
            "passes": v,
            "powerlu_ms": round(t_pl, 3), "randlu_ms": round(t_rl, 3),
            "randsvd_ms": round(t_sv, 3),
            "speedup_powerlu_over_randlu": round(t_rl / t_pl, 3),
            "speedup_powerlu_over_randsvd": round(t_sv / t_pl, 3),
            "residual_powerlu": h.residual(A, f_pl), "residual_randlu": h.residual(A, f_rl),
            "residual_randsvd": r_sv,
        }
    out["paper_cpu_speedup_powerlu_over_randlu"] = {"p0": 1.80, "p1": 1.44}
    return out


def sparse_section(h, n=20000, density=0.003, k=100, p_over=10, reps=3):
    """The paper's sparse experiment (Sec. 6.1, Fig. 2) at one size: a
    sprand-like n x n matrix (uniform values, density 0.3%) in compressed
    rows.  The SpMM passes (ms and the rate of X rows gathered), then
    PowerLU at v = 2p + 2 against RandLU and RandSVD at p (2p + 2 passes),
    p = 0 and 1, and PowerLU on the same matrix stored dense.  Residuals of
    the LU forms by plu_residual on the dense copy; RandSVD's from its
    singular values."""
    import torch
    from synth import sprand_csr
    ip, ix, d = sprand_csr(n, n, density, 4242)
    dev = torch.device("cuda", 0)
    rp, ci, vv = (torch.from_numpy(x).to(dev) for x in (ip, ix, d))
    S = h.sparse_matrix(rp, ci, vv, (n, n))
    nnz = int(d.size)
    l = k + p_over
    X = torch.randn(n, l, device=dev)
    res = {"n": n, "density": density, "nnz": nnz, "k": k, "p_over": p_over}
    for name, trans in (("spmm_N_ms", False), ("spmm_T_ms", True)):
        t, _ = _time_calls(lambda sync: h.sparse_pass(S, X, trans=trans), 10)
        res[name] = round(t, 4)
        res[name.replace("_ms", "_gather_GBps")] = round(nnz * l * 4 / (t * 1e-3) / 1e9, 1)
    Ad = torch.sparse_csr_tensor(rp, ci, vv, size=(n, n)).to_dense()
    nA2 = float((Ad.double() ** 2).sum())
    for pw in (0, 1):
        v = 2 * pw + 2
        t_pl, f_pl = _time_calls(
            lambda sync: h.fixed_rank(S, k, p_over, v, seed=81, sync_info=sync), reps)
        t_rl, f_rl = _time_calls(
            lambda sync: h.randlu(S, k, p_over, pw, seed=81, sync_info=sync), reps)
        t_sv, f_sv = _time_calls(
            lambda sync: h.randsvd(S, k, p_over, pw, seed=81, sync_info=sync), reps)
        t_dn, f_dn = _time_calls(
            lambda sync: h.fixed_rank(Ad, k, p_over, v, seed=81, sync_info=sync), reps)
        s_sv = f_sv[1].double()
        res[f"p{pw}"] = {
            "passes": v,
            "powerlu_ms": round(t_pl, 3), "randlu_ms": round(t_rl, 3),
            "randsvd_ms": round(t_sv, 3), "powerlu_dense_storage_ms": round(t_dn, 3),
            "residual_powerlu": h.residual(Ad, f_pl), "residual_randlu": h.residual(Ad, f_rl),
            "residual_randsvd": float(max(0.0, 1.0 - float((s_sv * s_sv).sum()) / nA2)) ** 0.5,
            "residual_powerlu_dense_storage": h.residual(Ad, f_dn),
        }
    del Ad
    S.close()
    torch.cuda.empty_cache()
    return res


def precision_forms(h, A, outs, m, n, k, p_over, resid_fp32, steps=3):
    """The precision form (rounded passes, fp32 refinement pass) on the same
    workload and seeds as the fp32 step; residuals against the fp32 path's.
    Timed both as four single calls in turn and as one plu_batched call
    (side by side, as the fp32 step), whose results must equal the single
    calls' bit for bit."""
    import torch
    l = k + p_over
    flops_step = sum(flops_fixed_rank(m, n, k, l, v) for v in VS)
    res = {}
    for name, prec in FORMS.items():
        def step(seed):
            for v in VS:
                h.fixed_rank(A, k, p_over, v, seed=seed * 16 + v, prec=prec, sync_info=False,
                             out=outs[v])
        probs = [dict(A=A, mode=0, k=k, p_over=p_over, v=v, seed=0, prec=prec, out=outs[v])
                 for v in VS]

        def step_batched(seed):
            for v, pr in zip(VS, probs):
                pr["seed"] = seed * 16 + v
            h.batched(probs)
        step(999)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            step(i)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        step_batched(7)
        torch.cuda.synchronize()
        got = {v: [t.clone() for t in outs[v]] for v in VS}
        step(7)
        torch.cuda.synchronize()
        identical = all(all(torch.equal(a, b) for a, b in zip(got[v], outs[v])) for v in VS)
        del got
        t0 = time.perf_counter()
        for i in range(steps):
            step_batched(i)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / steps
        rr = {}
        for v in VS:
            f = h.fixed_rank(A, k, p_over, v, seed=5 + v, prec=prec, sync_info=True, out=outs[v])
            rr[str(v)] = h.residual(A, f)
        res[name] = {
            "ms_per_step": round(dt * 1e3, 3),
            "gflops": round(flops_step / dt / 1e9, 2),
            "batched_ms_per_step": round(dtb * 1e3, 3),
            "batched_gflops": round(flops_step / dtb / 1e9, 2),
            "batched_equals_single_calls": bool(identical),
            "residual": rr,
            "residual_ratio_vs_fp32": {v_: rr[v_] / resid_fp32[v_] for v_ in rr},
        }
    # one rounded pass of each format over the kept copies (sketch rounding and
    # split-K sum included) against HBM
    passes = {}
    for name, prec, bytes_a in (("bf16", 1, 2.0 * m * n), ("fp8_e4m3", 2, m * n * (1 + 1 / 32.0))):
        t = _pass_times(h, A, l, prec=prec)
        ms = 0.5 * (t["N"] + t["T"])
        passes[name] = {"ms": t, "bound": "hbm", "algorithmic_bytes": bytes_a,
                        "achieved_gbs": round(bytes_a / (ms * 1e-3) / 1e9, 1),
                        "frac": round(bytes_a / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
    res["passes"] = passes
    return res


SOURCE_N = 8192


def serving_pool(pool_size, seed=5000):
    """Host sources of the serving workload: pool_size pinned 8192 x 8192
    low-rank-plus-noise matrices with ranks r spread evenly over [16, 256],
    sigma_i = exp(-i/(r/4)), ||noise||_F = 1e-4 ||signal||_F.  Each request
    takes its own m x n block of one of them (``request_stream``)."""
    import numpy as np
    import torch
    from synth import spectrum, lowrank_factors
    pool = []
    N = SOURCE_N
    for i, r in enumerate(np.linspace(16, 256, pool_size).round().astype(int)):
        r = int(r)
        sig = spectrum("exp", r, tau=r / 4.0)
        X, sg, Y = lowrank_factors(N, N, sig, seed + 100 * i + 1, seed + 100 * i + 2)
        XS = (X * sg).astype(np.float32)
        Yt = np.ascontiguousarray(Y.T.astype(np.float32))
        g = np.random.default_rng(seed + 100 * i + 3)
        scale = np.float32(1e-4 * np.linalg.norm(sig) / N)
        A = torch.empty((N, N), dtype=torch.float32, pin_memory=True)
        An = A.numpy()
        for r0 in range(0, N, 1024):
            blk = XS[r0:r0 + 1024] @ Yt
            blk += scale * g.standard_normal((blk.shape[0], N), dtype=np.float32)
            An[r0:r0 + 1024] = blk
        pool.append((A, r))
    return pool


def request_stream(pool, count, seed):
    """cfg5's request distribution: per request m, n ~ U[512, 8192] and
    r ~ U[16, 256]; the data is an m x n block at a random offset of the
    source whose rank is nearest r (a strided view of pinned host memory)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    ranks = np.array([r for (_, r) in pool])
    out = []
    for i in range(count):
        m, n = (int(x) for x in rng.integers(512, 8193, 2))
        r = int(rng.integers(16, 257))
        j = int(np.argmin(np.abs(ranks - r)))
        r0 = int(rng.integers(0, SOURCE_N - m + 1))
        c0 = int(rng.integers(0, SOURCE_N - n + 1))
        src = pool[j][0]
        out.append((src[r0:r0 + m, c0:c0 + n], int(ranks[j])))
    return out


def pass_roofline_s(prm, m, n, rank):
    """Attainable time of a request's passes over A on their roofline: each
    pass max(2 m n c / FP32 MFMA peak, 4 m n / HBM peak) with c its columns
    (every other step taken as free)."""
    def one(c):
        return max(2.0 * m * n * c / (PEAK_FP32_MFMA_TFLOPS * 1e12), 4.0 * m * n / (PEAK_HBM_GBS * 1e9))
    if prm["mode"] == 0:
        l = prm["k"] + prm["p_over"]
        return (prm["v"] - 1) * one(l) + one(prm["k"])
    l = min(50 * 16, 16 * ((min(m, n) - 1) // 16))
    return prm["v"] * one(l)


def request_params(i, r, m, n, rng):
    """Even requests fixed rank (k = r/2, p = 10, v ~ U{2..5}); odd ones
    fixed precision (eps = 1e-3, b = 16, default l, v = 4)."""
    if i % 2 == 0:
        k = max(1, r // 2)
        p_over = 10 if k + 10 < min(m, n) else 0
        return dict(mode=0, k=k, p_over=p_over, v=int(rng.integers(2, 6)), seed=7000 + i)
    return dict(mode=1, eps=1e-3, b=16, l=0, v=4, seed=7000 + i)


def request_flops(prm, m, n, rank):
    if prm["mode"] == 0:
        return flops_fixed_rank(m, n, prm["k"], prm["k"] + prm["p_over"], prm["v"])
    l = min(50 * 16, 16 * ((min(m, n) - 1) // 16))
    return flops_fixed_precision(m, n, l, rank, prm["v"])


def batched_vs_single(h, pool, count=32):
    """The same problems solved one call at a time and as one batch (and its
    graph replay for the fixed-rank ones) on the same GPU."""
    import numpy as np
    import torch
    rng = np.random.default_rng(11)
    dev = torch.device("cuda:0")
    probs = []
    for i, (Ab, r) in enumerate(request_stream(pool, count, seed=12)):
        m, n = Ab.shape
        prm = request_params(i, r, m, n, rng)
        probs.append(dict(A=Ab.to(dev).contiguous(), **prm))
    torch.cuda.synchronize()

    def single():
        outs = []
        for pr in probs:
            if pr["mode"] == 0:
                outs.append(h.fixed_rank(pr["A"], pr["k"], pr["p_over"], pr["v"], seed=pr["seed"],
                                         sync_info=False))
            else:
                outs.append(h.fixed_precision(pr["A"], pr["eps"], pr["b"], l=pr["l"], v=pr["v"],
                                              seed=pr["seed"]))
        torch.cuda.synchronize()
        return outs

    single()
    t0 = time.perf_counter()
    s_out = single()
    t_single = time.perf_counter() - t0
    h.batched(probs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b_out = h.batched(probs)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    same = all(np.array_equal(a.L.cpu().numpy(), b.L.cpu().numpy()) and
               np.array_equal(a.p.cpu().numpy(), b.p.cpu().numpy()) for a, b in zip(s_out, b_out))
    fr = [pr for pr in probs if pr["mode"] == 0]
    h.batched(fr, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h.batched(fr, graph=True)
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    t0 = time.perf_counter()
    h.batched(fr)
    torch.cuda.synchronize()
    t_fr_batch = time.perf_counter() - t0
    flops = sum(request_flops(pr, pr["A"].shape[0], pr["A"].shape[1], o.rank)
                for pr, o in zip(probs, b_out))
    t_att = sum(pass_roofline_s(pr, pr["A"].shape[0], pr["A"].shape[1], o.rank)
                for pr, o in zip(probs, b_out))
    return {
        "problems": count, "shapes": "per problem: m, n ~ U[512, 8192], r ~ U[16, 256]",
        "single_calls_ms": round(t_single * 1e3, 2), "batched_ms": round(t_batch * 1e3, 2),
        "speedup": round(t_single / t_batch, 3), "batched_gflops": round(flops / t_batch / 1e9, 1),
        "pass_roofline_ms": round(t_att * 1e3, 3),
        "attainable_frac": round(t_att / t_batch, 4),
        "results_identical": bool(same),
        "fixed_rank_subset": {"problems": len(fr), "batched_ms": round(t_fr_batch * 1e3, 2),
                              "graph_replay_ms": round(t_graph * 1e3, 2)},
    }


def serving(pool, count=1024, rate=200.0, budget_gb=64, slots=64, seed=5000):
    """Replay of a Poisson request stream through the serving loop: each
    request its own m x n block of a pinned host source (request_stream);
    latency = completion minus scheduled arrival.  rate None: every request
    submitted at once (the loop's capacity)."""
    import threading
    import numpy as np
    import paper_2002_07138_amd as plu
    rng = np.random.default_rng(seed + 1)
    gaps = rng.exponential(1.0 / rate, count) if rate else np.zeros(count)
    sched = np.cumsum(gaps)
    srv = plu.Server(0, hbm_budget_bytes=int(budget_gb) << 30, max_slots=slots)
    tickets, late, meta = [], [], []
    results = [None] * count

    def waiter():
        for i in range(count):
            while len(tickets) <= i:
                time.sleep(0.0005)
            results[i] = srv.wait(tickets[i])

    stream = request_stream(pool, count, seed=seed + 2)
    th = threading.Thread(target=waiter)
    th.start()
    t_start = time.perf_counter()
    for i in range(count):
        A, r = stream[i]
        m, n = A.shape
        prm = request_params(i, r, m, n, rng)
        delay = t_start + sched[i] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        late.append(max(0.0, time.perf_counter() - (t_start + sched[i])))
        kw = dict(prm)
        tickets.append(srv.submit(A, **kw))
        meta.append((prm, m, n))
    th.join()
    t_end = time.perf_counter()
    srv.close()
    lat = np.array([(res["t_done"] - res["t_submit"]) + lt for res, lt in zip(results, late)])
    queue = np.array([res["t_admit"] - res["t_submit"] for res in results])
    service = np.array([res["t_done"] - res["t_admit"] for res in results])
    flops = sum(request_flops(prm, m, n, res["rank"]) for (prm, m, n), res in zip(meta, results))
    t_att = sum(pass_roofline_s(prm, m, n, res["rank"]) for (prm, m, n), res in zip(meta, results))
    ok = sum(1 for res in results if res["status"] in (0, 1, 2))
    return {
        "requests": count, "rate_per_s": rate,
        "shapes": "per request: m, n ~ U[512, 8192], r ~ U[16, 256]",
        "sources": f"{len(pool)} pinned {SOURCE_N}^2 matrices, ranks {pool[0][1]}..{pool[-1][1]}",
        "p50_ms": round(float(np.percentile(lat, 50)) * 1e3, 2),
        "p99_ms": round(float(np.percentile(lat, 99)) * 1e3, 2),
        "mean_ms": round(float(lat.mean()) * 1e3, 2),
        "throughput_req_per_s": round(count / (t_end - t_start), 1),
        "gflops": round(flops / (t_end - t_start) / 1e9, 1),
        "pass_roofline_s": round(t_att, 4),
        "attainable_frac": round(t_att / (t_end - t_start), 4),
        "completed_ok": ok,
        "mean_queue_ms": round(float(queue.mean()) * 1e3, 2),
        "mean_service_ms": round(float(service.mean()) * 1e3, 2),
        "mean_service_ms_by_mode": {
            "fixed_rank": round(float(np.mean([sv for sv, (prm, m, n) in zip(service, meta)
                                                if prm["mode"] == 0])) * 1e3, 2),
            "fixed_precision": round(float(np.mean([sv for sv, (prm, m, n) in zip(service, meta)
                                                     if prm["mode"] == 1])) * 1e3, 2)},
        "hbm_budget_gb": budget_gb, "slots": slots,
        "latency_includes": "H2D copy of A, all steps, D2H copy of p, q, L, U",
    }


def kernel_source_hash() -> str:
    """sha256[:16] over the pass kernel's source and the split planner
    (pass_plan in api.hip): the counted bytes depend on both."""
    csrc = os.path.join(ROOT, "paper_2002_07138_amd", "csrc")
    api = open(os.path.join(csrc, "api.hip")).read()
    i = api.index("GemmPlan pass_plan(")
    planner = api[i:api.index("\n}\n", i) + 3]
    h = hashlib.sha256(open(os.path.join(csrc, "k_gemm.hip"), "rb").read())
    h.update(planner.encode())
    return h.hexdigest()[:16]


def load_traffic():
    """HBM bytes per pass launch from the committed rocprofv3 counter summary,
    only if it was taken on the current pass-kernel source."""
    p = os.path.join(ROOT, "profiles", "pass_kernel_square20000_traffic.json")
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d


def cpu_baseline(A_host, k, p_over, v, seed):
    """The FP64 oracle, as it stands, on one fixed-rank factorization of the
    same matrix (bounded sample: one v, not the four of a step)."""
    import numpy as np
    from oracle import powerlu as O
    from synth import gaussian_omega
    m, n = A_host.shape
    l = k + p_over
    Om = gaussian_omega(m if v % 2 == 0 else n, l, seed=seed).astype(np.float64)
    A64 = A_host.astype(np.float64)
    t0 = time.perf_counter()
    f = O.powerlu(A64, k, Om, v)
    dt = time.perf_counter() - t0
    r = O.relative_residual(A64, f.p, f.q, f.L, f.U)
    threads = None
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max((i.get("num_threads", 0) for i in info), default=None)
    except Exception:
        pass
    return {
        "value": flops_fixed_rank(m, n, k, l, v) / dt / 1e9,
        "unit": "GFLOP/s",
        "cores": threads or os.cpu_count(),
        "kind": "oracle",
        "sample": f"one fixed-rank PowerLU (v={v}, k={k}, l={l}) of the {m}x{n} workload "
                  f"matrix in float64 NumPy, {dt:.2f} s",
        "seconds": dt,
        "residual": r,
        "p": f.p, "q": f.q,
    }


def profile_lowp(m, n):
    """The precision-form pass kernels only: for BF16 and FP8, one pass per
    direction that makes the rounded copies of A, then 3 passes A X and 3
    passes A^T X on the kept copies (PLU_PREC_A_UNCHANGED), at the workload
    shape (l = 110) and at 32768^2 with l = 220 (the wide kernels); then 3
    copies of 1 GiB (the calibration kernel for the HBM byte counters)."""
    import torch
    import paper_2002_07138_amd as plu
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(3)
    h = plu.Handle(0)
    for (mm, nn, l) in ((m, n, K_RANK + P_OVER), (32768, 32768, 220)):
        A = torch.randn((mm, nn), device=dev, generator=g)
        X_n = _sketch(nn, l, dev, g)
        X_m = _sketch(mm, l, dev, g)
        out_m = _sketch(mm, l, dev, fill=False)
        out_n = _sketch(nn, l, dev, fill=False)
        for prec in (1, 2):
            h.pass_(A, X_n, trans=False, out=out_m, prec=prec)
            for _ in range(3):
                h.pass_(A, X_n, trans=False, out=out_m, prec=prec | A_UNCHANGED)
            for _ in range(3):
                h.pass_(A, X_m, trans=True, out=out_n, prec=prec | A_UNCHANGED)
        del A, X_n, X_m, out_m, out_n
        torch.cuda.empty_cache()
    src = torch.empty(2 ** 28, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def profile_pass(m, n):
    """Dominant kernel only: one tuning pass per direction, then 3 passes A X
    and 3 passes A^T X at the workload
    shape (A is a seeded Gaussian matrix of the workload size: the kernels do
    not depend on its values), then 3 copies of 1 GiB (the calibration
    kernel for the HBM byte counters: 1 GiB read and 1 GiB written each)."""
    import torch
    import paper_2002_07138_amd as plu
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    A = torch.randn((m, n), device=dev, generator=g)
    l = K_RANK + P_OVER
    X_n = _sketch(n, l, dev, g)
    X_m = _sketch(m, l, dev, g)
    out_m = _sketch(m, l, dev, fill=False)
    out_n = _sketch(n, l, dev, fill=False)
    h = plu.Handle(0)
    # the first pass of each direction picks its split plan (timed candidates);
    # the counted launches are the three of each direction after it
    h.pass_(A, X_n, trans=False, out=out_m)
    h.pass_(A, X_m, trans=True, out=out_n)
    for _ in range(3):
        h.pass_(A, X_n, trans=False, out=out_m)
    for _ in range(3):
        h.pass_(A, X_m, trans=True, out=out_n)
    src = torch.empty(2 ** 28, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    h.close()
    print(json.dumps({"profile_pass": True, "m": m, "n": n, "l": l,
                      "pass_algorithmic_bytes": 4.0 * m * n,
                      "copy_bytes_each_direction": 4 * 2 ** 28}))


def profile_lu(M=20000, c=110, reps=10):
    """The LU panel kernel alone: GETRF with partial pivoting of a seeded
    Gaussian M x c matrix (Alg. 6/7's lu(.) at the bench shape), one warm
    call, then reps calls, then 3 copies of 1 GiB (the byte counters'
    calibration kernel)."""
    import torch
    import paper_2002_07138_amd as plu
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(M + c)
    X0 = torch.randn(M, c, device=dev, generator=g)
    X = X0.clone()
    h = plu.Handle(0)
    h.getrf(X, sync_info=False)
    for _ in range(reps):
        X.copy_(X0)
        h.getrf(X, want_perm=True, want_u=True, sync_info=False)
    src = torch.empty(2 ** 28, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    h.close()
    print(json.dumps({"profile_lu": True, "M": M, "c": c, "reps": reps,
                      "algorithmic_bytes": 8.0 * M * c, "copy_bytes_each_direction": 4 * 2 ** 28}))


def measured_peaks(h, dev):
    """What this GPU sustains next to the datasheet peaks (plu_measure_peak):
    back-to-back matrix-core instructions of the kinds the passes issue, and
    a streaming read of 2 GiB from HBM; best of 5 launches each."""
    import torch
    import paper_2002_07138_amd as plu
    buf = torch.empty(2 ** 29, dtype=torch.float32, device=dev)
    out = {
        "mfma_fp32_tflops": round(h.measure_peak(plu.PEAK_MFMA_FP32), 2),
        "mfma_bf16_tflops": round(h.measure_peak(plu.PEAK_MFMA_BF16), 1),
        "mfma_fp8_tflops": round(h.measure_peak(plu.PEAK_MFMA_FP8), 1),
        "hbm_read_gbs": round(h.measure_peak(plu.PEAK_HBM_READ, buf), 1),
        "datasheet": {"mfma_fp32_tflops": PEAK_FP32_MFMA_TFLOPS,
                      "mfma_bf16_tflops": PEAK_BF16_MFMA_TFLOPS,
                      "mfma_fp8_tflops": PEAK_FP8_MFMA_TFLOPS, "hbm_gbs": PEAK_HBM_GBS},
    }
    del buf
    return out


def profile_residual(m, n, k=K_RANK, reps=3):
    """The residual kernel alone (plu_residual: ||A - L U||_F recomputed tile
    by tile with float64 accumulation, the bench's error measure): one
    fixed-rank factorization of a seeded Gaussian m x n matrix, one warm
    residual, then reps residuals, then 3 copies of 1 GiB (the byte
    counters' calibration kernel)."""
    import torch
    import paper_2002_07138_amd as plu
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(m + k)
    A = torch.randn((m, n), device=dev, generator=g)
    h = plu.Handle(0)
    f = h.fixed_rank(A, k, P_OVER, 2, seed=3)
    h.residual(A, f)
    for _ in range(reps):
        h.residual(A, f)
    src = torch.empty(2 ** 28, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    h.close()
    print(json.dumps({"profile_residual": True, "m": m, "n": n, "k": k, "reps": reps,
                      "bytes_of_A": 4.0 * m * n, "flops": 2.0 * m * n * k,
                      "copy_bytes_each_direction": 4 * 2 ** 28}))


def profile_single_pass(m, n, k=100):
    """HBM bytes of the single-pass LU: after a 1 GiB fill (the start mark),
    one call on a column-major A (one pass), a 1 GiB copy (calibration, and
    the boundary between the two), one call on the row-major A (two passes)."""
    import torch
    import paper_2002_07138_amd as plu
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev)
    g.manual_seed(2)
    A = torch.randn((m, n), device=dev, generator=g)
    Ac = A.t().contiguous().t()
    h = plu.Handle(0)
    src = torch.empty(2 ** 28, device=dev)
    dst = torch.empty_like(src)
    h.single_pass(Ac, k, seed=3, sync_info=True)      # workspace and plans
    h.single_pass(A, k, seed=3, sync_info=True)
    torch.cuda.synchronize()
    src.fill_(1.0)                                    # marks the start of the counted calls
    h.single_pass(Ac, k, seed=3, sync_info=False)
    dst.copy_(src)
    h.single_pass(A, k, seed=3, sync_info=False)
    torch.cuda.synchronize()
    h.close()
    print(json.dumps({"profile_single_pass": True, "m": m, "n": n, "k": k,
                      "bytes_of_A": 4.0 * m * n, "copy_bytes_each_direction": 4 * 2 ** 28}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--size", type=int, default=20000, help="reduced sizes for quick checks")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision forms")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 32768^2 precision-form and 30000x20000 fixed-precision sections")
    ap.add_argument("--no-baselines", action="store_true",
                    help="skip the RandLU / RandSVD comparison")
    ap.add_argument("--serving-count", type=int, default=1024,
                    help="requests of the serving replay (0 skips it and the batch comparison)")
    ap.add_argument("--pool", type=int, default=16, help="distinct matrices of the serving replay")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the batched comparison and the serving replay")
    ap.add_argument("--profile-single-pass", action="store_true",
                    help="run only the single-pass LU on a column-major and a row-major A "
                         "around a plain 1 GiB copy, for hardware-counter runs")
    ap.add_argument("--profile-lu", action="store_true",
                    help="run only the LU of a 20000 x 110 Gaussian matrix (10 calls) and a plain "
                         "1 GiB copy, for kernel-trace and hardware-counter runs")
    ap.add_argument("--profile-residual", action="store_true",
                    help="run only plu_residual on a 20000^2 fixed-rank factorization and a "
                         "plain 1 GiB copy, for kernel-trace and hardware-counter runs")
    ap.add_argument("--profile-lowp", action="store_true",
                    help="run only the BF16 and FP8 pass kernels (20000^2, l = 110 and "
                         "32768^2, l = 220) and a plain 1 GiB copy, for kernel-trace and "
                         "hardware-counter runs")
    ap.add_argument("--profile-pass", action="store_true",
                    help="run only the pass kernels at the workload shape (3 launches per "
                         "direction) and a plain 1 GiB copy, for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this library runs on one GPU only (the multi-GPU design is "
              "described, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2002_07138_amd as plu
    from synth import WORKLOADS, workload_matrix

    w = WORKLOADS[WORKLOAD]
    m = n = args.size
    if args.profile_pass:
        profile_pass(m, n)
        return
    if args.profile_lowp:
        profile_lowp(m, n)
        return
    if args.profile_residual:
        profile_residual(m, n)
        return
    if args.profile_single_pass:
        profile_single_pass(m, n)
        return
    if args.profile_lu:
        profile_lu()
        return
    if args.serving_only:
        pool = serving_pool(args.pool)
        h = plu.Handle(0)
        out = {"batched": batched_vs_single(h, pool)}
        h.close()
        out["serving"] = serving(pool, count=args.serving_count)
        out["serving_burst"] = serving(pool, count=max(args.serving_count // 2, 1), rate=None)
        print(json.dumps(out))
        return
    t_gen = time.perf_counter()
    A_host = workload_matrix(w, m, n)
    t_gen = time.perf_counter() - t_gen
    dev = torch.device("cuda:0")
    A = torch.from_numpy(A_host).to(dev)
    k, p_over = K_RANK, P_OVER
    l = k + p_over
    h = plu.Handle(0)
    stream = torch.cuda.current_stream(dev)
    outs = {v: (torch.empty(m, dtype=torch.int32, device=dev),
                torch.empty(n, dtype=torch.int32, device=dev),
                torch.empty((m, k), dtype=torch.float32, device=dev),
                torch.empty((k, n), dtype=torch.float32, device=dev)) for v in VS}

    probs = [dict(A=A, mode=0, k=k, p_over=p_over, v=v, seed=0, out=outs[v]) for v in VS]

    def step(seed):
        # the four factorizations as one batch (plu_batched): side by side on
        # the handle's streams, so one's LU panels overlap another's passes
        for v, pr in zip(VS, probs):
            pr["seed"] = seed * 16 + v
        h.batched(probs)

    def step_single(seed):
        # the same four factorizations one call after another on one stream
        for v in VS:
            h.fixed_rank(A, k, p_over, v, seed=seed * 16 + v, sync_info=False, out=outs[v])

    for i in range(args.warmup):
        step_single(1000 + i)
        step(1000 + i)
    torch.cuda.synchronize()
    # the batch gives the single calls' bits
    step(5)
    torch.cuda.synchronize()
    got = {v: [t.clone() for t in outs[v]] for v in VS}
    step_single(5)
    torch.cuda.synchronize()
    batch_identical = all(all(torch.equal(a, b) for a, b in zip(got[v], outs[v])) for v in VS)
    del got
    # per-step events on the library's stream (no host synchronization between steps)
    step_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
    t0 = time.perf_counter()
    for i in range(args.steps):
        step_ev[i][0].record(stream)
        step(i)
        step_ev[i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    step_ms = [e0.elapsed_time(e1) for e0, e1 in step_ev]
    ms_per_step = elapsed * 1e3 / args.steps
    flops_step = sum(flops_fixed_rank(m, n, k, l, v) for v in VS)
    gflops = flops_step / (elapsed / args.steps) / 1e9

    # the same step as four single calls in sequence, and as a graph replay
    # of the batch (same requests every replay)
    single_ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                 for _ in range(args.steps)]
    for i in range(args.steps):
        single_ev[i][0].record(stream)
        step_single(i)
        single_ev[i][1].record(stream)
    torch.cuda.synchronize()
    single_ms = [e0.elapsed_time(e1) for e0, e1 in single_ev]
    for v, pr in zip(VS, probs):
        pr["seed"] = 31 * 16 + v
    h.batched(probs, graph=True)
    graph_ms = []
    for i in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        h.batched(probs, graph=True)
        e1.record(stream)
        e1.synchronize()
        graph_ms.append(e0.elapsed_time(e1))

    # per-v latency (one call each, events on the library's stream)
    per_v = {}
    for v in VS:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for r in range(3):
            h.fixed_rank(A, k, p_over, v, seed=77 + r, sync_info=False, out=outs[v])
        e1.record(stream)
        e1.synchronize()
        per_v[str(v)] = e0.elapsed_time(e1) / 3

    # dominant kernel: one pass over A (both directions), timed live with HIP
    # events on the stream the library launches on
    # the sketch and the output laid out as the factorizations' own passes
    # have them (rows padded to whole float4s)
    X_n = _sketch(n, l, dev)
    X_m = _sketch(m, l, dev)
    out_m = _sketch(m, l, dev, fill=False)
    out_n = _sketch(n, l, dev, fill=False)
    reps = 20
    for _ in range(3):
        h.pass_(A, X_n, trans=False, out=out_m)
        h.pass_(A, X_m, trans=True, out=out_n)
    pass_ms = {}
    for name, fn in (("N", lambda: h.pass_(A, X_n, trans=False, out=out_m)),
                     ("T", lambda: h.pass_(A, X_m, trans=True, out=out_n))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        e1.synchronize()
        pass_ms[name] = e0.elapsed_time(e1) / reps
    pass_flops = 2.0 * m * n * l
    avg_pass_ms = 0.5 * (pass_ms["N"] + pass_ms["T"])
    achieved_tflops = pass_flops / (avg_pass_ms * 1e-3) / 1e12

    # quality at the timed configuration: GPU residual per v (plu_residual)
    resid = {}
    for v in VS:
        f = h.fixed_rank(A, k, p_over, v, seed=5 + v, sync_info=True, out=outs[v])
        resid[str(v)] = h.residual(A, f)

    if not args.no_forms:
        forms = precision_forms(h, A, outs, m, n, k, p_over, resid)
        single = single_pass_section(h, A, k)
    traffic = load_traffic()
    peaks = measured_peaks(h, dev)
    roofline = {
        "bound": "mfma",
        "achieved": round(achieved_tflops, 3),
        "peak": PEAK_FP32_MFMA_TFLOPS,
        "unit": "TFLOP/s",
        "frac": round(achieved_tflops / PEAK_FP32_MFMA_TFLOPS, 4),
        "traffic": traffic["bytes_per_launch"] if traffic else None,
        "kernel": "pass over A (k_pass + split-K reduction), FP32 MFMA 16x16x4",
        "flops_per_launch": pass_flops,
        "avg_launch_ms": {"N": round(pass_ms["N"], 4), "T": round(pass_ms["T"], 4)},
        "peak_measured": peaks["mfma_fp32_tflops"],
        "frac_of_measured": round(achieved_tflops / peaks["mfma_fp32_tflops"], 4),
    }

    result = {
        "metric": "PowerLU GFLOP/s (% MFMA roofline) at fixed residual; batched p50/p99 latency",
        "value": round(gflops, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "step_ms": _stats(step_ms),
        "step": "the four factorizations (v = 2, 3, 4, 5) as one plu_batched call, side by side "
                "on the handle's streams; bitwise equal to four single calls: "
                + str(bool(batch_identical)),
        "single_calls_step_ms": _stats(single_ms),
        "single_calls_gflops": round(flops_step / (float(np.median(single_ms)) * 1e-3) / 1e9, 2),
        "batch_graph_replay_step_ms": _stats(graph_ms),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "m": m, "n": n, "k": k, "p_over": p_over,
                   "v": list(VS), "signal_rank": w.rank, "sigma": "exp(-i/40)",
                   "noise": "1e-4*N(0,1)/sqrt(n)", "omega": "Philox4x32-10 on device"},
        "roofline": roofline,
        "measured_peaks": peaks,
        "per_v_ms": {k_: round(v_, 3) for k_, v_ in per_v.items()},
        "residual": resid,
        "input_generation_s": round(t_gen, 2),
    }
    if not args.no_forms:
        result["precision_forms"] = forms
        result["single_pass"] = single
    if not args.no_baselines:
        result["baselines"] = baselines_section(h, A, k, p_over)
        result["sparse"] = sparse_section(h)

    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        cb = cpu_baseline(A_host, k, p_over, 3, seed=1000 * w.index + 3)
        # the GPU on the same Omega, for the residual ratio at this workload
        from synth import gaussian_omega
        Om = gaussian_omega(n, l, seed=1000 * w.index + 3)
        f = h.fixed_rank(A, k, p_over, 3, Omega=torch.from_numpy(Om).to(dev), out=outs[3])
        r_gpu = h.residual(A, f)
        pg = f.p.cpu().numpy()[:k]
        qg = f.q.cpu().numpy()[:k]
        result["parity_v3"] = {
            "residual_gpu": r_gpu, "residual_oracle": cb["residual"],
            "ratio": r_gpu / cb["residual"],
            "row_pivots_equal_first_k": bool(np.array_equal(pg, cb["p"][:k])),
            "col_pivots_equal_first_k": bool(np.array_equal(qg, cb["q"][:k])),
        }
        result["cpu_baseline"] = {kk: cb[kk] for kk in ("value", "unit", "cores", "kind", "sample")}
    else:
        result["cpu_baseline"] = None
    del A
    torch.cuda.empty_cache()
    if not args.no_configs:
        result["square32768_pow15"] = square32768_section(h, cpu=not args.no_cpu_baseline)
        result["rect30000x20000_exp50"] = rect30000_section(h, cpu=not args.no_cpu_baseline)
    if args.serving_count > 0:
        t_pool = time.perf_counter()
        pool = serving_pool(args.pool)
        t_pool = time.perf_counter() - t_pool
        result["batched"] = batched_vs_single(h, pool)
        torch.cuda.empty_cache()
        result["serving"] = serving(pool, count=args.serving_count)
        result["serving"]["pool_generation_s"] = round(t_pool, 2)
        result["serving_burst"] = serving(pool, count=max(args.serving_count // 2, 1), rate=None)
    h.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
