"""Table 1 (Sec. 6.4) on the device: PowerLU_FP with the column rule
(Alg. 11), v = 4, l = 50 b, on square matrices of size 8000 of Matrix Types
1-3 (Sec. 6.2), the table's six (type, eps, b) rows, against the FP64
oracle's ranks on the same matrices and Gaussian test matrices (stored by
tests/golden/make_table1_oracle.py) and against the printed ranks.

The rank decision compares the indicator of Thm 4.3, E_j = ||A||^2 -
sum_{i<=j} ||A v_j||^2, with eps^2 ||A||^2.  A run's decision is resolved
at a precision whose indicator error is delta when the oracle's E after
k - 1 columns exceeds the threshold by more than delta and its E after k
columns falls below it by more than delta: then the device's rank must be
the oracle's.  delta is measured here (the device's E at its rank against
the oracle's curve at the same column), for both indicator forms: float32
column energies of G (the default), and PLU_PREC_FP64_INDICATOR (G in
float64).  The float32 form resolves E to about 1e-8 ||A||^2, so only the
eps = 1e-2 rows are decided above its rounding; the float64 form resolves
all six rows."""

import json
import os

import numpy as np
import pytest

from tests.gpu_common import torch, have_gpu, handle, dev, host
from oracle import powerlu as O
from synth import gaussian_omega, paper_type_family

pytestmark = [pytest.mark.gpu, pytest.mark.slow,
              pytest.mark.skipif(not have_gpu(), reason="needs a GPU")]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "table1_oracle.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


@pytest.fixture(scope="module")
def h():
    hh = handle()
    yield hh
    hh.close()


@pytest.fixture(scope="module")
def family():
    g = _golden()
    print(f"generating Matrix Types 1-3 at n = {g['n']} (host, float64)", flush=True)
    return paper_type_family(g["n"], g["family_seed"])


def omega_seed(row: int, s: int) -> int:
    return 8100 + 20 * row + s


def _run_row(h, family, r, row, prec=0):
    n, l, b, eps = row["n"], row["l"], row["b"], row["eps"]
    Ad = dev(family[row["type"]])
    out = []
    for run in row["runs"]:
        Om = gaussian_omega(n, l, seed=omega_seed(r, run["s"]))
        f = h.fixed_precision(Ad, eps, b, l=l, v=4, column_exact=True, Omega=dev(Om), prec=prec)
        res = h.residual(Ad, f) if run["s"] == 0 else None
        out.append(dict(s=run["s"], rank=f.rank, tol=f.info["tol_reached"],
                        e=f.info["E_final"] / f.info["normA2"], residual=res))
    del Ad
    torch.cuda.empty_cache()
    return out


def _resolved(run, eps2, delta):
    return run["e_prev"] - eps2 > delta and eps2 - run["e_at"] > delta


FP64_INDICATOR = 128
# bands of the indicator error (||A||_F^2-relative): float32 column energies
# of a float32 G = A V (measured up to 1.9e-8 on these inputs), and the
# float64 indicator (G in float64, first-order correction for V^T V - I;
# measured up to 4.7e-11, the largest on Type 1's slow decay, where the
# device's float32 basis spans a slightly different subspace than the
# oracle's)
BAND = {"float32": 2e-7, "float64": 1e-10}


@pytest.mark.parametrize("form", ["float32", "float64"])
@pytest.mark.parametrize("r", range(6))
def test_table1_row(h, family, r, form):
    """Rank parity: the runs whose oracle decision sits more than 3x the
    measured indicator error (device E at its rank against the oracle's E
    curve at the same column, run s = 0) from eps^2 give the oracle's rank
    exactly; with the float64 indicator the others stay within 2 columns and
    the mean rank over the runs is within 3% (or one column) of the printed
    average.  With the float32 indicator only the eps = 1e-2 rows resolve
    (eps^2 far above the float32 band): there every run matches and the
    residual is within 1.05x of the oracle's."""
    g = _golden()
    row = g["rows"][r]
    eps2 = row["eps"] ** 2
    got = _run_row(h, family, r, row, prec=0 if form == "float32" else FP64_INDICATOR)
    g0 = got[0]
    dev_err = abs(g0["e"] - row["E_s0"][g0["rank"] - 1])
    ranks = [x["rank"] for x in got]
    orc = [x["rank"] for x in row["runs"]]
    delta = max(3.0 * dev_err, 1e-13)
    compared = 0
    for x, o in zip(got, row["runs"]):
        if _resolved(o, eps2, delta):
            assert x["rank"] == o["rank"], (x, o)
            compared += 1
        elif form == "float64":
            assert abs(x["rank"] - o["rank"]) <= 2, (x, o)
    print(f"[{form}] row {r}: type {row['type']} eps {row['eps']:g} b {row['b']} l {row['l']}: "
          f"device ranks {ranks} (mean {np.mean(ranks):.2f}); oracle {orc} "
          f"(mean {np.mean(orc):.2f}); printed tsvd {row['k_tsvd']} powerlu_fp "
          f"{row['k_fp_printed']}; indicator error at s = 0: {dev_err:.3e} (eps^2 {eps2:.1e}); "
          f"runs decided above it: {compared} of {len(got)}; residual s = 0 device "
          f"{g0['residual']:.4e} oracle {row['residual_s0']:.4e}")
    assert dev_err <= BAND[form]
    if form == "float64":
        assert abs(np.mean(ranks) - row["k_fp_printed"]) <= max(1.0, 0.03 * row["k_fp_printed"])
    if form == "float64" or eps2 > 20 * BAND[form]:
        if form == "float32":
            assert compared == len(got)
        if g0["rank"] == row["runs"][0]["rank"]:
            assert g0["residual"] <= 1.05 * row["residual_s0"] + 1e-7
        assert g0["residual"] <= row["eps"] * (1 + 1e-3)
