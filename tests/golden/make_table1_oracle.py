"""Writes table1_oracle.json: the FP64 oracle's PowerLU_FP ranks on the
setting of Table 1 (Sec. 6.4): square matrices of size 8000 of Matrix Types
1-3 (Sec. 6.2; synth.paper_type_family(8000, seed 8), one pair of random
orthonormal factors shared by the three types, rounded to float32 as the
device gets them), v = 4, l = 50 b, the column rule (Alg. 11), for each of
the table's six (type, eps, b) rows.

Per row and Gaussian test matrix s (synth.gaussian_omega(8000, l,
seed 8100 + 20 row + s)): the rank, and the indicator of Thm 4.3 after k - 1
and after k columns over ||A||_F^2 (how far the decision sits from the
threshold eps^2).  Twenty test matrices per row as in the paper's averages,
five for the l = 2000 row (each of its runs takes minutes here).  Run s = 0
also records the whole indicator curve over ||A||_F^2 and the relative
residual of the assembled factorization.

Calls only oracle/ and synth/ (run from the repository root:
python tests/golden/make_table1_oracle.py; about half an hour on 8 cores)."""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import powerlu as O  # noqa: E402
from synth import gaussian_omega, paper_type_family  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N, FAMILY_SEED, V_PASSES = 8000, 8, 4


def table_rows():
    rows = []
    with open(os.path.join(HERE, "table1_tsvd_ranks.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                t, eps, n, k_tsvd, k_fp, b = line.split()
                rows.append(dict(type=int(t), eps=float(eps), n=int(n), k_tsvd=int(k_tsvd),
                                 k_fp_printed=int(k_fp), b=int(b)))
    return rows


def omega_seed(row: int, s: int) -> int:
    return 8100 + 20 * row + s


def rank_only(A64, normA2, Om, eps, b):
    """Alg. 7's basis, G = A V, the column rule on Thm 4.3's indicator."""
    V = O.range_basis(A64, Om, V_PASSES)
    G = A64 @ V
    c = np.sum(G * G, axis=0)
    k, ok = O.rank_rule(normA2, c, eps, b, True)
    E = O.indicator(normA2, c)
    return k, ok, E


def main():
    rows = table_rows()
    fam = paper_type_family(N, FAMILY_SEED)
    out = {"n": N, "family_seed": FAMILY_SEED, "v": V_PASSES, "rule": "column (Alg. 11)",
           "omega_seed": "8100 + 20 * row + s", "rows": []}
    for r, row in enumerate(rows):
        t, eps, b = row["type"], row["eps"], row["b"]
        l = 50 * b
        A64 = fam[t].astype(np.float64)
        normA2 = float(np.sum(A64 * A64))
        runs = 5 if l > 1000 else 20
        res = dict(row, l=l, normA2=normA2, runs=[])
        for s in range(runs):
            t0 = time.time()
            Om = gaussian_omega(N, l, seed=omega_seed(r, s)).astype(np.float64)
            if s == 0:
                f = O.powerlu_fp(A64, eps, b, Om, V_PASSES, column_mode=True)
                k, ok, E = f.rank, f.tol_reached, f.E
                res["residual_s0"] = O.relative_residual(A64, f.p, f.q, f.L, f.U)
                res["E_s0"] = [float(e / normA2) for e in E]
            else:
                k, ok, E = rank_only(A64, normA2, Om, eps, b)
            res["runs"].append(dict(s=s, rank=int(k), tol_reached=bool(ok),
                                    e_prev=float(E[k - 2] / normA2) if k >= 2 else 1.0,
                                    e_at=float(E[k - 1] / normA2)))
            print(f"row {r} type {t} eps {eps:g} b {b} s {s}: rank {k} ({time.time() - t0:.1f} s)",
                  flush=True)
        res["mean_rank"] = float(np.mean([x["rank"] for x in res["runs"]]))
        out["rows"].append(res)
    with open(os.path.join(HERE, "table1_oracle.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
