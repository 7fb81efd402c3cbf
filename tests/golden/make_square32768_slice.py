"""Writes square32768_slice4096_oracle.json: the FP64 oracle's relative
residual on the 4096 x 4096 leading block of the 32768^2 workload (rank 1000,
sigma_i = i^-1.5; synth.workload_slice), k = 200, oversampling 20, v = 4, the
Gaussian test matrix synth.gaussian_omega(4096, 220, seed 3003) -- exact
arithmetic, and each precision form's rounding (oracle.lowp) with its number
of exact closing passes.  Calls only oracle/ and synth/ (run from the
repository root: python tests/golden/make_square32768_slice.py)."""

import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import lowp as LP  # noqa: E402
from oracle import powerlu as O  # noqa: E402
from synth import WORKLOADS, gaussian_omega, workload_slice  # noqa: E402

FORMS = {                       # name -> (rounding, exact closing passes)
    "fp32": (None, 0),
    "bf16": (LP.round_bf16, 0),
    "bf16+refine_last": (LP.round_bf16, 1),
    "fp8_e4m3+refine_last": (LP.round_mx_e4m3, 1),
    "fp8_e4m3+refine_two": (LP.round_mx_e4m3, 2),
}


def main():
    w = WORKLOADS["square32768_pow15"]
    k, p_over, v = 200, 20, 4
    S = workload_slice(w, 4096, 4096)
    Om = gaussian_omega(4096, k + p_over, seed=1000 * w.index + 3).astype(np.float64)
    S64 = S.astype(np.float64)
    out = {"workload": w.name, "slice": [4096, 4096], "k": k, "p_over": p_over, "v": v,
           "omega_seed": 1000 * w.index + 3, "residual": {}}
    for name, (rnd, tail) in FORMS.items():
        f = O.powerlu(S64, k, Om, v, pass_round=rnd, exact_tail=tail)
        out["residual"][name] = O.relative_residual(S64, f.p, f.q, f.L, f.U)
        print(name, out["residual"][name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)),
                        "square32768_slice4096_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
