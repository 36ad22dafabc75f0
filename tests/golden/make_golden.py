"""Writes the stored oracle reference for the small chirp workload.

The paper prints no numeric worked example (its figures carry no data), so
the fixture here is the oracle's own record on the 1,000 x 2,000 chirp
workload at tol 1e-10.  It is written only by this script, which calls
only `oracle/` and the shared seeded input generator; nothing produced by
the HIP path enters it.  tests/test_golden.py checks that the oracle still
reproduces it, so an unintended change to the oracle's arithmetic shows.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import rb_inputs as ri  # noqa: E402


def main():
    w = ri.WORKLOADS["chirp_small_c128"]
    S = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    out = {"workload": w.name, "N": w.N, "M": w.M, "tol": w.tol, "kmax": w.kmax}
    for mode in ("explicit", "pythag"):
        g = oracle.greedy(S, w.tol, w.kmax, mode=mode)
        out[mode] = {"k": g["k"], "status": g["status"], "piv": g["piv"].tolist(),
                     "err": [float(x) for x in g["err"]], "rho": [float(x) for x in g["rho"]],
                     "nu": g["nu"].tolist()}
    path = os.path.join(HERE, "chirp_small_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
