"""The oracle reproduces its stored record on the small chirp workload
(tests/golden/chirp_small_oracle.json, written by tests/golden/make_golden.py
from the oracle alone).  This guards the oracle against unintended changes;
the record itself is pinned by tests/test_oracle_pins.py (Householder QRCP,
closed forms, theorems).  CPU only."""
import json
import os

import numpy as np

import oracle
import rb_inputs as ri

HERE = os.path.dirname(os.path.abspath(__file__))


def test_oracle_reproduces_golden_record():
    with open(os.path.join(HERE, "golden", "chirp_small_oracle.json")) as f:
        ref = json.load(f)
    w = ri.WORKLOADS[ref["workload"]]
    S = oracle.chirp(w.params(), w.N, w.flo, w.fhi)
    for mode in ("explicit", "pythag"):
        g = oracle.greedy(S, ref["tol"], ref["kmax"], mode=mode)
        r = ref[mode]
        assert g["k"] == r["k"] and g["status"] == r["status"]
        np.testing.assert_array_equal(g["piv"], r["piv"])
        np.testing.assert_allclose(g["err"], r["err"], rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(g["rho"], r["rho"], rtol=1e-12, atol=1e-15)
    # the explicit form reaches the tolerance; the Pythagorean form stalls at
    # its resolution floor far above it
    assert ref["explicit"]["err"][-1] < ref["tol"] <= ref["explicit"]["err"][-2]
    assert ref["pythag"]["err"][-1] > 100 * ref["tol"]
