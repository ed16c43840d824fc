"""The oracle still reproduces its frozen c0 result (tests/golden/c0_oracle.txt,
written by tests/golden/make_golden.py from the oracle alone)."""
import os

import numpy as np

import synth

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _read():
    beta, scal = {}, {}
    for line in open(os.path.join(HERE, "c0_oracle.txt")):
        if line.startswith("#"):
            continue
        parts = line.split()
        if parts[0] == "beta":
            beta[int(parts[1])] = float(parts[2])
        else:
            scal[parts[0]] = float(parts[1])
    return beta, scal


def test_oracle_matches_golden(orc):
    beta, scal = _read()
    d = synth.c0()
    lmax = orc.precompute(d["X"], d["y"])["lambda_max"]
    assert lmax == scal["lambda_max"]
    r = orc.lasso_path(d["X"], d["y"], lambdas=[lmax, lmax * d["lambda_ratio"]])
    b = r["beta"][1]
    assert set(np.flatnonzero(b)) == set(beta)
    for j, v in beta.items():
        assert b[j] == v
    assert r["gap"][1] == scal["gap"]
    assert r["epochs"][1] == scal["epochs"]
