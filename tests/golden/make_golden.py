"""Writes tests/golden/c0_oracle.txt from the CPU oracle only.

The workload is the single FP64 Lasso (50 x 500, lambda = lambda_max / 10,
screening every 10 epochs, gap <= 1e-8 ||y||^2) from the seeded generator.
The file freezes the oracle's result so that any later change to the
oracle's arithmetic shows up as a failing comparison.
Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    d = synth.c0()
    o = oracle.oracle()
    lmax = o.precompute(d["X"], d["y"])["lambda_max"]
    r = o.lasso_path(d["X"], d["y"], lambdas=[lmax, lmax * d["lambda_ratio"]])
    b = r["beta"][1]
    nz = np.flatnonzero(b)
    with open(os.path.join(HERE, "c0_oracle.txt"), "w") as fh:
        fh.write("# CPU oracle on the c0 workload (seed 0), written by make_golden.py\n")
        fh.write(f"lambda_max {float(lmax)!r}\n")
        fh.write(f"gap {float(r['gap'][1])!r}\n")
        fh.write(f"epochs {int(r['epochs'][1])}\n")
        fh.write(f"nactive {int(r['nactive'][1])}\n")
        for j in nz:
            fh.write(f"beta {int(j)} {float(b[j])!r}\n")


if __name__ == "__main__":
    main()
