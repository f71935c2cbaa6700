"""Writes oracle_step_sizes.txt: the FP64 oracle's Lipschitz estimates L = ||A_s D_f||^2
(100 power iterations from the constant unit vector; the step size of Sec. 3 is 1 / L) for
the workloads whose full-size GPU parity tests would otherwise spend minutes of host time
recomputing them. Calls only the oracle and the seeded geometry rules of synth.

    python tests/golden/make_oracle_step_sizes.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2203_07308_amd import synth  # noqa: E402

ITERS = 100


def entries():
    w = synth.WORKLOADS["ms2g512"]
    for f, _ in w.stages:
        yield "ms2g512", w.geometry, f
    bw = synth.BATCH_WORKLOADS["batch64"]
    shapes = bw.shapes()
    for i in (3, 24):  # the batch's 384^2 x 720-view and 512^2 x 360-view slices
        n, V = shapes[i]
        for f, _ in bw.stages:
            yield f"batch64[{i}]", synth.fan_geometry(n, V), f


def main():
    out = os.path.join(HERE, "oracle_step_sizes.txt")
    lines = ["# FP64 oracle Lipschitz estimates L = ||A_s D_f||_2^2, 100 power iterations",
             "# (written by make_oracle_step_sizes.py; the oracle only)",
             "# workload  factor  L"]
    for name, gd, f in entries():
        L = oracle.power_lipschitz(oracle.Geometry(**gd), f, ITERS)
        lines.append(f"{name} {f} {L!r}")
        print(lines[-1], flush=True)
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
