"""Writes config4_gradients.txt: the FP64 oracle's exact parameter-shift
gradients of the 20-qubit hardware-efficient ansatz (10 layers of RY, RZ on
every qubit and a CZ ring; loss sum_i <Z_i Z_i+1>) for the 64 seeded parameter
vectors: all 400 angles of vectors 0 and 63, two angles drawn with
numpy.random.default_rng(400 + b) on every other vector b, and every loss
value.

Calls only the oracle and the seeded workload generator.  About 20 minutes on
8 cores:  python tests/golden/make_config4_gradients.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config4_gradients.txt")
VECTORS = (0, 63)


def sampled_angles(b, n_params):
    return sorted(int(x) for x in np.random.default_rng(400 + b).choice(n_params, size=2, replace=False))


def main():
    circ, params, (m, c) = workloads.config4()
    lines = ["# FP64 oracle, exact two-term parameter shift (each angle in one gate exp(-i t P/2)):",
             "# dE/dt = [E(t + pi/2) - E(t - pi/2)] / 2.  20-qubit HEA, 10 layers, loss sum_i <Z_i Z_(i+1) mod 20>.",
             "# Written by tests/golden/make_config4_gradients.py (oracle and workloads only).",
             "# columns: vector  index  value   (index -1: the loss E itself)"]
    for b in range(params.shape[0]):
        e = oracle.circuit_expectation(circ, params[b], m, c)
        lines.append(f"{b} -1 {e!r}")
        which = list(range(circ.n_params)) if b in VECTORS else sampled_angles(b, circ.n_params)
        g = oracle.param_shift_gradient(circ, params[b], m, c, which=which)
        for j in which:
            lines.append(f"{b} {j} {float(g[j])!r}")
        print(f"vector {b} done", flush=True)
    with open(OUT + ".tmp", "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    main()
