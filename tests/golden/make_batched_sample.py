"""Writes tests/golden/batched_sample.npz: the oracle's F_r for three layers of the batched
workload (256 layers, seed 3; layers 0, 2 and 10 have N = 48, 64 and 16) on a sample of outputs,
every 8th outgoing node, incident node and azimuth difference, all 16 Mueller elements, with each
layer's max |F_II| over all outputs. Calls only the oracle and the input generator; about 1.5
minutes on 8 CPU cores.

    python tests/golden/make_batched_sample.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dom  # noqa: E402
from workloads import workload  # noqa: E402

LAYERS = (0, 2, 10)
STRIDE = 8


def main():
    w = workload("batched")
    out = {"layers": np.array(LAYERS), "stride": np.array(STRIDE)}
    for i in LAYERS:
        F = dom.brdf(w.coef[i], w.tau[i], w.omega[i], w.N[i], w.M[i], w.n_dphi[i])
        out[f"F{i}"] = F[::STRIDE, ::STRIDE, ::STRIDE]
        out[f"scale{i}"] = np.abs(F[..., 0, 0]).max()
    np.savez_compressed(os.path.join(HERE, "batched_sample.npz"), **out)


if __name__ == "__main__":
    main()
