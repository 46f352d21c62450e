"""Writes tests/golden/large_sample.npz: the oracle's F_r for the large workload (one layer,
N = 128, L = M = n_dphi = 256, tau = 50, omega = 0.999, seed 5) on a sample of outputs, every
16th outgoing node i, every 16th incident node q and every 32nd azimuth difference, all 16 Mueller
elements. Calls only the oracle and the input generator; about 7 minutes on 8 CPU cores.

    python tests/golden/make_large_sample.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dom  # noqa: E402
from workloads import workload  # noqa: E402

STRIDE_I, STRIDE_Q, STRIDE_K = 16, 16, 32


def main():
    w = workload("large")
    F = dom.brdf(w.coef[0], w.tau[0], w.omega[0], w.N[0], w.M[0], w.n_dphi[0])
    np.savez_compressed(os.path.join(HERE, "large_sample.npz"),
                        F=F[::STRIDE_I, ::STRIDE_Q, ::STRIDE_K],
                        scale=np.abs(F[..., 0, 0]).max(),
                        strides=np.array([STRIDE_I, STRIDE_Q, STRIDE_K]))


if __name__ == "__main__":
    main()
