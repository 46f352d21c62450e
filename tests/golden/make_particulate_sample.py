"""Writes tests/golden/particulate_sample.npz: oracle values for the particulate workload (one
layer, N = 32, L = M = n_dphi = 64, tau = 10, omega = 0.99, seed 2): F_r for every (outgoing,
incident) node pair at the azimuth differences k = 0, 8, 16 = n_dphi/4 and 33 (cosine and sine
blocks), all 16 Mueller elements, shape (32, 32, 4, 4, 4), with max |F_II| over all outputs.
Calls only the oracle and the input generator; about 10 seconds on 8 CPU cores.

    python tests/golden/make_particulate_sample.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dom  # noqa: E402
from workloads import workload  # noqa: E402

AZ = (0, 8, 16, 33)


def main():
    w = workload("particulate")
    F = dom.brdf(w.coef[0], w.tau[0], w.omega[0], w.N[0], w.M[0], w.n_dphi[0])
    np.savez_compressed(os.path.join(HERE, "particulate_sample.npz"), F=np.ascontiguousarray(F[:, :, list(AZ)]),
                        az=np.array(AZ), scale=np.abs(F[..., 0, 0]).max())


if __name__ == "__main__":
    main()
