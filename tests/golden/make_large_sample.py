"""Writes tests/golden/large_sample.npz: oracle values for the large workload (one layer, N = 128,
L = M = n_dphi = 256, tau = 50, omega = 0.999, seed 5).

Stored:
  F       F_r for every (outgoing i, incident q) node pair, including both ends of the mu grid, at
          the azimuth differences AZ (k = 0, 37, 64 = n_dphi/4 and 128 = n_dphi/2, so both the
          cosine and the sine blocks of the synthesis are hit), all 16 Mueller elements:
          shape (128, 128, 4, 4, 4)
  az      the azimuth indices k
  scale   max |F_II| over all outputs (the normalisation of the parity metric)
  orders  the Fourier orders m of the per-order samples
  idx     Stokes-system indices (4 i + r) of the nodes NODES, all four Stokes components
  Rrows   R^m[idx, :] for each m in orders: shape (len(orders), len(idx), 512)
  Rcols   R^m[:, idx] for each m in orders: shape (len(orders), 512, len(idx))
  Rscale  max |R^m| over all orders and entries
Calls only the oracle and the input generator; about 6 minutes on 8 CPU cores.

    python tests/golden/make_large_sample.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dom  # noqa: E402
from workloads import workload  # noqa: E402

AZ = (0, 37, 64, 128)
ORDERS = (0, 1, 2, 64, 255)
NODES = (0, 1, 63, 64, 126, 127)


def main():
    w = workload("large")
    F, R = dom.brdf(w.coef[0], w.tau[0], w.omega[0], w.N[0], w.M[0], w.n_dphi[0], return_orders=True)
    idx = np.array([4 * i + r for i in NODES for r in range(4)])
    np.savez_compressed(os.path.join(HERE, "large_sample.npz"),
                        F=np.ascontiguousarray(F[:, :, list(AZ)]),
                        az=np.array(AZ),
                        scale=np.abs(F[..., 0, 0]).max(),
                        orders=np.array(ORDERS),
                        idx=idx,
                        Rrows=np.stack([R[m][idx, :] for m in ORDERS]),
                        Rcols=np.stack([R[m][:, idx] for m in ORDERS]),
                        Rscale=max(np.abs(r).max() for r in R))


if __name__ == "__main__":
    main()
