"""Writes tests/golden/batched_sample.npz: oracle values for one layer of each quadrature order of
the batched workload (256 layers, seed 3): layers 10, 9, 3, 0 and 2 have N = 16, 24, 32, 48 and
64; layer HARD is the one with the largest omega among the N = 64 layers.

Per layer i: F{i} = F_r for every (outgoing, incident) node pair at the azimuth differences
k = 0, n_dphi/8, n_dphi/4 and n_dphi/2 + 1 (cosine and sine blocks), all 16 Mueller elements,
shape (N, N, 4, 4, 4); az{i} = those k; scale{i} = max |F_II| over all outputs of the layer;
R{i} = R^m for m = 0, 1 and M - 1 (full 4N x 4N), Rscale{i} = max |R^m| over all orders.
Calls only the oracle and the input generator; about 2 minutes on 8 CPU cores.

    python tests/golden/make_batched_sample.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dom  # noqa: E402
from workloads import workload  # noqa: E402

PER_N = (10, 9, 3, 0, 2)


def layers(w):
    n64 = [i for i in range(w.n_layers) if w.N[i] == 64]
    hard = max(n64, key=lambda i: w.omega[i])
    return PER_N + (hard,)


def main():
    w = workload("batched")
    ls = layers(w)
    out = {"layers": np.array(ls)}
    for i in ls:
        F, R = dom.brdf(w.coef[i], w.tau[i], w.omega[i], w.N[i], w.M[i], w.n_dphi[i], return_orders=True)
        P = w.n_dphi[i]
        az = (0, P // 8, P // 4, P // 2 + 1)
        out[f"F{i}"] = np.ascontiguousarray(F[:, :, list(az)])
        out[f"az{i}"] = np.array(az)
        out[f"scale{i}"] = np.abs(F[..., 0, 0]).max()
        out[f"orders{i}"] = np.array([0, 1, w.M[i] - 1])
        out[f"R{i}"] = np.stack([R[m] for m in (0, 1, w.M[i] - 1)])
        out[f"Rscale{i}"] = max(np.abs(r).max() for r in R)
    np.savez_compressed(os.path.join(HERE, "batched_sample.npz"), **out)


if __name__ == "__main__":
    main()
