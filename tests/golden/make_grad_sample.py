"""Writes tests/golden/grad_sample.npz: central finite differences of the oracle for the
differentiation workload (64 layers, N = 32, L = 64, M = n_dphi = 32, seed 4; targets from
workloads.differentiation_targets). Per layer the loss is
    sum over (i, q, k), r in {I, Q} and p of (F_r - F_r*)^2,
F_r* being the oracle's F_r at the layer's target parameters. Stored:
  tau_grad[64], omega_grad[64]       d loss / d tau and d loss / d omega of every layer
  coef_idx[32, 3], coef_grad[32]     (layer, family, degree) and d loss / d coefficient for eight
                                     random coefficients (degree >= 1) on each of layers 0..3
with the step h = 1e-6 max(1, |p|). Calls only the oracle and the input generators; about 10
minutes on 8 CPU cores.

    python tests/golden/make_grad_sample.py
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dom  # noqa: E402
from workloads import differentiation_targets, workload  # noqa: E402


def layer_loss(F, Ft):
    d = (F - Ft)[..., :2, :]
    return float(np.sum(d * d))


def main():
    w = workload("differentiation")
    t = differentiation_targets(w)
    n = w.n_layers
    args = lambda i: (w.N[i], w.M[i], w.n_dphi[i])
    Ft = [dom.brdf(t.coef[i], t.tau[i], t.omega[i], *args(i)) for i in range(n)]

    def loss(i, coef, tau, omega):
        return layer_loss(dom.brdf(coef, tau, omega, *args(i)), Ft[i])

    tau_grad = np.zeros(n)
    omega_grad = np.zeros(n)
    for i in range(n):
        h = 1e-6 * max(1.0, abs(w.tau[i]))
        tau_grad[i] = (loss(i, w.coef[i], w.tau[i] + h, w.omega[i]) - loss(i, w.coef[i], w.tau[i] - h, w.omega[i])) / (2 * h)
        h = 1e-6 * max(1.0, abs(w.omega[i]))
        omega_grad[i] = (loss(i, w.coef[i], w.tau[i], w.omega[i] + h) - loss(i, w.coef[i], w.tau[i], w.omega[i] - h)) / (2 * h)
    rng = np.random.default_rng(404)
    idx, cgrad = [], []
    for i in range(4):
        for _ in range(8):
            fam, l = int(rng.integers(0, 6)), int(rng.integers(1, w.L[i]))
            c = w.coef[i]
            h = 1e-6 * max(1.0, abs(c[fam, l]))
            cp, cm = c.copy(), c.copy()
            cp[fam, l] += h
            cm[fam, l] -= h
            idx.append((i, fam, l))
            cgrad.append((loss(i, cp, w.tau[i], w.omega[i]) - loss(i, cm, w.tau[i], w.omega[i])) / (2 * h))
    np.savez_compressed(os.path.join(HERE, "grad_sample.npz"), tau_grad=tau_grad, omega_grad=omega_grad,
                        coef_idx=np.array(idx), coef_grad=np.array(cgrad))


if __name__ == "__main__":
    main()
