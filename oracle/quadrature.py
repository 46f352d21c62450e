"""Double-Gauss quadrature on each hemisphere (Sec. 2.B, eq. 15).

N-point Gauss-Legendre on [0, 1]: mu_i = (1 + x_i) / 2 and alpha_i = w_i / 2 with (x_i, w_i) the
rule on [-1, 1]. Nodes are positive and ascending; sum(alpha) = 1. The angular integral over
[-1, 1] is sum_i alpha_i [f(mu_i) + f(-mu_i)].
"""

import numpy as np


def double_gauss(N: int):
    if N < 1:
        raise ValueError("N must be >= 1")
    x, w = np.polynomial.legendre.leggauss(N)
    return (1.0 + x) / 2.0, w / 2.0
