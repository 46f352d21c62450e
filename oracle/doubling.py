"""Eigenvector-free reference at any N: adding-doubling of the per-order homogeneous system.

The semi-discrete per-order equation dI/dtau = K_m I (eq. 18-21) is integrated over a thin slice
dtau = tau0 / 2^k with the matrix exponential (well conditioned because dtau * ||K_m|| <= 1/2).
The slice propagator Psi, split into downward (+) and upward (-) streams, gives the slice's
reflection and transmission operators (zero incoming light on the far face):
    R_top = -Psi_{--}^-1 Psi_{-+},  T_up = Psi_{--}^-1,
    T_down = Psi_{++} - Psi_{+-} Psi_{--}^-1 Psi_{-+},  R_bot = Psi_{+-} Psi_{--}^-1.
Two identical slices are combined by the interaction principle (multiple reflections between
them summed by (I - R R)^-1) and the doubling is repeated k times. The reflected radiance at the
top for stream-form incidence on node q is R_top diag(1/(pi alpha_q)).
This route shares only the operator K_m with the eigen-based solver.
"""

import numpy as np
from scipy.linalg import expm

from .dom import order_operator, stream_rhs


def slab_operators(K, tau0, max_step=0.5):
    n2 = K.shape[0]
    n = n2 // 2
    norm = np.abs(K).sum(axis=1).max()
    k = max(0, int(np.ceil(np.log2(max(tau0 * norm / max_step, 1.0)))))
    d = tau0 / 2 ** k
    Psi = expm(K * d)
    Ppp, Ppm, Pmp, Pmm = Psi[:n, :n], Psi[:n, n:], Psi[n:, :n], Psi[n:, n:]
    Pinv = np.linalg.inv(Pmm)
    Rt = -Pinv @ Pmp
    Tu = Pinv
    Td = Ppp + Ppm @ Rt
    Rb = Ppm @ Pinv
    I = np.eye(n)
    for _ in range(k):
        A1 = np.linalg.solve(I - Rb @ Rt, Td)          # (I - Rb_A Rt_B)^-1 Td_A
        A2 = np.linalg.solve(I - Rt @ Rb, Tu)          # (I - Rt_B Rb_A)^-1 Tu_B
        Rt, Td, Rb, Tu = Rt + Tu @ Rt @ A1, Td @ A1, Rb + Td @ Rb @ A2, Tu @ A2
    return Rt, Td, Rb, Tu


def solve_order(coef, omega, tau0, m, mu, alpha):
    """R^m (stream form, same layout as dom.solve_order) without eigenvectors."""
    K = order_operator(coef, omega, m, mu, alpha)
    Rt = slab_operators(K, tau0)[0]
    return Rt @ stream_rhs(alpha)
