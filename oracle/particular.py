"""Incidence off the quadrature nodes through the particular solution (Sec. 2.C.2, eq. 28-33).

For a collimated beam along (mu0, phi0), the order-m source is X exp(-tau/mu0) with
X(+-mu_i) = (omega / 2pi) A^m(+-mu_i, mu0) e_p for unit Stokes input e_p. The particular solution
Z exp(-tau/mu0) solves (-Mhat/mu0 + I - omega/2 script-A W) Z = X (eq. 33, weights on the right).
The homogeneous part is fixed by zero incoming diffuse light at the top and at the black base.
"""

import numpy as np
import scipy.linalg as sla

from .dom import eigen_basis, full_phase_block, order_operator, validate
from .legendre import phase_fourier_matrix
from .quadrature import double_gauss


def solve_order_beam(coef, omega, tau0, m, mu, alpha, mu0):
    """Reflected diffuse response R^m[(i, r), p] (shape (4N, 4)) to a unit Stokes beam at mu0."""
    N = len(mu)
    n = 4 * N
    K = order_operator(coef, omega, m, mu, alpha)
    H0, H1, _, _ = eigen_basis(K, tau0)
    mus = np.concatenate([mu, -mu])
    A0 = phase_fourier_matrix(coef, m, mus, np.array([mu0]))[:, 0]  # (2N, 4, 4)
    X = (omega / (2.0 * np.pi)) * A0.reshape(2 * n, 4)  # column p = A e_p
    w = np.repeat(np.concatenate([alpha, alpha]), 4)
    mh = np.repeat(np.concatenate([mu, -mu]), 4)
    Abig = full_phase_block(coef, m, mu)
    P = -np.diag(mh) / mu0 + np.eye(2 * n) - 0.5 * omega * Abig * w[None, :]
    Z = np.linalg.solve(P, X)
    Bc = np.vstack([H0[:n, :], H1[n:, :]])
    rhs = -np.vstack([Z[:n, :], Z[n:, :] * np.exp(-tau0 / mu0)])
    c = sla.lu_solve(sla.lu_factor(Bc), rhs)
    R = H0[n:, :] @ c + Z[n:, :]
    return R.real


def brdf_beam(coef, tau0, omega, N, M, n_dphi, mu0):
    """F_r[i, k, r, p] for incidence at an arbitrary mu0 (outgoing on the Gauss nodes)."""
    from .dom import synthesize

    coef, om = validate(coef, tau0, omega, N, M)
    mu, alpha = double_gauss(N)
    R = [solve_order_beam(coef, om, tau0, m, mu, alpha, mu0) for m in range(M)]
    return synthesize(R, np.array([mu0]), n_dphi)[:, 0]
