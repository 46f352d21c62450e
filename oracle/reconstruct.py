"""Radiance towards arbitrary outgoing directions by source-function integration (Sec. 2.C
"Reconstruction", eq. 36-38).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The per-order discrete-ordinate solution is a sum of exponentials in depth: the eigen modes of
eq. 16-25 (anchored so that every exponential is at most 1) plus, for a beam, the particular
solution Z exp(-t/mu0) of eq. 28-30. The source of eq. 38,
    S(t, mu) = omega/2 sum_j alpha_j A^m(mu, mu_j) I(t, mu_j) + X(mu) exp(-t/mu0),
(the sum over both hemispheres' nodes) is then a sum of the same exponentials, and the formal
solution along the upward direction -mu (tau downward, reading 1 of the geometry; black base) is
    I(0, -mu) = int_0^tau0 S(t, -mu) exp(-t/mu) dt / mu,
which is eq. 37 with the factor 1/mu that its printed form lacks. Each exponential integrates in
closed form. At a Gauss node the result is the discrete-ordinate value itself.
"""

import numpy as np
import scipy.linalg as sla

from .dom import eigen_basis, full_phase_block, order_operator, stream_rhs, synthesize, validate
from .legendre import phase_fourier_matrix
from .quadrature import double_gauss


def _expint(rate, tau0, mu):
    """int_0^tau0 exp(rate t) exp(-t/mu) dt / mu for complex rates with Re(rate) <= 0 (the limit
    where rate and 1/mu cancel)."""
    a = rate - 1.0 / mu
    small = np.abs(a * tau0) < 1e-8
    safe = np.where(small, 1.0, a)
    val = np.expm1(np.where(small, 0.0, a) * tau0) / (mu * safe)
    return np.where(small, tau0 / mu * (1.0 + 0.5 * a * tau0), val)


def _expint_base(rate, tau0, mu):
    """int_0^tau0 exp(rate (t - tau0)) exp(-t/mu) dt / mu for Re(rate) > 0 (a mode anchored at the
    base): (exp(-tau0/mu) - exp(-rate tau0)) / (mu (rate - 1/mu)), both exponentials at most 1."""
    a = rate - 1.0 / mu
    small = np.abs(a * tau0) < 1e-8
    safe = np.where(small, 1.0, a)
    val = (np.exp(-tau0 / mu) - np.exp(-rate * tau0)) / (mu * safe)
    return np.where(small, tau0 / mu * np.exp(-tau0 / mu) * (1.0 - 0.5 * a * tau0), val)


def _field_coefficients(coef, omega, tau0, m, mu, alpha, mu0):
    """Eigen basis, anchoring and mode coefficients of the per-order solution.

    mu0 None: the stream inputs of every node (4N columns); otherwise a unit Stokes beam at mu0
    (4 columns) with its particular solution Z."""
    N = len(mu)
    n = 4 * N
    K = order_operator(coef, omega, m, mu, alpha)
    H0, H1, kappa, V = eigen_basis(K, tau0)
    Bc = np.vstack([H0[:n, :], H1[n:, :]])
    if mu0 is None:
        rhs = np.zeros((2 * n, n))
        rhs[:n, :] = stream_rhs(alpha)
        Z = None
    else:
        mus = np.concatenate([mu, -mu])
        A0 = phase_fourier_matrix(coef, m, mus, np.array([mu0]))[:, 0]
        X = (omega / (2.0 * np.pi)) * A0.reshape(2 * n, 4)
        w = np.repeat(np.concatenate([alpha, alpha]), 4)
        mh = np.repeat(np.concatenate([mu, -mu]), 4)
        Abig = full_phase_block(coef, m, mu)
        P = -np.diag(mh) / mu0 + np.eye(2 * n) - 0.5 * omega * Abig * w[None, :]
        Z = np.linalg.solve(P, X)
        rhs = -np.vstack([Z[:n, :], Z[n:, :] * np.exp(-tau0 / mu0)])
    c = sla.lu_solve(sla.lu_factor(Bc), rhs)
    return kappa, V, c, Z


def solve_order_outgoing(coef, omega, tau0, m, mu, alpha, mu_out, mu0=None):
    """Upward radiance at the top towards -mu_out (each in (0, 1]) per unit input: shape
    (4 len(mu_out), 4N) for the stream inputs of the nodes, or (4 len(mu_out), 4) for a beam at mu0."""
    N = len(mu)
    n = 4 * N
    kappa, V, c, Z = _field_coefficients(coef, omega, tau0, m, mu, alpha, mu0)
    dec = kappa.real < 0
    mus = np.concatenate([mu, -mu])
    w = np.repeat(np.concatenate([alpha, alpha]), 4)
    out = []
    for mo in np.atleast_1d(mu_out):
        # source rows: omega/2 sum_j alpha_j A^m(-mo, mu_j) (both hemispheres)
        Ao = phase_fourier_matrix(coef, m, np.array([-mo]), mus)[0]  # (2N, 4, 4): [j, r, p]
        rows = 0.5 * omega * Ao.transpose(1, 0, 2).reshape(4, 2 * n) * w[None, :]
        # mode k at depth t: V_k exp(kappa_k t) (decaying, anchored at the top) or
        # V_k exp(kappa_k (t - tau0)) (growing, anchored at the base)
        f = np.where(dec, _expint(np.where(dec, kappa, 0.0), tau0, mo),
                     _expint_base(np.where(dec, 1.0, kappa), tau0, mo))
        R = (rows @ V) @ (f[:, None] * c)
        if Z is not None:
            Xo = (omega / (2.0 * np.pi)) * phase_fourier_matrix(coef, m, np.array([-mo]), np.array([mu0]))[0, 0]
            R = R + (rows @ Z + Xo) * _expint(np.array([-1.0 / mu0]), tau0, mo)[0]
        if np.abs(R.imag).max() > 1e-9 * max(np.abs(R).max(), 1e-300):
            raise FloatingPointError("complex residue in the reconstructed radiance")
        out.append(R.real)
    return np.vstack(out)


def brdf_beam_outgoing(coef, tau0, omega, N, M, n_dphi, mu0, mu_out):
    """F_r[o, k, r, p] for incidence at mu0 and reflection towards -mu_out[o] (both arbitrary)."""
    coef, om = validate(coef, tau0, omega, N, M)
    mu, alpha = double_gauss(N)
    R = [solve_order_outgoing(coef, om, tau0, m, mu, alpha, mu_out, mu0) for m in range(M)]
    return synthesize(R, np.array([mu0]), n_dphi)[:, 0]
