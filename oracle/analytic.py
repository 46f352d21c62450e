"""Closed-form limits used to pin the oracle.

single_scattering: first-order reflection of a thin layer over a black base, straight from the
radiative transfer equation (eq. 2-4) with the geometric phase matrix (no Fourier series):
    F_ss = omega/(4 pi) Z(-mu, phi <- mu0, phi0) (1 - exp(-tau0 (1/mu + 1/mu0))) / (mu + mu0).

chandrasekhar_h: for isotropic scattering (alpha1 = [1], everything else 0) over a semi-infinite
medium, the discrete-ordinate emergent intensity is given by Chandrasekhar's N-th approximation
    H(mu) = prod_i (mu + mu_i) / (prod_i mu_i * prod_a (1 + k_a mu)),
with k_a the N positive roots of 1 = omega sum_j alpha_j / (1 - k^2 mu_j^2), and
    F_11(mu <- mu0) = omega/(4 pi) H(mu) H(mu0) / (mu + mu0).
"""

import numpy as np
from scipy.optimize import brentq

from .phase import phase_matrix


def single_scattering(coef, omega, tau0, mu_out, mu_in, dphi):
    """F_ss[i, q, k, 4, 4] for outgoing -mu_out[i], incident mu_in[q], azimuth difference dphi[k]."""
    mo = np.asarray(mu_out, dtype=np.float64)[:, None, None]
    mi = np.asarray(mu_in, dtype=np.float64)[None, :, None]
    dp = np.asarray(dphi, dtype=np.float64)[None, None, :]
    Z = phase_matrix(coef, -mo, dp, mi, 0.0)
    fac = omega / (4 * np.pi) * (-np.expm1(-tau0 * (1.0 / mo + 1.0 / mi))) / (mo + mi)
    return Z * fac[..., None, None]


def characteristic_roots(omega, mu, alpha):
    """Positive roots k_a of 1 = omega sum_j alpha_j / (1 - k^2 mu_j^2), ascending."""
    mu = np.asarray(mu, dtype=np.float64)
    alpha = np.asarray(alpha, dtype=np.float64)

    def f(k2):
        return omega * np.sum(alpha / (1.0 - k2 * mu * mu)) - 1.0

    poles = np.sort(1.0 / (mu * mu))
    roots = []
    lo = 0.0
    for p in poles:
        eps = 1e-13 * p
        a = lo + (eps if lo > 0 else 0.0)
        roots.append(brentq(f, a, p - eps, xtol=1e-300, rtol=1e-15, maxiter=500))
        lo = p
    return np.sqrt(np.array(roots))


def chandrasekhar_h(omega, mu_nodes, alpha, mu_eval):
    k = characteristic_roots(omega, mu_nodes, alpha)
    mu_eval = np.asarray(mu_eval, dtype=np.float64)
    num = np.prod(mu_eval[:, None] + np.asarray(mu_nodes)[None, :], axis=1)
    den = np.prod(mu_nodes) * np.prod(1.0 + k[None, :] * mu_eval[:, None], axis=1)
    return num / den
