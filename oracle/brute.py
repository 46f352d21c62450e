"""Eigenvector-free reference for tiny N: the per-order propagator at extended precision.

The homogeneous per-order system dI/dtau = K_m I (eq. 18-21) is integrated across the layer with the
matrix exponential Psi = expm(K_m tau0) in mpmath. Splitting the 8N unknowns into downward (+) and
upward (-) streams, a black base gives I-(tau0) = 0, hence the upward field at the top is
I-(0) = -Psi_{--}^{-1} Psi_{-+} I+(0). No eigen-decomposition, no boundary-matrix assembly and no
Legendre recurrence is used: the phase-matrix Fourier coefficients come from the direct azimuthal
projection of the geometric phase matrix.
"""

import mpmath as mp
import numpy as np

from .phase import projected_fourier_matrix
from .quadrature import double_gauss


def _operator_mp(coef, omega, m, mu, alpha):
    N = len(mu)
    mus = np.concatenate([mu, -mu])
    A = projected_fourier_matrix(coef, m, mus, mus).transpose(0, 2, 1, 3).reshape(8 * N, 8 * N)
    w = np.repeat(np.concatenate([alpha, alpha]), 4)
    mh = np.repeat(np.concatenate([mu, -mu]), 4)
    K = mp.matrix(8 * N, 8 * N)
    for a in range(8 * N):
        for b in range(8 * N):
            v = mp.mpf(0.5) * mp.mpf(omega) * mp.mpf(A[a, b]) * mp.mpf(w[b])
            if a == b:
                v -= 1
            K[a, b] = v / mp.mpf(mh[a])
    return K, A, mh


def _nodes(N, extra):
    """Gauss nodes followed by extra directions of zero weight: an extra direction is carried
    through the layer by its own transport equation but adds nothing to the scattering integral,
    so its upward radiance at the top is the exact formal solution towards it."""
    mu, alpha = double_gauss(N)
    extra = np.asarray(extra, dtype=float).reshape(-1)
    return np.concatenate([mu, extra]), np.concatenate([alpha, np.zeros(len(extra))])


def stream_response(coef, omega, tau0, m, N, dps=40, extra=()):
    """R^m for unit Stokes inputs on each node (stream form), computed through expm.

    Rows: the 4N node rows followed by 4 rows per extra outgoing direction; columns: the 4N node
    inputs."""
    mu, alpha = _nodes(N, extra)
    n = 4 * len(mu)
    with mp.workdps(dps):
        K, _, _ = _operator_mp(coef, omega, m, mu, alpha)
        Psi = mp.expm(K * mp.mpf(tau0))
        Pmm = Psi[n:, n:]
        Pmp = Psi[n:, :n]
        Rop = -(mp.inverse(Pmm) * Pmp)
        out = np.zeros((n, 4 * N))
        for a in range(n):
            for b in range(4 * N):
                out[a, b] = float(Rop[a, b] / (mp.pi * mp.mpf(alpha[b // 4])))
    return out


def beam_response(coef, omega, tau0, m, N, mu0, dps=40, extra=()):
    """Reflected diffuse response (4N x 4, then 4 rows per extra outgoing direction) to a unit
    Stokes beam at an off-node mu0.

    The beam enters as the extra state s(tau) = exp(-tau/mu0) of the augmented system
    [[K, Mhat^-1 X], [0, -1/mu0]], X = (omega/2pi) A^m(+-mu_i, mu0) e_p.
    """
    mu, alpha = _nodes(N, extra)
    n = 4 * len(mu)
    mus = np.concatenate([mu, -mu])
    A0 = projected_fourier_matrix(coef, m, mus, np.array([mu0]))[:, 0].reshape(2 * n, 4)
    out = np.zeros((n, 4))
    with mp.workdps(dps):
        K, _, mh = _operator_mp(coef, omega, m, mu, alpha)
        for p in range(4):
            Ka = mp.matrix(2 * n + 1, 2 * n + 1)
            for a in range(2 * n):
                for b in range(2 * n):
                    Ka[a, b] = K[a, b]
                Ka[a, 2 * n] = mp.mpf(omega) / (2 * mp.pi) * mp.mpf(A0[a, p]) / mp.mpf(mh[a])
            Ka[2 * n, 2 * n] = -1 / mp.mpf(mu0)
            Psi = mp.expm(Ka * mp.mpf(tau0))
            Pmm = Psi[n:2 * n, n:2 * n]
            Pms = Psi[n:2 * n, 2 * n]
            x = -(mp.inverse(Pmm) * Pms)
            for a in range(n):
                out[a, p] = float(x[a])
    return out


def stack_stream_response(layers, m, N, Xb=None, dps=40):
    """R^m at the top of a stack (stream form) through the product of the layers' propagators.

    layers: [(coef, omega, tau0), ...] from the top down. Xb: the base as a matrix on the downward
    radiance at the base (upward = Xb downward), or None for a black base. With
    Psi = expm(K_last tau_last) ... expm(K_first tau_first) the field at the base is Psi times the
    field at the top, so with the downward field at the top given the base condition reads
    (Psi_{--} - Xb Psi_{+-}) I-(0) = (Xb Psi_{++} - Psi_{-+}) I+(0).
    """
    mu, alpha = double_gauss(N)
    n = 4 * N
    with mp.workdps(dps):
        Psi = mp.eye(2 * n)
        for coef, omega, tau0 in layers:
            K, _, _ = _operator_mp(coef, omega, m, mu, alpha)
            Psi = mp.expm(K * mp.mpf(tau0)) * Psi
        X = mp.zeros(n, n)
        if Xb is not None:
            for a in range(n):
                for b in range(n):
                    X[a, b] = mp.mpf(float(Xb[a, b]))
        Ppp, Ppm = Psi[:n, :n], Psi[:n, n:]
        Pmp, Pmm = Psi[n:, :n], Psi[n:, n:]
        Rop = mp.inverse(Pmm - X * Ppm) * (X * Ppp - Pmp)
        out = np.zeros((n, n))
        for a in range(n):
            for b in range(n):
                out[a, b] = float(Rop[a, b] / (mp.pi * mp.mpf(alpha[b // 4])))
    return out
