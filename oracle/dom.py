"""Per-order discrete-ordinate solution and synthesis of the BRDF Mueller matrix.

Conventions (readings of the paper, each pinned by a test):
  * tau grows downward from the top (0) to the base (tau0); mu > 0 propagates downward, so eq. 2
    holds as printed and the beam attenuates as exp(-tau/mu0) (eq. 4). Reflected light is
    I(0, -mu). The boundary section's labels are the mirror image and are read this way.
  * Stokes series of eq. 12 with Phi_k^m(phi - phi0) and the factor 1/2; phase-matrix series of
    eq. 6 with outgoing-minus-incoming azimuth. The per-order equation is eq. 13 with the operator
    A^m of eq. 9 and source (omega / 2pi) A^m(mu, mu0) D_k I0 exp(-tau/mu0).
  * In eq. 15 order the 8N unknowns are [I(+mu_1..N); I(-mu_1..N)], each a Stokes 4-vector; the
    scattering matrix carries the weights on the right (script-A W), with A(mu_i, -mu_j) in the
    upper-right block.
  * Incidence on Gauss node mu_q is carried as a discrete stream (the "stream form"): the total
    discrete field solves the homogeneous system with I(0, +mu_i) = delta_iq I0 / (pi alpha_q) and
    I(tau0, -mu_i) = 0 (black base). Its quadrature-weighted scattering equals the source of eq. 14
    exactly, so the reflected field equals the particular-plus-homogeneous solution of eq. 28-33
    whenever the latter exists.
  * F_r is defined with the horizontal irradiance E = mu0 I0 (eq. 1) and obtained from the four
    unit Stokes inputs (eq. 39).
  * The albedo is clamped to at most 1 - 1e-12 (at omega = 1 the m = 0 spectrum has a double zero).
"""

import numpy as np
import scipy.linalg as sla

from .legendre import phase_fourier_matrix
from .quadrature import double_gauss

OMEGA_MAX = 1.0 - 1e-12

IQ = np.array([True, True, False, False])


def validate(coef, tau0, omega, N, M):
    coef = np.asarray(coef, dtype=np.float64)
    if coef.ndim != 2 or coef.shape[0] != 6:
        raise ValueError("coef must have shape (6, L)")
    L = coef.shape[1]
    if not (np.isfinite(tau0) and tau0 > 0):
        raise ValueError("tau0 must be finite and > 0")
    if not (np.isfinite(omega) and 0 < omega <= 1):
        raise ValueError("omega must lie in (0, 1]")
    if not np.all(np.isfinite(coef)):
        raise ValueError("coefficients must be finite")
    if abs(coef[0, 0] - 1.0) > 1e-12:
        raise ValueError("alpha1_0 must be 1")
    if N < 1 or M < 1 or M > L:
        raise ValueError("need N >= 1 and 1 <= M <= L")
    return coef, min(float(omega), OMEGA_MAX)


def full_phase_block(coef, m, mu):
    """The 8N x 8N matrix script-A of eq. 19-23 (rows: outgoing stream and Stokes index)."""
    N = len(mu)
    mus = np.concatenate([mu, -mu])
    A = phase_fourier_matrix(coef, m, mus, mus)  # (2N, 2N, 4, 4)
    return A.transpose(0, 2, 1, 3).reshape(8 * N, 8 * N)


def order_operator(coef, omega, m, mu, alpha):
    """K_m with dI/dtau = K_m I for the homogeneous per-order system (eq. 18-21).

    K_m = Mhat^-1 (omega/2 script-A W - I), Mhat = diag(mu_i I4, -mu_i I4), W = diag(alpha_i I4).
    """
    N = len(mu)
    Abig = full_phase_block(coef, m, mu)
    w = np.repeat(np.concatenate([alpha, alpha]), 4)
    mh = np.repeat(np.concatenate([mu, -mu]), 4)
    return (0.5 * omega * Abig * w[None, :] - np.eye(8 * N)) / mh[:, None]


def eigen_basis(K, tau0):
    """Eigen-decomposition of K (eq. 16-17) and the scaled basis of eq. 24-25.

    Decaying modes (Re kappa < 0) are anchored at the top, growing modes at the base, so every
    exponential has modulus <= 1. Returns (H0, H1): basis values at tau = 0 and tau = tau0.
    """
    kappa, V = np.linalg.eig(K)
    n = K.shape[0] // 2
    dec = kappa.real < 0
    if int(dec.sum()) != n:
        raise FloatingPointError("eigenvalues do not split into decaying/growing halves")
    s0 = np.exp(np.where(dec, 0.0, -kappa * tau0))
    s1 = np.exp(np.where(dec, kappa * tau0, 0.0))
    return V * s0[None, :], V * s1[None, :], kappa, V


def stream_rhs(alpha):
    """One column per (incident node q, Stokes p): value 1/(pi alpha_q) at downward row (q, p)."""
    return np.diag(np.repeat(1.0 / (np.pi * np.asarray(alpha)), 4))


def solve_order(coef, omega, tau0, m, mu, alpha, want_transmission=False, basis_hook=None):
    """Per-order emergent response R^m[(i, r), (q, p)] (and optionally the transmitted field).

    R^m is the Stokes component r of the upward radiance at the top on stream i for a unit Stokes
    vector e_p incident on node mu_q (order-m, k-type set by p). The transmitted field includes the
    attenuated incident stream.
    """
    N = len(mu)
    n = 4 * N
    K = order_operator(coef, omega, m, mu, alpha)
    H0, H1, kappa, V = eigen_basis(K, tau0)
    if basis_hook is not None:
        H0, H1 = basis_hook(H0, H1, kappa, V, tau0)
    # rows: downward components at the top, upward components at the base (eq. 49-56)
    Bc = np.vstack([H0[:n, :], H1[n:, :]])
    rhs = np.zeros((2 * n, n))
    rhs[:n, :] = stream_rhs(alpha)
    c = sla.lu_solve(sla.lu_factor(Bc), rhs)
    R = H0[n:, :] @ c
    scale = max(np.abs(R).max(), 1e-300)
    if np.abs(R.imag).max() > 1e-9 * scale + 1e-300:
        raise FloatingPointError("complex residue in the emergent radiance")
    if not want_transmission:
        return R.real
    T = H1[:n, :] @ c
    return R.real, T.real


def azimuth_factors(m, dphi):
    """tau_rp(m dphi) of the synthesis: cos on same-type blocks, +sin on UV<-IQ, -sin on IQ<-UV."""
    c = np.cos(m * dphi)
    s = np.sin(m * dphi)
    out = np.empty(dphi.shape + (4, 4))
    for r in range(4):
        for p in range(4):
            if IQ[r] == IQ[p]:
                out[..., r, p] = c
            elif IQ[p]:
                out[..., r, p] = s
            else:
                out[..., r, p] = -s
    return out


def synthesize(R_orders, mu_in, n_dphi):
    """F_r[i, q, k, r, p] = 1/(2 mu_q) sum_m c_m tau_rp(m dphi_k) R^m[(i, r), (q, p)] (eq. 12, 39).

    R_orders: sequence of (4 N_out, 4 N_in) arrays, m = 0..M-1. dphi_k = 2 pi k / n_dphi.
    """
    mu_in = np.asarray(mu_in, dtype=np.float64)
    n_out = R_orders[0].shape[0] // 4
    n_in = R_orders[0].shape[1] // 4
    dphi = 2.0 * np.pi * np.arange(n_dphi) / n_dphi
    F = np.zeros((n_out, n_in, n_dphi, 4, 4))
    for m, R in enumerate(R_orders):
        cm = 1.0 if m == 0 else 2.0
        Rb = R.reshape(n_out, 4, n_in, 4).transpose(0, 2, 1, 3)  # (i, q, r, p)
        F += cm * azimuth_factors(m, dphi)[None, None] * Rb[:, :, None, :, :]
    return F / (2.0 * mu_in[None, :, None, None, None])


def brdf(coef, tau0, omega, N, M, n_dphi, return_orders=False):
    """Polarized subsurface BRDF F_r[i, q, k, r, p] of one layer on the double-Gauss node grid.

    i: outgoing node (reflected direction -mu_i), q: incident node mu_q, k: dphi_k = 2 pi k/n_dphi,
    (r, p): Mueller row/column over (I, Q, U, V).
    """
    coef, om = validate(coef, tau0, omega, N, M)
    mu, alpha = double_gauss(N)
    R = [solve_order(coef, om, tau0, m, mu, alpha) for m in range(M)]
    F = synthesize(R, mu, n_dphi)
    return (F, R) if return_orders else F
