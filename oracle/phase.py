"""Scattering matrix, geometric phase matrix and its azimuthal Fourier projection.

Scattering matrix in the scattering plane (randomly oriented mirror-symmetric particles; Sec. 2.A,
the phase matrix depends on the scattering angle only, eq. 5 read as cos(Theta)):

    F(Theta) = [[a1, b1, 0, 0], [b1, a2, 0, 0], [0, 0, a3, b2], [0, 0, -b2, a4]]

expanded in Wigner d-functions of x = cos(Theta):
a1 = sum alpha1_l d^l_00, a4 = sum alpha4_l d^l_00, a2 + a3 = sum (alpha2 + alpha3)_l d^l_22,
a2 - a3 = sum (alpha2 - alpha3)_l d^l_{2,-2}, b1 = -sum beta1_l d^l_02, b2 = -sum beta2_l d^l_02.

Geometric phase matrix Z(k <- k'). A direction (mu, phi) is the unit vector
k = (s cos phi, s sin phi, mu), s = sqrt(1 - mu^2), with its Stokes frame (e_theta, e_phi),
e_theta = (mu cos phi, mu sin phi, -s), e_phi = (-sin phi, cos phi, 0). Q = |E1|^2 - |E2|^2 and
U = 2 Re(E1 E2*) are referred to that frame. With n the unit normal k' x k of the scattering plane,
the scattering-plane frames are (n x k', n) and (n x k, n), and

    Z = L(psi_out) F(Theta) L(psi_in),  L(psi) = [[1,0,0,0],[0,c2,s2,0],[0,-s2,c2,0],[0,0,0,1]]

with c2 = cos 2psi, s2 = sin 2psi, psi_in the angle from e_theta' to n x k' (towards e_phi') and
psi_out the angle from n x k to e_theta (towards n).

Fourier projection (the eq. 6 structure): with Delta = phi - phi',
Z = sum_m c_m [A^m cos(m Delta) on the IQ-IQ and UV-UV blocks, +A^m sin(m Delta) on the UV<-IQ
block, -A^m sin(m Delta) on the IQ<-UV block], c_m = 2 - delta_m0. Under this reading of eq. 6
(the argument is outgoing minus incoming azimuth) the per-order operator of eq. 13 is exactly A^m
for the Stokes series of eq. 12.
"""

import numpy as np

from .legendre import wigner_d_seq


def scattering_matrix(coef: np.ndarray, x) -> np.ndarray:
    """F(Theta) at x = cos(Theta), shape x.shape + (4, 4)."""
    coef = np.asarray(coef, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    L = coef.shape[1]
    d00 = wigner_d_seq(L, 0, 0, x)
    d22 = wigner_d_seq(L, 2, 2, x)
    d2m = wigner_d_seq(L, 2, -2, x)
    d02 = wigner_d_seq(L, 0, 2, x)
    a1 = np.tensordot(coef[0], d00, 1)
    a4 = np.tensordot(coef[3], d00, 1)
    apl = np.tensordot(coef[1] + coef[2], d22, 1)
    ami = np.tensordot(coef[1] - coef[2], d2m, 1)
    b1 = -np.tensordot(coef[4], d02, 1)
    b2 = -np.tensordot(coef[5], d02, 1)
    a2 = 0.5 * (apl + ami)
    a3 = 0.5 * (apl - ami)
    F = np.zeros(x.shape + (4, 4))
    F[..., 0, 0] = a1
    F[..., 0, 1] = b1
    F[..., 1, 0] = b1
    F[..., 1, 1] = a2
    F[..., 2, 2] = a3
    F[..., 2, 3] = b2
    F[..., 3, 2] = -b2
    F[..., 3, 3] = a4
    return F


def _rot(psi_c, psi_s):
    """L(psi) from cos(psi), sin(psi) arrays."""
    c2 = psi_c * psi_c - psi_s * psi_s
    s2 = 2.0 * psi_s * psi_c
    out = np.zeros(np.shape(psi_c) + (4, 4))
    out[..., 0, 0] = 1.0
    out[..., 3, 3] = 1.0
    out[..., 1, 1] = c2
    out[..., 2, 2] = c2
    out[..., 1, 2] = s2
    out[..., 2, 1] = -s2
    return out


def _frame(mu, phi):
    mu = np.asarray(mu, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    s = np.sqrt(np.clip(1.0 - mu * mu, 0.0, None))
    cp, sp = np.cos(phi), np.sin(phi)
    k = np.stack([s * cp, s * sp, mu * np.ones_like(cp)], -1)
    et = np.stack([mu * cp, mu * sp, -s * np.ones_like(cp)], -1)
    ep = np.stack([-sp, cp, np.zeros_like(cp)], -1)
    return k, et, ep


def phase_matrix(coef, mu, phi, mu_in, phi_in) -> np.ndarray:
    """Z(mu, phi <- mu_in, phi_in), broadcasting over the four arguments.

    The scattering plane must be defined (k and k' not collinear).
    """
    mu, phi, mu_in, phi_in = np.broadcast_arrays(*[np.asarray(a, dtype=np.float64) for a in (mu, phi, mu_in, phi_in)])
    k, et, _ = _frame(mu, phi)
    k1, et1, ep1 = _frame(mu_in, phi_in)
    cos_t = np.clip(np.sum(k * k1, -1), -1.0, 1.0)
    nrm = np.cross(k1, k)
    nn = np.linalg.norm(nrm, axis=-1)
    if np.any(nn < 1e-12):
        raise ValueError("scattering plane undefined (collinear directions)")
    nrm = nrm / nn[..., None]
    par_in = np.cross(nrm, k1)
    par_out = np.cross(nrm, k)
    L_in = _rot(np.sum(par_in * et1, -1), np.sum(par_in * ep1, -1))
    L_out = _rot(np.sum(et * par_out, -1), np.sum(et * nrm, -1))
    F = scattering_matrix(coef, cos_t)
    return L_out @ F @ L_in


IQ = np.array([True, True, False, False])
UV = ~IQ


def projected_fourier_matrix(coef, m: int, mu_out, mu_in, n_az: int = None) -> np.ndarray:
    """A^m(mu, mu') by direct azimuthal Fourier projection of the geometric phase matrix.

    Uses n_az half-step-shifted azimuths Delta_k = 2 pi (k + 1/2) / n_az (so that Theta is never 0
    or pi), which integrates trigonometric polynomials of degree < n_az - m exactly. Shape
    (len(mu_out), len(mu_in), 4, 4).
    """
    coef = np.asarray(coef, dtype=np.float64)
    L = coef.shape[1]
    if n_az is None:
        n_az = 2 * L + 4
    delta = 2.0 * np.pi * (np.arange(n_az) + 0.5) / n_az
    mo = np.asarray(mu_out, dtype=np.float64)[:, None, None]
    mi = np.asarray(mu_in, dtype=np.float64)[None, :, None]
    Z = phase_matrix(coef, mo, delta[None, None, :], mi, 0.0)  # (no, ni, naz, 4, 4)
    c = np.cos(m * delta) / n_az
    s = np.sin(m * delta) / n_az
    Zc = np.einsum("ijkab,k->ijab", Z, c)
    Zs = np.einsum("ijkab,k->ijab", Z, s)
    A = np.zeros_like(Zc)
    same = np.outer(IQ, IQ) | np.outer(UV, UV)
    A[..., same] = Zc[..., same]
    A[..., np.outer(UV, IQ)] = Zs[..., np.outer(UV, IQ)]
    A[..., np.outer(IQ, UV)] = -Zs[..., np.outer(IQ, UV)]
    return A
