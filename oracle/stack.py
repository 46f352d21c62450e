"""Layer stacks and reflecting bases for the per-order discrete-ordinate solution.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.C closes the per-order system with two boundary conditions: no diffuse light enters at the
top, and at the base the upward field is the base's reflection of the downward field (the base
BRDF integral of Sec. 2.C). Sec. 3.C ("Base Reflection", eq. 57-66) discretises that integral
with the quadrature of eq. 15 and moves the homogeneous part to the left of the boundary system.
For several layers Sec. 2.C gives each layer its own homogeneous solution (8N more coefficients
per layer) and requires the radiance to be continuous across every interface.

This module writes exactly that out: one full 8N eigen basis per layer (dom.eigen_basis), and one
dense system for the coefficients of all layers whose rows are
  * the top condition: the downward field at tau = 0 is the incident streams (stream form),
  * 8N continuity rows per interface: the whole field at the bottom of layer k equals the whole
    field at the top of layer k + 1,
  * the base condition (eq. 58 in quadrature form):
        I_up(base, mu_i) = sum_j alpha_j mu_j R_b^m(mu_i, mu_j) I_down(base, mu_j).
In stream form the attenuated incident stream is part of the downward field at the base, so the
beam term of eq. 58 is the j = q term of this same sum; its normalisation is fixed by the
Lambertian limit (a vanishing layer over a Lambertian base has F_r = rho / pi).

R_b^m is a per-order 4x4 block per node pair, in the same per-order representation as the phase
matrix Fourier components (cos part on the IQ-IQ and UV-UV blocks, sin part on the cross blocks):
Rb[i, j, r, p] is Stokes component r of the upward radiance on node i per unit component p of the
downward radiance on node j, Stokes vectors in the frames of the rest of the oracle.
"""

import numpy as np
import scipy.linalg as sla

from .dom import eigen_basis, order_operator, stream_rhs, synthesize, validate
from .quadrature import double_gauss


def lambertian_base(rho, m, N):
    """Rb of the ideal depolarising Lambertian base (eq. 66): R_00 = 2 rho, nothing else, and only
    in order 0 (a Lambertian reflector does not depend on azimuth)."""
    Rb = np.zeros((N, N, 4, 4))
    if m == 0:
        Rb[:, :, 0, 0] = 2.0 * rho
    return Rb


def base_operator(Rb, mu, alpha):
    """X_b[(i, r), (j, p)] = alpha_j mu_j Rb[i, j, r, p]: the quadrature sum of eq. 58 as a matrix
    acting on the downward radiance at the base."""
    N = len(mu)
    w = np.asarray(alpha) * np.asarray(mu)
    return (Rb * w[None, :, None, None]).transpose(0, 2, 1, 3).reshape(4 * N, 4 * N)


def solve_order_stack(layers, m, mu, alpha, Rb=None):
    """R^m[(i, r), (q, p)] at the top of a stack (stream form, as dom.solve_order).

    layers: [(coef, omega, tau0), ...] from the top down (omega already clamped); Rb: the base's
    (N, N, 4, 4) blocks for order m, or None for a black base.
    """
    N = len(mu)
    n = 4 * N
    K = len(layers)
    bases = []
    for coef, om, tau0 in layers:
        H0, H1, _, _ = eigen_basis(order_operator(coef, om, m, mu, alpha), tau0)
        bases.append((H0, H1))
    A = np.zeros((2 * n * K, 2 * n * K), dtype=complex)
    rhs = np.zeros((2 * n * K, n))
    # top: downward field of layer 0 at its top = incident streams
    A[:n, :2 * n] = bases[0][0][:n, :]
    rhs[:n, :] = stream_rhs(alpha)
    # interfaces: field at the bottom of layer k = field at the top of layer k + 1
    for k in range(K - 1):
        r0 = n + 2 * n * k
        A[r0:r0 + 2 * n, 2 * n * k:2 * n * (k + 1)] = bases[k][1]
        A[r0:r0 + 2 * n, 2 * n * (k + 1):2 * n * (k + 2)] = -bases[k + 1][0]
    # base: upward field at the bottom of the last layer = X_b (downward field there)
    H1 = bases[-1][1]
    last = H1[n:, :].astype(complex)
    if Rb is not None:
        last = last - base_operator(Rb, mu, alpha) @ H1[:n, :]
    A[2 * n * K - n:, 2 * n * (K - 1):] = last
    c = sla.lu_solve(sla.lu_factor(A), rhs)
    R = bases[0][0][n:, :] @ c[:2 * n, :]
    scale = max(np.abs(R).max(), 1e-300)
    if np.abs(R.imag).max() > 1e-9 * scale + 1e-300:
        raise FloatingPointError("complex residue in the emergent radiance")
    return R.real


def brdf_stack(layers, N, M, n_dphi, base=None, rho=0.0, Rb_orders=None, return_orders=False):
    """F_r[i, q, k, r, p] at the top of a stack of layers [(coef, tau0, omega), ...] (top first).

    base: None (black), "lambertian" (albedo rho) or "mueller" (Rb_orders[m] of shape (N, N, 4, 4)
    for m = 0..M-1).
    """
    mu, alpha = double_gauss(N)
    ls = []
    for coef, tau0, omega in layers:
        c, om = validate(coef, tau0, omega, N, M)
        ls.append((c, om, float(tau0)))
    R = []
    for m in range(M):
        if base is None:
            Rb = None
        elif base == "lambertian":
            Rb = lambertian_base(rho, m, N)
        elif base == "mueller":
            Rb = np.asarray(Rb_orders[m], dtype=np.float64)
        else:
            raise ValueError("base must be None, 'lambertian' or 'mueller'")
        R.append(solve_order_stack(ls, m, mu, alpha, Rb))
    F = synthesize(R, mu, n_dphi)
    return (F, R) if return_orders else F
