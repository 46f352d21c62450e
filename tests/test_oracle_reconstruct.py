"""Pins of the source-function-integration oracle (oracle/reconstruct.py, Sec. 2.C "Reconstruction",
eq. 36-38): at the Gauss nodes it must return the discrete-ordinate values themselves (stream and
beam inputs), and at small albedo it must approach single scattering at arbitrary angle pairs with
a remainder of second order in omega (the closed-form single-scattering BRDF shares no code with it)."""

import numpy as np
import pytest

from oracle import analytic, dom, particular, reconstruct
from oracle.quadrature import double_gauss
from workloads.layers import hg_like_coefficients


def hg(seed, L):
    return hg_like_coefficients(np.random.default_rng(seed), L)[0]


@pytest.mark.parametrize("m", [0, 1, 3])
def test_reconstruction_at_the_nodes_is_the_dom_value(m):
    N, tau, om = 6, 1.7, 0.93
    coef = hg(3, 10)
    mu, al = double_gauss(N)
    Ro = dom.solve_order(coef, om, tau, m, mu, al)
    Rr = reconstruct.solve_order_outgoing(coef, om, tau, m, mu, al, mu)
    assert np.abs(Rr - Ro).max() < 1e-12 * np.abs(Ro).max()
    Rb = particular.solve_order_beam(coef, om, tau, m, mu, al, 0.3137)
    Rrb = reconstruct.solve_order_outgoing(coef, om, tau, m, mu, al, mu, 0.3137)
    assert np.abs(Rrb - Rb).max() < 1e-12 * np.abs(Rb).max()


def test_single_scattering_limit_at_arbitrary_angles():
    """F(omega) - F_ss(omega) = O(omega^2) for a beam at mu0 = 0.437 reflected towards -0.21 and
    -0.83 (neither a node): halving omega quarters the remainder (F_ss itself is O(omega), so the
    remainder relative to it is O(omega))."""
    N, L, P, tau = 6, 8, 5, 0.8
    coef = hg(5, L)
    mu0, mo = 0.437, np.array([0.21, 0.83])
    dphi = 2 * np.pi * np.arange(P) / P
    rem = []
    for om in (2e-3, 1e-3):
        F = reconstruct.brdf_beam_outgoing(coef, tau, om, N, L, P, mu0, mo)  # (o, k, 4, 4)
        Fss = analytic.single_scattering(coef, om, tau, mo, np.array([mu0]), dphi)[:, 0]
        assert np.abs(F - Fss).max() < om * np.abs(Fss[..., 0, 0]).max()
        rem.append(np.abs(F - Fss).max())
    assert 3.8 < rem[0] / rem[1] < 4.2, rem


@pytest.mark.parametrize("m", [0, 1, 2])
def test_reconstruction_matches_propagator_with_zero_weight_directions(m):
    """An outgoing direction carried through the 40-digit propagator as a node of zero weight
    (its own transport equation, no share in the scattering integral) gives the exact radiance
    towards it; the source-function integration must agree, for the stream inputs of the nodes and
    for an off-node beam. No eigenvector, Legendre recurrence or closed-form integral is shared."""
    from oracle import brute

    N, tau, om, mu0 = 2, 0.9, 0.95, 0.437
    mo = np.array([0.21, 0.83])
    coef = hg(7, 6)
    mu, al = double_gauss(N)
    Rs = brute.stream_response(coef, om, tau, m, N, dps=30, extra=mo)[4 * N:]
    Rr = reconstruct.solve_order_outgoing(coef, om, tau, m, mu, al, mo)
    assert np.abs(Rr - Rs).max() < 1e-11 * np.abs(Rs).max()
    Rb = brute.beam_response(coef, om, tau, m, N, mu0, dps=30, extra=mo)[4 * N:]
    Rrb = reconstruct.solve_order_outgoing(coef, om, tau, m, mu, al, mo, mu0)
    assert np.abs(Rrb - Rb).max() < 1e-11 * np.abs(Rb).max()
