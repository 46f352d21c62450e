"""Pins of the stack and reflecting-base oracle (oracle/stack.py) against results that do not come
from it: the 40-digit propagator product (no eigenvectors, no boundary matrix), the splitting of one
layer into two, the unscattered closed form over a Lambertian base, flux conservation over a white
base, and a planted mistake in the base weights."""

import numpy as np
import pytest

from oracle import brute, dom, stack
from oracle.quadrature import double_gauss
from workloads.layers import hg_like_coefficients


def hg(seed, L):
    return hg_like_coefficients(np.random.default_rng(seed), L)[0]


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("m", [0, 1, 2])
def test_two_layers_against_propagator(m):
    """Interface continuity (Sec. 2.C): two different layers over a black base against the product
    of their expm propagators."""
    N = 2
    mu, al = double_gauss(N)
    layers = [(hg(1, 6), 0.9, 0.6), (hg(2, 6), 0.7, 1.1)]
    ref = brute.stack_stream_response(layers, m, N)
    assert rel(stack.solve_order_stack(layers, m, mu, al), ref) < 1e-13


@pytest.mark.parametrize("m", [0, 1, 2])
def test_mueller_base_against_propagator(m):
    """Base condition of eq. 57-58 with a general per-order Mueller base (random blocks), two layers,
    against the propagator closed by the same base matrix."""
    N = 2
    mu, al = double_gauss(N)
    Rb = np.random.default_rng(10 + m).standard_normal((N, N, 4, 4)) * 0.2
    layers = [(hg(3, 6), 0.95, 0.5), (hg(4, 6), 0.8, 0.9)]
    ref = brute.stack_stream_response(layers, m, N, stack.base_operator(Rb, mu, al))
    assert rel(stack.solve_order_stack(layers, m, mu, al, Rb), ref) < 1e-13


def test_lambertian_base_against_propagator():
    N = 2
    mu, al = double_gauss(N)
    layers = [(hg(5, 5), 0.97, 1.4)]
    Rb = stack.lambertian_base(0.8, 0, N)
    ref = brute.stack_stream_response(layers, 0, N, stack.base_operator(Rb, mu, al))
    assert rel(stack.solve_order_stack(layers, 0, mu, al, Rb), ref) < 1e-13


@pytest.mark.parametrize("base", [None, "lambertian"])
def test_split_layer_is_the_same_layer(base):
    """A layer of optical thickness 2.0 cut into 0.7 + 1.3 of the same material is the same layer."""
    N = 4
    mu, al = double_gauss(N)
    c = hg(6, 8)
    for m in range(4):
        Rb = None if base is None else stack.lambertian_base(0.5, m, N)
        one = stack.solve_order_stack([(c, 0.95, 2.0)], m, mu, al, Rb)
        two = stack.solve_order_stack([(c, 0.95, 0.7), (c, 0.95, 1.3)], m, mu, al, Rb)
        assert rel(two, one) < 1e-12
        if base is None:
            assert rel(one, dom.solve_order(c, 0.95, 2.0, m, mu, al)) < 1e-12


def lambertian_unscattered(rho, tau, mu):
    """Stream of radiance 1 / (pi alpha_q) on node q, attenuated to the base, reflected
    isotropically with radiance 2 rho sum_j alpha_j mu_j I_j and attenuated back:
    R^0[(i, I), (q, I)] = (2 rho / pi) mu_q exp(-tau / mu_q - tau / mu_i)."""
    N = len(mu)
    ref = np.zeros((4 * N, 4 * N))
    for i in range(N):
        for q in range(N):
            ref[4 * i, 4 * q] = 2 * rho * mu[q] / np.pi * np.exp(-tau / mu[q] - tau / mu[i])
    return ref


def test_lambertian_base_without_scattering():
    """omega -> 0: only the base reflects; at tau -> 0 this is the Lambertian BRDF rho / pi."""
    N, rho = 4, 0.6
    mu, al = double_gauss(N)
    c = hg(7, 8)
    for tau in (0.3, 1e-9):
        R = stack.solve_order_stack([(c, 1e-14, tau)], 0, mu, al, stack.lambertian_base(rho, 0, N))
        assert np.abs(R - lambertian_unscattered(rho, tau, mu)).max() < 1e-13
    F = stack.brdf_stack([(c, 1e-9, 1e-14)], N, 3, 5, base="lambertian", rho=rho)
    att = np.exp(-1e-9 / mu[:, None] - 1e-9 / mu[None, :])[:, :, None]
    assert np.abs(F[..., 0, 0] - rho / np.pi * att).max() < 1e-13
    assert np.abs(F[..., 0, 0] - rho / np.pi).max() < 1e-7
    assert np.abs(F[..., 1:, :]).max() < 1e-12 and np.abs(F[..., 0, 1:]).max() < 1e-12
    for m in (1, 2):
        R = stack.solve_order_stack([(c, 1e-14, 0.3)], m, mu, al, stack.lambertian_base(rho, m, N))
        assert np.abs(R).max() < 1e-13


def test_planted_base_weight_mistake_is_caught():
    """Dropping mu_j from the quadrature weights of eq. 58 breaks the unscattered closed form."""
    N, rho, tau = 4, 0.6, 0.3
    mu, al = double_gauss(N)
    c = hg(7, 8)
    wrong = stack.lambertian_base(rho, 0, N) / mu[None, :, None, None]  # alpha_j instead of alpha_j mu_j
    R = stack.solve_order_stack([(c, 1e-14, tau)], 0, mu, al, wrong)
    assert np.abs(R - lambertian_unscattered(rho, tau, mu)).max() > 1e-3


@pytest.mark.parametrize("tau", [0.5, 4.0])
def test_white_base_conserves_flux(tau):
    """omega = 1 over a white Lambertian base: nothing is absorbed, so every unit I stream's
    reflected m = 0 flux is 1 (the clamp omega <= 1 - 1e-12 leaves ~1e-11)."""
    N = 6
    mu, al = double_gauss(N)
    R = stack.solve_order_stack([(hg(8, 12), 1 - 1e-12, tau)], 0, mu, al, stack.lambertian_base(1.0, 0, N))
    for q in range(N):
        flux = np.pi / mu[q] * np.sum(al * mu * R[0::4, 4 * q])
        assert abs(flux - 1.0) < 1e-9, (q, flux)


def test_mueller_base_equal_to_a_layer_is_that_layer():
    """A base whose Mueller blocks are the reflection of layer B (Rb = R_B R0^-1 / (alpha_j mu_j))
    gives the two-layer stack (A over B)."""
    N = 4
    mu, al = double_gauss(N)
    A, B = (hg(9, 8), 0.9, 0.7), (hg(10, 8), 0.98, 3.0)
    r0 = np.repeat(1.0 / (np.pi * al), 4)
    for m in range(3):
        RB = dom.solve_order(B[0], B[1], B[2], m, mu, al)
        Xb = RB / r0[None, :]
        Rb = (Xb.reshape(N, 4, N, 4).transpose(0, 2, 1, 3)) / (al * mu)[None, :, None, None]
        via_base = stack.solve_order_stack([A], m, mu, al, Rb)
        assert rel(via_base, stack.solve_order_stack([A, B], m, mu, al)) < 1e-12
