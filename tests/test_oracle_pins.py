"""Pins of the CPU oracle against facts fixed by the paper, by mathematics or by physics.

Each test checks the oracle against something other than itself: closed forms, library routines,
an independent eigenvector-free solve at extended precision, conservation laws and symmetry
relations. The mutation tests at the end plant a plausible mistake in the oracle (on the CPU) and
check that the pins catch it.
"""

import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import gammaln, lpmv

from oracle import analytic, brute, dom, doubling, legendre, particular, phase
from oracle.quadrature import double_gauss
from workloads.layers import _d_sequences, hg_like_coefficients, rayleigh_coefficients

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
D4 = np.diag([1.0, 1.0, -1.0, -1.0])
QF = np.diag([1.0, 1.0, -1.0, 1.0])


def hg(seed, L):
    return hg_like_coefficients(np.random.default_rng(seed), L)[0]


# ---------------------------------------------------------------- P1: quadrature (eq. 15)
@pytest.mark.parametrize("N", [1, 2, 5, 16, 32])
def test_quadrature_moments(N):
    mu, al = double_gauss(N)
    assert np.all(np.diff(mu) > 0) and mu[0] > 0 and mu[-1] < 1
    for k in range(2 * N):
        assert abs(np.sum(al * mu ** k) - 1.0 / (k + 1)) < 1e-15 * 4


# ---------------------------------------------------------------- Wigner d / Legendre functions
def test_wigner_d_matches_jacobi_closed_form():
    x = np.linspace(-0.999, 0.999, 41)
    L = 60
    d00, d22, d2m2, d02 = _d_sequences(L, x)
    assert np.abs(legendre.wigner_d_seq(L, 0, 0, x) - d00).max() < 1e-13
    assert np.abs(legendre.wigner_d_seq(L, 2, 2, x) - d22).max() < 1e-13
    assert np.abs(legendre.wigner_d_seq(L, 2, -2, x) - d2m2).max() < 1e-13
    assert np.abs(legendre.wigner_d_seq(L, 0, 2, x) - d02).max() < 1e-13


@pytest.mark.parametrize("m", [0, 1, 3, 7])
def test_normalised_associated_legendre(m):
    """d^l_{m0} = sqrt((l-m)!/(l+m)!) P_l^m (library associated Legendre, Condon-Shortley phase)."""
    x = np.linspace(-0.99, 0.99, 23)
    L = 30
    d = legendre.wigner_d_seq(L, m, 0, x)
    for l in range(m, L):
        ref = np.exp(0.5 * (gammaln(l - m + 1) - gammaln(l + m + 1))) * lpmv(m, l, x)
        assert np.abs(d[l] - ref).max() < 1e-13


def test_wigner_orthogonality():
    x, w = np.polynomial.legendre.leggauss(80)
    for (m, n) in [(0, 0), (2, 2), (2, -2), (0, 2), (3, 2), (5, -2)]:
        d = legendre.wigner_d_seq(40, m, n, x)
        G = (d * w) @ d.T
        lmin = max(abs(m), abs(n))
        ref = np.diag([2.0 / (2 * l + 1) if l >= lmin else 0.0 for l in range(40)])
        assert np.abs(G - ref).max() < 1e-13


@pytest.mark.parametrize("m", [0, 1, 2, 5])
def test_legendre_matrix_parity(m):
    """eq. 10: P_l^m(-mu) = (-1)^(l-m) D P_l^m(mu) D."""
    mu = np.array([0.1, 0.45, 0.9])
    L = 12
    Pp = legendre.legendre_matrices(L, m, mu)
    Pm = legendre.legendre_matrices(L, m, -mu)
    for l in range(m, L):
        assert np.abs(Pm[l] - (-1) ** (l - m) * D4 @ Pp[l] @ D4).max() < 1e-14


# ---------------------------------------------------------------- P2: Rayleigh expansion
def test_rayleigh_projection_matches_hand_derivation():
    ref = np.loadtxt(os.path.join(GOLDEN, "rayleigh_expansion.txt"))
    assert np.abs(rayleigh_coefficients() - ref).max() < 1e-14


def test_rayleigh_resynthesis():
    coef = np.loadtxt(os.path.join(GOLDEN, "rayleigh_expansion.txt"))
    x = np.linspace(-1, 1, 101)
    F = phase.scattering_matrix(coef, x)
    assert np.abs(F[:, 0, 0] - 0.75 * (1 + x * x)).max() < 1e-14
    assert np.abs(F[:, 1, 1] - 0.75 * (1 + x * x)).max() < 1e-14
    assert np.abs(F[:, 2, 2] - 1.5 * x).max() < 1e-14
    assert np.abs(F[:, 3, 3] - 1.5 * x).max() < 1e-14
    assert np.abs(F[:, 0, 1] + 0.75 * (1 - x * x)).max() < 1e-14
    assert np.abs(F[:, 2, 3]).max() < 1e-14


def test_geometric_phase_matrix_forward_and_normalisation():
    """Z reduces to F(0) in the forward direction limit and (1/4pi) int a1 dOmega = 1."""
    coef = hg(3, 10)
    x, w = np.polynomial.legendre.leggauss(40)
    a1 = phase.scattering_matrix(coef, x)[:, 0, 0]
    assert abs(0.5 * np.sum(w * a1) - 1.0) < 1e-13
    # meridian and scattering planes coincide for phi = phi' : no rotation
    Z = phase.phase_matrix(coef, 0.3, 0.0, 0.8, 0.0)
    cos_t = 0.3 * 0.8 + np.sqrt(1 - 0.09) * np.sqrt(1 - 0.64)
    F = phase.scattering_matrix(coef, np.array([cos_t]))[0]
    assert np.abs(np.abs(Z) - np.abs(F)).max() < 1e-13


# ---------------------------------------------------------------- P3: A^m two ways (eq. 9 vs projection)
@pytest.mark.parametrize("seed,L", [(0, 8), (5, 14)])
def test_fourier_matrix_two_ways(seed, L):
    coef = hg(seed, L)
    mu, _ = double_gauss(4)
    mus = np.concatenate([mu, -mu, [0.3, -0.77]])
    for m in range(L):
        A1 = legendre.phase_fourier_matrix(coef, m, mus, mus)
        A2 = phase.projected_fourier_matrix(coef, m, mus, mus)
        scale = np.abs(legendre.phase_fourier_matrix(coef, 0, mus, mus)).max()
        assert np.abs(A1 - A2).max() < 1e-13 * scale, m


def test_fourier_matrix_rayleigh_two_ways():
    coef = rayleigh_coefficients()
    mus = np.array([0.05, 0.5, 0.95, -0.2, -0.6])
    for m in range(3):
        A1 = legendre.phase_fourier_matrix(coef, m, mus, mus)
        A2 = phase.projected_fourier_matrix(coef, m, mus, mus, n_az=16)
        assert np.abs(A1 - A2).max() < 1e-14


# ---------------------------------------------------------------- P4: half-size reduction (eq. 40-45)
@pytest.mark.parametrize("m", [0, 1, 4])
def test_half_size_reduction_matches_full_eigenproblem(m):
    """eig(F E) = 1/nu^2 and Phi+- of eq. 45 solve the full eq. 21 problem."""
    coef = hg(7, 8)
    N = 4
    n = 4 * N
    omega = 0.93
    mu, al = double_gauss(N)
    L = coef.shape[1]
    P = legendre.legendre_matrices(L, m, mu)
    B = legendre.b_matrices(coef)
    Sp = np.zeros((N, N, 4, 4))
    Sm = np.zeros((N, N, 4, 4))
    for l in range(m, L):
        sg = (-1.0) ** (l - m)
        Sp += np.einsum("iab,bc,jcd->ijad", P[l], B[l] @ (np.eye(4) + sg * D4), P[l])
        Sm += np.einsum("iab,bc,jcd->ijad", P[l], B[l] @ (np.eye(4) - sg * D4), P[l])
    Sp = Sp.transpose(0, 2, 1, 3).reshape(n, n)
    Sm = Sm.transpose(0, 2, 1, 3).reshape(n, n)
    Mv = np.repeat(mu, 4)
    Wv = np.repeat(al, 4)
    Et = (np.eye(n) - 0.5 * omega * Sp * Wv[None, :]) / Mv[:, None]
    Ft = (np.eye(n) - 0.5 * omega * Sm * Wv[None, :]) / Mv[:, None]
    lam, U = np.linalg.eig(Ft @ Et)
    K = dom.order_operator(coef, omega, m, mu, al)
    kap = np.linalg.eigvals(K)
    lam_full = np.sort_complex((kap[kap.real < 0] ** 2))
    assert np.abs(np.sort_complex(lam) - lam_full).max() < 1e-10 * np.abs(lam_full).max()
    Delta = np.kron(np.eye(N), D4)
    for j in range(n):
        nu = 1.0 / np.sqrt(lam[j])
        V = Et @ U[:, j]
        phip = 0.5 * (U[:, j] + nu * V)
        phim = 0.5 * (U[:, j] - nu * V)
        v = np.concatenate([phip, Delta @ phim])
        res = K @ v + v / nu
        assert np.abs(res).max() < 1e-9 * np.abs(K).max() * np.abs(v).max()


# ---------------------------------------------------------------- P5: tiny-N brute force (expm)
@pytest.mark.parametrize("N,tau0,omega", [(1, 0.1, 0.5), (2, 1.0, 0.9), (3, 1.0, 0.5), (3, 0.1, 0.9)])
def test_stream_form_matches_expm_propagator(N, tau0, omega):
    coef = hg(11 + N, 5)
    mu, al = double_gauss(N)
    for m in range(coef.shape[1]):
        R = dom.solve_order(coef, omega, tau0, m, mu, al)
        Rb = brute.stream_response(coef, omega, tau0, m, N, dps=30)
        assert np.abs(R - Rb).max() < 1e-13 * max(1.0, np.abs(Rb).max()), m


@pytest.mark.parametrize("N,tau0,omega", [(1, 0.1, 0.5), (2, 1.0, 0.9), (3, 3.0, 0.99)])
def test_doubling_matches_expm_propagator(N, tau0, omega):
    """The adding-doubling reference (thin-slice expm, interaction principle) against the
    extended-precision propagator: two eigenvector-free routes that share only the operator."""
    coef = hg(41 + N, 5)
    mu, al = double_gauss(N)
    for m in range(coef.shape[1]):
        Rd = doubling.solve_order(coef, omega, tau0, m, mu, al)
        Rb = brute.stream_response(coef, omega, tau0, m, N, dps=30)
        assert np.abs(Rd - Rb).max() < 1e-13 * max(1.0, np.abs(Rb).max()), m


def test_eigen_oracle_matches_doubling_every_order():
    """The eigen-based per-order solve against adding-doubling at a size the propagator cannot
    reach (N = 16, 8N = 128, thick and nearly conservative). Both are FP64; the eigen route errs by
    about eps times the condition of its 8N basis and the doubling route by about eps per doubling
    (k = 12 here), each relative to max |R|, so 1e-11 leaves two orders of margin over both."""
    coef = hg(51, 32)
    N, tau0, omega = 16, 10.0, 0.99
    mu, al = double_gauss(N)
    Rs = [dom.solve_order(coef, omega, tau0, m, mu, al) for m in range(32)]
    scale = max(np.abs(R).max() for R in Rs)
    for m in range(32):
        Rd = doubling.solve_order(coef, omega, tau0, m, mu, al)
        assert np.abs(Rs[m] - Rd).max() < 1e-11 * scale, m


@pytest.mark.parametrize("N,mu0", [(2, 0.37), (3, 0.81)])
def test_particular_form_matches_expm_propagator(N, mu0):
    coef = hg(21 + N, 5)
    tau0, omega = 0.8, 0.9
    mu, al = double_gauss(N)
    for m in range(coef.shape[1]):
        R = particular.solve_order_beam(coef, omega, tau0, m, mu, al, mu0)
        Rb = brute.beam_response(coef, omega, tau0, m, N, mu0, dps=30)
        assert np.abs(R - Rb).max() < 1e-13 * max(1.0, np.abs(Rb).max()), m


# ---------------------------------------------------------------- P6: stream form vs particular form
def test_stream_form_equals_particular_form_at_nodes():
    coef = hg(31, 10)
    N = 5
    tau0, omega = 2.0, 0.95
    mu, al = double_gauss(N)
    checked = 0
    for m in range(coef.shape[1]):
        R = dom.solve_order(coef, omega, tau0, m, mu, al)
        K = dom.order_operator(coef, omega, m, mu, al)
        nus = 1.0 / np.abs(np.linalg.eigvals(K).real)
        for q in range(N):
            if np.min(np.abs(nus - mu[q])) < 1e-3 * mu[q]:
                continue  # particular system (eq. 33) near-singular: mu0 close to an eigen-nu
            Rp = particular.solve_order_beam(coef, omega, tau0, m, mu, al, mu[q])
            assert np.abs(Rp - R[:, 4 * q:4 * q + 4]).max() < 1e-11 * max(1.0, np.abs(R).max())
            checked += 1
    assert checked > 10


def test_off_node_beam_converges_to_node_stream():
    coef = hg(32, 6)
    N = 4
    tau0, omega, m = 1.0, 0.9, 1
    mu, al = double_gauss(N)
    q = 2
    R = dom.solve_order(coef, omega, tau0, m, mu, al)[:, 4 * q:4 * q + 4]
    errs = []
    for dlt in (1e-3, 1e-4):
        lo = particular.solve_order_beam(coef, omega, tau0, m, mu, al, mu[q] * (1 - dlt))
        hi = particular.solve_order_beam(coef, omega, tau0, m, mu, al, mu[q] * (1 + dlt))
        errs.append(np.abs(0.5 * (lo + hi) - R).max())
        assert np.abs(lo - R).max() < 50 * dlt * np.abs(R).max()
    assert errs[1] < errs[0] / 50  # symmetric bracket: O(delta^2)


# ---------------------------------------------------------------- P7: single-scattering limit
def test_single_scattering_limit():
    coef = hg(41, 6)
    N, L, omega, nd = 4, 6, 0.8, 12
    mu, _ = double_gauss(N)
    dphi = 2 * np.pi * np.arange(nd) / nd
    mask = np.ones((N, N, nd), bool)
    for i in range(N):
        mask[i, i, 0] = False
        mask[i, i, nd // 2] = False
    diffs = []
    for tau0 in (1e-4, 5e-5):
        F = dom.brdf(coef, tau0, omega, N, L, nd)
        Fss = np.zeros_like(F)
        for i in range(N):
            for q in range(N):
                for k in range(nd):
                    if mask[i, q, k]:
                        Fss[i, q, k] = analytic.single_scattering(coef, omega, tau0, [mu[i]], [mu[q]], [dphi[k]])[0, 0, 0]
        d = np.abs(F - Fss)[mask].max()
        assert d <= 2 * tau0 * np.abs(Fss[mask]).max() * 10
        diffs.append(d)
    ratio = diffs[0] / diffs[1]
    assert 3.9 < ratio < 4.1  # residual is second order in tau0


# ---------------------------------------------------------------- P8/P9: reciprocity and structure
@pytest.fixture(scope="module")
def polarized_brdf():
    coef = hg(51, 8)
    F = dom.brdf(coef, 0.7, 0.9, 5, 8, 12)
    return F


def test_reciprocity(polarized_brdf):
    """F(i <- q, dphi) = Q F(q <- i, -dphi)^T Q, Q = diag(1, 1, -1, 1) (incident and reflected
    directions swapped and reversed, which reverses the azimuth difference)."""
    F = polarized_brdf
    nd = F.shape[2]
    Fm = F[:, :, (-np.arange(nd)) % nd].transpose(1, 0, 2, 4, 3)
    assert np.abs(F - QF @ Fm @ QF).max() < 1e-12 * np.abs(F).max()


def test_mirror_structure(polarized_brdf):
    F = polarized_brdf
    nd = F.shape[2]
    Fm = F[:, :, (-np.arange(nd)) % nd]
    assert np.abs(Fm - D4 @ F @ D4).max() < 1e-14 * np.abs(F).max()


def test_rayleigh_v_decouples():
    F = dom.brdf(rayleigh_coefficients(), 1.0, 0.9, 4, 3, 8)
    assert np.abs(F[..., 3, :3]).max() < 1e-14 * np.abs(F).max()
    assert np.abs(F[..., :3, 3]).max() < 1e-14 * np.abs(F).max()
    assert np.abs(F[..., 3, 3]).max() > 1e-4


# ---------------------------------------------------------------- P10: flux conservation
@pytest.mark.parametrize("N,L,tau0", [(4, 8, 1.3), (6, 12, 0.2)])
def test_flux_conservation(N, L, tau0):
    coef = hg(61 + N, L)
    mu, al = double_gauss(N)
    R0, T0 = dom.solve_order(coef, dom.OMEGA_MAX, tau0, 0, mu, al, want_transmission=True)
    for q in range(N):
        tot = np.pi / mu[q] * np.sum(al * mu * (R0[0::4, 4 * q] + T0[0::4, 4 * q]))
        assert abs(tot - 1.0) < 1e-9


def test_absorbing_layer_loses_flux():
    coef = hg(62, 8)
    mu, al = double_gauss(4)
    R0, T0 = dom.solve_order(coef, 0.7, 1.0, 0, mu, al, want_transmission=True)
    for q in range(4):
        tot = np.pi / mu[q] * np.sum(al * mu * (R0[0::4, 4 * q] + T0[0::4, 4 * q]))
        assert 0 < tot < 1


# ---------------------------------------------------------------- P11: Chandrasekhar H (isotropic)
@pytest.mark.parametrize("N,omega", [(2, 0.9), (8, 0.9), (6, 0.5)])
def test_isotropic_semi_infinite_h_function(N, omega):
    mu, al = double_gauss(N)
    coef = np.zeros((6, 1))
    coef[0, 0] = 1.0
    F = dom.brdf(coef, 100.0, omega, N, 1, 4)
    H = analytic.chandrasekhar_h(omega, mu, al, mu)
    F11 = omega / (4 * np.pi) * H[:, None] * H[None, :] / (mu[:, None] + mu[None, :])
    for k in range(4):
        assert np.abs(F[:, :, k, 0, 0] - F11).max() < 1e-12 * np.abs(F11).max()
    F2 = F.copy()
    F2[..., 0, 0] = 0.0
    assert np.abs(F2).max() == 0.0


# ---------------------------------------------------------------- P12: unpolarized limit vs scalar DOM
def _scalar_reflection(alpha1, omega, tau0, m, N):
    """Independent scalar DOM: A = sum alpha1_l Pbar Pbar (library Legendre), propagator solve."""
    mu, al = double_gauss(N)
    mus = np.concatenate([mu, -mu])
    L = len(alpha1)
    A = np.zeros((2 * N, 2 * N))
    for l in range(m, L):
        p = np.exp(0.5 * (gammaln(l - m + 1) - gammaln(l + m + 1))) * lpmv(m, l, mus)
        A += alpha1[l] * np.outer(p, p)
    w = np.concatenate([al, al])
    K = (0.5 * omega * A * w[None, :] - np.eye(2 * N)) / mus[:, None]
    Psi = expm(K * tau0)
    R = -np.linalg.solve(Psi[N:, N:], Psi[N:, :N])
    return R / (np.pi * al[None, :])


def test_unpolarized_limit_matches_scalar_solver():
    L, N, tau0, omega = 6, 3, 0.6, 0.85
    coef = np.zeros((6, L))
    g = 0.6
    coef[0] = (2 * np.arange(L) + 1) * g ** np.arange(L)
    mu, al = double_gauss(N)
    for m in range(L):
        R = dom.solve_order(coef, omega, tau0, m, mu, al)
        Rs = _scalar_reflection(coef[0], omega, tau0, m, N)
        assert np.abs(R[0::4, 0::4] - Rs).max() < 1e-12 * max(1, np.abs(Rs).max())
        Rb = R.reshape(N, 4, N, 4).copy()
        Rb[:, 0, :, 0] = 0.0
        assert np.abs(Rb).max() == 0.0
    F = dom.brdf(coef, tau0, omega, N, L, 8)
    assert np.abs(F[..., 1:, :]).max() == 0.0 and np.abs(F[..., :, 1:]).max() == 0.0


# ---------------------------------------------------------------- P13/P14: soft physics checks
def test_positivity_and_degree_of_polarization(polarized_brdf):
    F = polarized_brdf
    assert np.all(F[..., 0, 0] > 0)
    dop = np.sqrt(F[..., 1, 0] ** 2 + F[..., 2, 0] ** 2 + F[..., 3, 0] ** 2)
    assert np.all(dop <= F[..., 0, 0])


def test_truncation_partial_sums_converge():
    coef = hg(71, 12)
    F_full, R = dom.brdf(coef, 1.0, 0.9, 4, 12, 8, return_orders=True)
    mu, _ = double_gauss(4)
    errs = [np.abs(dom.synthesize(R[:M], mu, 8) - F_full).max() for M in (2, 6, 10)]
    assert errs[0] > errs[1] > errs[2]


# ---------------------------------------------------------------- P15: gauge invariance of eigenbasis
def test_eigenbasis_gauge_invariance():
    coef = hg(81, 8)
    N = 4
    mu, al = double_gauss(N)
    rng = np.random.default_rng(5)

    def hook(H0, H1, kappa, V, tau0):
        n2 = V.shape[1]
        perm = rng.permutation(n2)
        sc = rng.uniform(0.2, 5.0, n2) * np.exp(1j * rng.uniform(0, 2 * np.pi, n2))
        return (H0 * sc[None, :])[:, perm], (H1 * sc[None, :])[:, perm]

    for m in range(4):
        R = dom.solve_order(coef, 0.9, 1.5, m, mu, al)
        Rg = dom.solve_order(coef, 0.9, 1.5, m, mu, al, basis_hook=hook)
        assert np.abs(R - Rg).max() < 1e-13 * np.abs(R).max()


# ---------------------------------------------------------------- validation
def test_validation_errors():
    coef = hg(1, 5)
    with pytest.raises(ValueError):
        dom.brdf(coef, -1.0, 0.9, 2, 2, 4)
    with pytest.raises(ValueError):
        dom.brdf(coef, 1.0, 1.5, 2, 2, 4)
    with pytest.raises(ValueError):
        dom.brdf(coef, 1.0, 0.9, 2, 6, 4)
    bad = coef.copy()
    bad[0, 0] = 0.9
    with pytest.raises(ValueError):
        dom.brdf(bad, 1.0, 0.9, 2, 2, 4)
    bad = coef.copy()
    bad[3, 2] = np.nan
    with pytest.raises(ValueError):
        dom.brdf(bad, 1.0, 0.9, 2, 2, 4)


def test_oracle_deterministic():
    coef = hg(2, 6)
    a = dom.brdf(coef, 1.0, 0.9, 3, 6, 8)
    b = dom.brdf(coef, 1.0, 0.9, 3, 6, 8)
    assert np.array_equal(a, b)


# ---------------------------------------------------------------- planted mistakes must be caught
def test_planted_t_sign_flip_is_caught(monkeypatch):
    orig = legendre.legendre_scalars

    def flipped(L, m, mu):
        pb, r, t = orig(L, m, mu)
        return pb, r, -t

    monkeypatch.setattr(legendre, "legendre_scalars", flipped)
    coef = hg(0, 8)
    mus = np.array([0.2, 0.7, -0.4])
    worst = max(np.abs(legendre.phase_fourier_matrix(coef, m, mus, mus)
                       - phase.projected_fourier_matrix(coef, m, mus, mus)).max() for m in range(1, 4))
    assert worst > 1e-3


def test_planted_left_weights_are_caught(monkeypatch):
    """Weights on the left (eq. 19 as printed) instead of the right disagree with the propagator."""
    def op_left(coef, omega, m, mu, alpha):
        N = len(mu)
        Abig = dom.full_phase_block(coef, m, mu)
        w = np.repeat(np.concatenate([alpha, alpha]), 4)
        mh = np.repeat(np.concatenate([mu, -mu]), 4)
        return (0.5 * omega * w[:, None] * Abig - np.eye(8 * N)) / mh[:, None]

    coef = hg(13, 5)
    mu, al = double_gauss(3)  # N = 2 has equal weights, which would hide the mistake
    Rb = brute.stream_response(coef, 0.9, 1.0, 0, 3, dps=30)
    monkeypatch.setattr(dom, "order_operator", op_left)
    R = dom.solve_order(coef, 0.9, 1.0, 0, mu, al)
    assert np.abs(R - Rb).max() > 1e-4


def test_planted_mirrored_boundary_labels_are_caught(monkeypatch):
    """Zero light imposed on the outgoing instead of the incoming streams is not the black-base BVP."""
    coef = hg(14, 5)
    mu, al = double_gauss(2)
    n = 8
    Rb = brute.stream_response(coef, 0.9, 1.0, 0, 2, dps=30)
    K = dom.order_operator(coef, 0.9, 0, mu, al)
    H0, H1, _, _ = dom.eigen_basis(K, 1.0)
    Bc = np.vstack([H0[n:, :], H1[:n, :]])  # mirrored labels
    rhs = np.zeros((2 * n, n))
    rhs[:n, :] = dom.stream_rhs(al)
    c = np.linalg.solve(Bc, rhs)
    R = (H0[:n, :] @ c).real
    assert np.abs(R - Rb).max() > 1e-3


def test_planted_source_normalisation_is_caught():
    """The printed omega/(4 pi) of eq. 14 (with the 1/2 of eq. 12) halves the beam response."""
    coef = hg(15, 5)
    N, mu0, tau0, om = 2, 0.37, 0.8, 0.9
    mu, al = double_gauss(N)
    Rb = brute.beam_response(coef, om, tau0, 1, N, mu0, dps=30)
    R = particular.solve_order_beam(coef, om, tau0, 1, mu, al, mu0)
    assert np.abs(R - Rb).max() < 1e-13
    assert np.abs(0.5 * R - Rb).max() > 1e-3
