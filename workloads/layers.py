"""Synthetic homogeneous particulate layers (expansion coefficients, optical thickness, albedo).

The paper's materials come from a Mie code whose phase matrices are not available here, so the
workloads below stand in for them: seeded "Henyey-Greenstein-like" coefficient sets whose
scattering matrix passes the standard validity inequalities, plus the closed-form Rayleigh matrix
projected onto the expansion functions. Everything here is input construction; nothing in this
module takes part in the radiative transfer solution.

Coefficient convention (rows of a ``(6, L)`` array, degree ``l = 0..L-1``)::

    a1(x)      =  sum_l alpha1_l d^l_{00}(x)
    a4(x)      =  sum_l alpha4_l d^l_{00}(x)
    a2 + a3    =  sum_l (alpha2_l + alpha3_l) d^l_{2,2}(x)
    a2 - a3    =  sum_l (alpha2_l - alpha3_l) d^l_{2,-2}(x)
    b1(x)      = -sum_l beta1_l d^l_{0,2}(x)
    b2(x)      = -sum_l beta2_l d^l_{0,2}(x)

with ``x = cos(Theta)`` and ``d^l_{mn}`` the Wigner d-functions. The scattering matrix is
``F = [[a1, b1, 0, 0], [b1, a2, 0, 0], [0, 0, a3, b2], [0, 0, -b2, a4]]`` and the normalisation is
``alpha1_0 = 1`` (half the integral of a1 over x is one). Under this convention the Rayleigh
matrix has ``beta1_2 = +sqrt(6)/2``.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache
from typing import List

import numpy as np
from scipy.special import eval_jacobi, gammaln, roots_legendre

COEF_ROWS = ("alpha1", "alpha2", "alpha3", "alpha4", "beta1", "beta2")


# --------------------------------------------------------------------------------------------
# Wigner d-functions through Jacobi polynomials (library route, used for projection/validation)
# --------------------------------------------------------------------------------------------
def _wigner_d(j: int, m: int, n: int, x: np.ndarray) -> np.ndarray:
    """d^j_{mn}(beta) at x = cos(beta), from the Jacobi-polynomial closed form."""
    if j < max(abs(m), abs(n)):
        return np.zeros_like(x)
    if n - m >= 0 and n + m >= 0:
        lp = 0.5 * (gammaln(j + n + 1) + gammaln(j - n + 1) - gammaln(j + m + 1) - gammaln(j - m + 1))
        half_sin = np.sqrt(np.clip((1.0 - x) / 2.0, 0.0, None))
        half_cos = np.sqrt(np.clip((1.0 + x) / 2.0, 0.0, None))
        return np.exp(lp) * half_sin ** (n - m) * half_cos ** (n + m) * eval_jacobi(j - n, n - m, n + m, x)
    if m - n >= 0 and m + n >= 0:
        return (-1.0) ** (m - n) * _wigner_d(j, n, m, x)
    return _wigner_d(j, -n, -m, x)


def _jacobi_sequence(K: int, a: float, b: float, x: np.ndarray) -> np.ndarray:
    """P^{(a,b)}_k(x) for k = 0..K-1 by the standard three-term recurrence in the degree."""
    out = np.zeros((max(K, 0),) + x.shape)
    if K <= 0:
        return out
    out[0] = 1.0
    if K > 1:
        out[1] = (a + 1) + (a + b + 2) * (x - 1) / 2
    for k in range(2, K):
        c = 2 * k + a + b
        out[k] = ((c - 1) * (c * (c - 2) * x + a * a - b * b) * out[k - 1]
                  - 2 * (k + a - 1) * (k + b - 1) * c * out[k - 2]) / (2 * k * (k + a + b) * (c - 2))
    return out


def _d_sequences(L: int, x: np.ndarray):
    """Rows l = 0..L-1 of d^l_{00}, d^l_{2,2}, d^l_{2,-2}, d^l_{0,2} at x (Jacobi closed forms)."""
    hs2 = np.clip((1.0 - x) / 2.0, 0.0, None)  # sin^2(beta/2)
    hc2 = np.clip((1.0 + x) / 2.0, 0.0, None)  # cos^2(beta/2)
    d00 = _jacobi_sequence(L, 0, 0, x)
    d22 = np.zeros((L,) + x.shape)
    d2m2 = np.zeros((L,) + x.shape)
    d02 = np.zeros((L,) + x.shape)
    if L > 2:
        j = np.arange(2, L, dtype=np.float64)
        d22[2:] = hc2 ** 2 * _jacobi_sequence(L - 2, 0, 4, x)
        d2m2[2:] = hs2 ** 2 * _jacobi_sequence(L - 2, 4, 0, x)
        pref = np.exp(0.5 * (gammaln(j + 3) + gammaln(j - 1) - 2 * gammaln(j + 1)))
        d02[2:] = pref[:, None] * (hs2 * hc2) * _jacobi_sequence(L - 2, 2, 2, x)
    return d00, d22, d2m2, d02


def scattering_elements(coef: np.ndarray, x: np.ndarray):
    """(a1, a2, a3, a4, b1, b2) at x = cos(Theta) for a (6, L) coefficient array."""
    coef = np.asarray(coef, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    d00, d22, d2m2, d02 = _d_sequences(coef.shape[1], x)
    a1 = coef[0] @ d00
    a4 = coef[3] @ d00
    apl = (coef[1] + coef[2]) @ d22
    ami = (coef[1] - coef[2]) @ d2m2
    b1 = -(coef[4] @ d02)
    b2 = -(coef[5] @ d02)
    return a1, 0.5 * (apl + ami), 0.5 * (apl - ami), a4, b1, b2


@lru_cache(maxsize=4)
def _check_grid(n_points: int) -> np.ndarray:
    x, _ = roots_legendre(n_points)
    x.setflags(write=False)
    return x


def positivity_ok(coef: np.ndarray, n_points: int = 4096, slack: float = 1e-12) -> bool:
    """Validity inequalities of a single-scattering matrix, checked on a Gauss grid in x."""
    x = _check_grid(n_points)
    a1, a2, a3, a4, b1, b2 = scattering_elements(coef, x)
    tol = slack * max(1.0, float(np.max(np.abs(a1))))
    if np.any(a1 < -tol):
        return False
    for e in (a2, a3, a4, b1, b2):
        if np.any(np.abs(e) > a1 + tol):
            return False
    if np.any((a3 + a4) ** 2 + 4 * b2 ** 2 > (a1 + a2) ** 2 - 4 * b1 ** 2 + tol):
        return False
    if np.any(np.abs(a3 - a4) > a1 - a2 + tol):
        return False
    return True


def rayleigh_coefficients() -> np.ndarray:
    """Rayleigh (depolarisation 0) matrix projected onto the expansion functions, L = 3.

    The closed form is a1 = a2 = 3/4 (1 + x^2), a3 = a4 = 3/2 x, b1 = -3/4 (1 - x^2), b2 = 0. The
    projection uses the orthogonality of d^l_{mn} (weight 2/(2l+1)) with a Gauss rule exact for the
    polynomial integrands.
    """
    x, w = np.polynomial.legendre.leggauss(16)
    a1 = 0.75 * (1 + x * x)
    a2 = a1.copy()
    a3 = 1.5 * x
    a4 = a3.copy()
    b1 = -0.75 * (1 - x * x)
    b2 = np.zeros_like(x)
    L = 3
    coef = np.zeros((6, L))
    for l in range(L):
        h = (2 * l + 1) / 2.0
        d00 = _wigner_d(l, 0, 0, x)
        coef[0, l] = h * np.sum(w * a1 * d00)
        coef[3, l] = h * np.sum(w * a4 * d00)
        if l >= 2:
            s = h * np.sum(w * (a2 + a3) * _wigner_d(l, 2, 2, x))
            d = h * np.sum(w * (a2 - a3) * _wigner_d(l, 2, -2, x))
            coef[1, l] = 0.5 * (s + d)
            coef[2, l] = 0.5 * (s - d)
            d02 = _wigner_d(l, 0, 2, x)
            coef[4, l] = -h * np.sum(w * b1 * d02)
            coef[5, l] = -h * np.sum(w * b2 * d02)
    coef[np.abs(coef) < 1e-15] = 0.0
    coef[0, 0] = 1.0
    return coef


def hg_like_coefficients(rng: np.random.Generator, L: int, max_tries: int = 1000):
    """Henyey-Greenstein-like decaying coefficient set of degree L-1 that passes positivity.

    Draws g ~ U[0.5, 0.9], rho, rho4 ~ U[0.5, 0.95], eta ~ U[0, 0.3], zeta ~ U[0, 0.1] and sets
    alpha1_l = (2l+1) g^l, alpha2_l = alpha3_l = rho (2l+1) g^l (l >= 2), alpha4_l = rho4 (2l+1) g^l,
    beta1_l = -eta (2l+1) g^l (l >= 2), beta2_l = zeta (2l+1) g^l (l >= 2). A set that fails the
    validity inequalities is redrawn whole from the same stream. Returns (coef, params, draws).
    """
    l = np.arange(L, dtype=np.float64)
    for tries in range(1, max_tries + 1):
        g = rng.uniform(0.5, 0.9)
        rho = rng.uniform(0.5, 0.95)
        rho4 = rng.uniform(0.5, 0.95)
        eta = rng.uniform(0.0, 0.3)
        zeta = rng.uniform(0.0, 0.1)
        base = (2 * l + 1) * g ** l
        hi = (l >= 2).astype(np.float64)
        coef = np.zeros((6, L))
        coef[0] = base
        coef[0, 0] = 1.0
        coef[1] = rho * base * hi
        coef[2] = rho * base * hi
        coef[3] = rho4 * base
        coef[4] = -eta * base * hi
        coef[5] = zeta * base * hi
        if positivity_ok(coef):
            return coef, dict(g=g, rho=rho, rho4=rho4, eta=eta, zeta=zeta), tries
    raise RuntimeError(f"no valid coefficient set after {max_tries} draws (L={L})")


# --------------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------------
@dataclass
class LayerSet:
    name: str
    tau: np.ndarray
    omega: np.ndarray
    coef: List[np.ndarray]
    N: List[int]
    L: List[int]
    M: List[int]
    n_dphi: List[int]
    draws: List[int] = field(default_factory=list)

    @property
    def n_layers(self) -> int:
        return len(self.N)

    def subset(self, idx) -> "LayerSet":
        idx = list(idx)
        return LayerSet(
            name=f"{self.name}[{len(idx)}]",
            tau=self.tau[idx].copy(),
            omega=self.omega[idx].copy(),
            coef=[self.coef[i] for i in idx],
            N=[self.N[i] for i in idx],
            L=[self.L[i] for i in idx],
            M=[self.M[i] for i in idx],
            n_dphi=[self.n_dphi[i] for i in idx],
            draws=[self.draws[i] for i in idx] if self.draws else [],
        )

    def units(self) -> int:
        """Orders x incident directions (zenith nodes x azimuths), summed over layers."""
        return int(sum(m * n * p for m, n, p in zip(self.M, self.N, self.n_dphi)))


def _streams(seed: int, n: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(n)]


def _rayleigh_c1() -> LayerSet:
    return LayerSet("rayleigh_N8", np.array([1.0]), np.array([0.9]), [rayleigh_coefficients()],
                    [8], [3], [3], [16], [1])


def _particulate_c2() -> LayerSet:
    rng = _streams(2, 1)[0]
    coef, _, draws = hg_like_coefficients(rng, 64)
    return LayerSet("particulate_N32_L64_M64", np.array([10.0]), np.array([0.99]), [coef],
                    [32], [64], [64], [64], [draws])


def _batched_c3(n_layers: int = 256) -> LayerSet:
    taus, omegas, coefs, Ns, draws = [], [], [], [], []
    for rng in _streams(3, n_layers):
        N = int(rng.choice([16, 24, 32, 48, 64]))
        tau = 10.0 ** rng.uniform(-1.0, 2.0)
        omega = rng.uniform(0.5, 0.999)
        coef, _, d = hg_like_coefficients(rng, 2 * N)
        taus.append(tau)
        omegas.append(omega)
        coefs.append(coef)
        Ns.append(N)
        draws.append(d)
    two_n = [2 * n for n in Ns]
    return LayerSet(f"batched_{n_layers}", np.array(taus), np.array(omegas), coefs, Ns, two_n,
                    list(two_n), list(two_n), draws)


def _differentiation_c4(n_layers: int = 64) -> LayerSet:
    taus, omegas, coefs, draws = [], [], [], []
    for rng in _streams(4, n_layers):
        tau = 10.0 ** rng.uniform(-1.0, 2.0)
        omega = rng.uniform(0.5, 0.999)
        coef, _, d = hg_like_coefficients(rng, 64)
        taus.append(tau)
        omegas.append(omega)
        coefs.append(coef)
        draws.append(d)
    n = n_layers
    return LayerSet(f"differentiation_{n}", np.array(taus), np.array(omegas), coefs, [32] * n,
                    [64] * n, [32] * n, [32] * n, draws)


def _large_c5() -> LayerSet:
    rng = _streams(5, 1)[0]
    coef, _, draws = hg_like_coefficients(rng, 256)
    return LayerSet("large_N128_L256_M256", np.array([50.0]), np.array([0.999]), [coef],
                    [128], [256], [256], [256], [draws])


SPECTRAL_WAVELENGTHS_NM = (400.0, 437.5, 475.0, 512.5, 550.0, 587.5, 625.0, 662.5, 700.0)


def _spectral(n_materials: int = 8, N: int = 32, L: int = 64) -> LayerSet:
    """Spectral batching: each material seen at nine wavelengths across the visible range (a
    rendering needs one BRDF per wavelength), all (material, wavelength) layers in one batch,
    material-major. Per material (seed 6, one substream each): a coefficient set from the HG-like
    generator with asymmetry g, an optical thickness tau_550 and an albedo; across wavelengths
    tau scales as (550 / lambda)^a (a ~ U[0.5, 2]), the co-albedo 1 - omega as (lambda / 550)^b
    (b ~ U[-1, 1]), and the Legendre degree l of every family is damped by (550 / lambda)^(0.1 l)
    relative to the material's set (the phase function loses forward peak towards the red). A
    damped set that fails the validity inequalities keeps the material's set. N, L, M = L and
    n_dphi = 32 are shared by all layers."""
    taus, omegas, coefs, draws = [], [], [], []
    for rng in _streams(6, n_materials):
        base, _, d = hg_like_coefficients(rng, L)
        tau550 = 10.0 ** rng.uniform(-0.5, 1.5)
        om550 = rng.uniform(0.8, 0.995)
        a, b = rng.uniform(0.5, 2.0), rng.uniform(-1.0, 1.0)
        for lam in SPECTRAL_WAVELENGTHS_NM:
            r = 550.0 / lam
            c = base * (r ** (0.1 * np.arange(L)))[None, :]
            c[0, 0] = 1.0
            coefs.append(c if positivity_ok(c) else base.copy())
            taus.append(tau550 * r ** a)
            omegas.append(min(1.0 - (1.0 - om550) * (lam / 550.0) ** b, 0.999))
            draws.append(d)
    n = len(taus)
    return LayerSet(f"spectral_{n_materials}x{len(SPECTRAL_WAVELENGTHS_NM)}", np.array(taus), np.array(omegas), coefs,
                    [N] * n, [L] * n, [L] * n, [32] * n, draws)


WORKLOADS = {
    "rayleigh": _rayleigh_c1,
    "particulate": _particulate_c2,
    "batched": _batched_c3,
    "differentiation": _differentiation_c4,
    "large": _large_c5,
    "spectral": _spectral,
}


def workload(name: str, **kw) -> LayerSet:
    """One of: rayleigh (N=8), particulate (N=32, L=M=64), batched (256 uneven layers),
    differentiation (64 layers N=32), large (N=128, L=M=256)."""
    return WORKLOADS[name](**kw)


def differentiation_targets(layers: LayerSet, seed: int = 40, max_tries: int = 100) -> LayerSet:
    """Target parameters for the differentiation workload: tau* = tau (1 + 0.05 xi),
    omega* = min(omega + 0.01 xi, 0.999), coefficient* = coefficient (1 + 0.02 xi_l) for degrees
    l >= 1 of all six families (xi ~ N(0, 1), one PCG64 substream per layer); a perturbed set that
    fails the validity inequalities is redrawn from the same stream, with the 0.02 amplitude halved
    after every 20 failed draws (sets close to the validity boundary)."""
    taus, omegas, coefs = [], [], []
    for i, rng in enumerate(_streams(seed, layers.n_layers)):
        taus.append(layers.tau[i] * (1.0 + 0.05 * rng.standard_normal()))
        omegas.append(min(layers.omega[i] + 0.01 * rng.standard_normal(), 0.999))
        for k in range(max_tries):
            c = layers.coef[i].copy()
            amp = 0.02 * 0.5 ** (k // 20)
            c[:, 1:] *= 1.0 + amp * rng.standard_normal(c[:, 1:].shape)
            if positivity_ok(c):
                break
        else:
            raise RuntimeError(f"no valid target set for layer {i}")
        coefs.append(c)
    return LayerSet(layers.name + "_target", np.array(taus), np.array(omegas), coefs, list(layers.N),
                    list(layers.L), list(layers.M), list(layers.n_dphi), [])
