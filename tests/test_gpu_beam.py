"""GPU parity of off-node incidence (Sec. 2.C particular solution, eq. 28-33, in the half-size form of
Sec. 3.B, eq. 46-48) against the oracle's full 8N particular-form solver, and properties that hold at
any size: the full-size particulate layer, and a beam at a resonance reported NUMERIC."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import particular
from oracle.quadrature import double_gauss
from paper_1707_05882_amd import api, binding
from paper_1707_05882_amd.api import BRDFSolver
from workloads import workload
from workloads.layers import hg_like_coefficients

pytestmark = pytest.mark.gpu
TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    binding.load()


def hg(seed, L):
    return hg_like_coefficients(np.random.default_rng(seed), L)[0]


def err(F, Fo):
    return float(np.abs(F - Fo).max() / np.abs(Fo[..., 0, 0]).max())


def test_beams_against_oracle():
    """Six incident cosines across (0, 1], including grazing and normal incidence."""
    N, L, P = 8, 12, 7
    mu0 = [0.05, 0.3137, 0.5, 0.8123, 0.99, 1.0]
    coef, tau, om = hg(301, L), 1.7, 0.93
    s = BRDFSolver([N], [L], [L], [P], mu0=mu0)
    F = s([tau], [om], [coef])[0].cpu().numpy()
    Fb = s.beams(0).cpu().numpy()
    assert Fb.shape == (N, len(mu0), P, 4, 4) and np.isfinite(F).all()
    for j, m0 in enumerate(mu0):
        Fo = particular.brdf_beam(coef, tau, om, N, L, P, m0)  # (N, P, 4, 4)
        assert err(Fb[:, j], Fo) < TOL, (m0, err(Fb[:, j], Fo))


def test_beams_in_a_plan_of_several_layers():
    """Layers of different N, L and M share the plan's incident cosines."""
    Ns, Ls, Ms, Ps = [5, 9, 6], [8, 14, 10], [8, 10, 10], [4, 6, 5]
    mu0 = [0.21, 0.66, 0.93]
    layers = [(hg(310 + i, Ls[i]), t, w) for i, (t, w) in enumerate([(0.4, 0.9), (3.0, 0.99), (1.1, 0.7)])]
    s = BRDFSolver(Ns, Ls, Ms, Ps, mu0=mu0)
    s([l[1] for l in layers], [l[2] for l in layers], [l[0] for l in layers])
    for i, (c, t, w) in enumerate(layers):
        Fb = s.beams(i).cpu().numpy()
        for j, m0 in enumerate(mu0):
            Fo = particular.brdf_beam(c, t, w, Ns[i], Ms[i], Ps[i], m0)
            assert err(Fb[:, j], Fo) < TOL, (i, m0)


def test_beams_at_full_particulate_size():
    """N = 32, L = M = n_dphi = 64 (the particulate layer, tau0 = 10, omega = 0.99): two off-node
    beams against the oracle at every output. A beam exactly on a Gauss node is resonant in this
    layer's high orders (the scattering there is below 1e-12 of the unscattered term, so FE has
    1/mu_q^2 as an eigenvalue to that accuracy) and the layer is reported NUMERIC."""
    w = workload("particulate")
    N, L, M, P = w.N[0], w.L[0], w.M[0], w.n_dphi[0]
    mu0 = [0.2371, 0.7519]
    s = BRDFSolver([N], [L], [M], [P], mu0=mu0)
    s([w.tau[0]], [w.omega[0]], [w.coef[0]])
    Fb = s.beams(0).cpu().numpy()
    for j, m0 in enumerate(mu0):
        Fo = particular.brdf_beam(w.coef[0], w.tau[0], w.omega[0], N, M, P, m0)
        assert err(Fb[:, j], Fo) < TOL, (m0, err(Fb[:, j], Fo))
    mu, _ = double_gauss(N)
    r = BRDFSolver([N], [L], [M], [P], mu0=[mu[20]])
    t, om, c = r.upload([w.tau[0]], [w.omega[0]], [w.coef[0]])
    r.solve_device(t, om, c)
    torch.cuda.synchronize()
    assert r.status.cpu().tolist() == [binding.E_NUMERIC]


def test_resonant_beam_is_numeric():
    """mu0 = lambda_k^-1/2 for a real eigenvalue lambda_k of FE in order 0 (read back from a first
    solve) puts the particular solution at its pole: the layer is NUMERIC, F_r NaN-filled, and every
    kernel exits normally."""
    N, L = 6, 8
    coef = hg(320, L)
    s = BRDFSolver([N], [L], [L], [3])
    s([2.0], [0.9], [coef])
    _, lam = s.plan.inspect(0, 0)
    real = lam[(lam.imag == 0) & (lam.real > 1.0)].real
    m0 = float(1.0 / np.sqrt(real[len(real) // 2]))
    r = BRDFSolver([N], [L], [L], [3], mu0=[0.5, m0])
    t, w, c = r.upload([2.0], [0.9], [coef])
    r.solve_device(t, w, c)
    torch.cuda.synchronize()
    assert r.status.cpu().tolist() == [binding.E_NUMERIC]
    assert torch.isnan(r.beams(0)).all() and torch.isnan(r.layer(0)).all()


def test_node_table_unchanged_by_beams_and_python_entry_point():
    """The node table of a plan with beams equals the one without, bit for bit; api.brdf_beam."""
    N, L, P = 7, 10, 5
    coef = hg(330, L)
    a = BRDFSolver([N], [L], [L], [P])
    Fa = a([1.3], [0.95], [coef])[0].clone()
    b = BRDFSolver([N], [L], [L], [P], mu0=[0.42])
    Fb = b([1.3], [0.95], [coef])[0]
    assert torch.equal(Fa, Fb)
    Fx = api.brdf_beam(1.3, 0.95, coef, N, L, P, [0.42, 0.77])
    assert tuple(Fx.shape) == (N, 2, P, 4, 4)
    assert err(Fx[:, 0].cpu().numpy(), particular.brdf_beam(coef, 1.3, 0.95, N, L, P, 0.42)) < TOL


def test_outgoing_directions_against_oracle():
    """Source-function integration (eq. 36-38) towards five arbitrary outgoing cosines, for two
    beams, against the oracle's reconstruction from the full 8N solution."""
    from oracle import reconstruct

    N, L, P = 8, 12, 7
    mu0, mo = [0.3137, 0.8123], [0.07, 0.21, 0.5, 0.83, 0.999]
    coef, tau, om = hg(340, L), 1.7, 0.93
    s = BRDFSolver([N], [L], [L], [P], mu0=mu0, mu_out=mo)
    s([tau], [om], [coef])
    Fb = s.beams(0).cpu().numpy()
    assert Fb.shape == (N + len(mo), len(mu0), P, 4, 4)
    for j, m0 in enumerate(mu0):
        Fo = reconstruct.brdf_beam_outgoing(coef, tau, om, N, L, P, m0, np.array(mo))
        assert err(Fb[N:, j], Fo) < TOL, (m0, err(Fb[N:, j], Fo))
        assert err(Fb[:N, j], particular.brdf_beam(coef, tau, om, N, L, P, m0)) < TOL


def test_outgoing_at_full_size_and_at_the_nodes():
    """N = 32, L = M = n_dphi = 64 (the particulate layer): towards directions placed exactly on
    Gauss nodes 3 and 17 the reconstruction gives the beams' node rows (the discrete-ordinate values);
    towards two off-node directions it matches the oracle."""
    from oracle import reconstruct

    w = workload("particulate")
    N, L, M, P = w.N[0], w.L[0], w.M[0], w.n_dphi[0]
    mu, _ = double_gauss(N)
    mu0 = [0.2371, 0.7519]
    mo = [mu[3], mu[17], 0.1234, 0.6789]
    s = BRDFSolver([N], [L], [M], [P], mu0=mu0, mu_out=mo)
    s([w.tau[0]], [w.omega[0]], [w.coef[0]])
    Fb = s.beams(0).cpu().numpy()
    for j in range(len(mu0)):
        assert err(Fb[N + 0, j], Fb[3, j]) < TOL
        assert err(Fb[N + 1, j], Fb[17, j]) < TOL
    Fo = reconstruct.brdf_beam_outgoing(w.coef[0], w.tau[0], w.omega[0], N, M, P, mu0[0], np.array(mo[2:]))
    assert err(Fb[N + 2:, 0], Fo) < TOL
