"""The FP32-refined path (boundary factorisations and right divisions in FP32, recovered by
iterative refinement against FP64 residuals) against the FP64 oracle, through the C-ABI.

Gate (metric G18 for the refined path): max |F - F_oracle| / max |F_oracle,II| <= 1e-6 per layer.
The refinement is expected to recover the FP64 result (the boundary matrices are well
conditioned), so the tests also report, and bound loosely, the distance to the FP64 GPU path.
"""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dom
from paper_1707_05882_amd import binding
from paper_1707_05882_amd.api import BRDFSolver
from workloads import workload
from workloads.layers import hg_like_coefficients

pytestmark = pytest.mark.gpu
TOL_REFINED = 1e-6
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
R32 = binding.PRECISION_FP32_REFINED


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    binding.load()


def hg(seed, L):
    return hg_like_coefficients(np.random.default_rng(seed), L)[0]


def _solve(w, **kw):
    s = BRDFSolver(w.N, w.L, w.M, w.n_dphi, **kw)
    t, om, c = s.upload(w.tau, w.omega, w.coef)
    s.solve_device(t, om, c)
    torch.cuda.synchronize()
    return s


@pytest.mark.parametrize("name", ["particulate", "large"])
def test_refined_single_layer_workloads(name):
    """Particulate (N = 32) and large (N = 128) workloads: every node pair at the stored azimuths."""
    g = np.load(os.path.join(GOLDEN, f"{name}_sample.npz"))
    w = workload(name)
    s = _solve(w, precision=R32)
    assert s.status.cpu().tolist() == [0]
    F = s.layer(0)[:, :, [int(k) for k in g["az"]]].cpu().numpy()
    err = np.abs(F - g["F"]).max() / float(g["scale"])
    print(f"{name}: refined err vs oracle {err:.3e}")
    assert err < TOL_REFINED


def test_refined_batched_one_layer_per_N():
    g = np.load(os.path.join(GOLDEN, "batched_sample.npz"))
    w = workload("batched")
    s = _solve(w, precision=R32)
    assert (s.status.cpu().numpy() == 0).all()
    worst = 0.0
    for i in (int(v) for v in g["layers"]):
        F = s.layer(i)[:, :, [int(k) for k in g[f"az{i}"]]].cpu().numpy()
        worst = max(worst, np.abs(F - g[f"F{i}"]).max() / float(g[f"scale{i}"]))
    print(f"batched: refined err vs oracle {worst:.3e}")
    assert worst < TOL_REFINED


def test_refined_matches_fp64_path_on_uneven_layers():
    layers = [(3, 6, 5, 0.3, 0.7, hg(91, 6)), (13, 20, 11, 4.0, 0.99, hg(92, 20)), (21, 30, 7, 25.0, 0.95, hg(93, 30))]
    N = [l[0] for l in layers]
    L = [l[1] for l in layers]
    P = [l[2] for l in layers]
    args = ([l[3] for l in layers], [l[4] for l in layers], [l[5] for l in layers])
    F64 = [f.clone() for f in BRDFSolver(N, L, L, P)(*args)]
    F32 = BRDFSolver(N, L, L, P, precision=R32)(*args)
    for l, a, b in zip(layers, F64, F32):
        scale = a[..., 0, 0].abs().max().item()
        assert (a - b).abs().max().item() / scale < 1e-9, l[0]
        Fo = dom.brdf(l[5], l[3], l[4], l[0], l[1], l[2])
        assert np.abs(b.cpu().numpy() - Fo).max() / np.abs(Fo[..., 0, 0]).max() < TOL_REFINED


def test_unrefined_fp32_falls_back_to_fp64():
    """With no correction steps the FP32 solve misses the residual test, so every side is redone in
    FP64: the result equals the FP64 path's."""
    coef = hg(94, 12)
    args = ([2.0], [0.95], [coef])
    F64 = BRDFSolver([9], [12], [12], [6])(*args)[0].clone()
    s = BRDFSolver([9], [12], [12], [6], precision=R32, refine_steps=-1)
    F = s(*args)[0]
    assert torch.equal(F, F64)


def test_disabled_fallback_reports_nonconverged():
    coef = hg(95, 12)
    s = BRDFSolver([9, 5], [12, 6], [12, 6], [6, 4], precision=R32, refine_steps=-1,
                   flags=binding.FLAG_DISABLE_FP64_FALLBACK)
    t, w, c = s.upload([2.0, 1.0], [0.95, 0.9], [coef, hg(96, 6)])
    s.solve_device(t, w, c)
    torch.cuda.synchronize()
    assert s.status.cpu().tolist() == [binding.E_NONCONVERGED] * 2
    assert torch.isnan(s.layer(0)).all() and torch.isnan(s.layer(1)).all()
    with pytest.raises(binding.VbrdfError) as e:
        s.check()
    assert e.value.code == binding.E_NONCONVERGED
