"""The allocation-free entry point against the plan-based one, through the C-ABI.

Two calls in a row on one GPU (the second with a smaller layer, so the shared static array holds
the first call's larger contents) must each give the plan-based result for the same inputs, to
the FP64 parity bar, and a layer too large for the static array must be refused with NOMEM
before anything is enqueued.
"""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1707_05882_amd import binding
from paper_1707_05882_amd.api import pack_coefficients
from workloads.layers import hg_like_coefficients

pytestmark = pytest.mark.gpu
TOL = 1e-10


def _layer(seed, N, L, M, P, tau, omega):
    coef = hg_like_coefficients(np.random.default_rng(seed), L)[0]
    return dict(N=N, L=L, M=M, P=P, tau=tau, omega=omega, coef=coef)


def _dev(l):
    d = "cuda"
    return (torch.tensor([l["tau"]], dtype=torch.float64, device=d),
            torch.tensor([l["omega"]], dtype=torch.float64, device=d),
            torch.as_tensor(pack_coefficients([l["coef"]]), device=d))


def _plan_solve(l, stream):
    plan = binding.Plan([l["N"]], [l["L"]], [l["M"]], [l["P"]])
    t, w, c = _dev(l)
    F = torch.empty(plan.output_bytes() // 8, dtype=torch.float64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    plan.solve(t, w, c, F, st, stream.cuda_stream)
    stream.synchronize()
    assert st.item() == 0
    return F


def test_noalloc_matches_plan_two_calls():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    stream = torch.cuda.Stream()
    big = _layer(71, N=32, L=40, M=36, P=12, tau=5.0, omega=0.97)
    small = _layer(72, N=9, L=11, M=7, P=5, tau=0.7, omega=0.8)
    for l in (big, small):
        ref = _plan_solve(l, stream)
        t, w, c = _dev(l)
        F = torch.full_like(ref, float("nan"))
        st = torch.full((1,), -99, dtype=torch.int32, device="cuda")
        with torch.cuda.stream(stream):
            binding.solve_noalloc(l["N"], l["L"], l["M"], l["P"], t, w, c, F, st, stream.cuda_stream)
        stream.synchronize()
        assert st.item() == 0
        Fr, Fn = ref.cpu().numpy(), F.cpu().numpy()
        scale = np.abs(Fr.reshape(l["N"], l["N"], l["P"], 4, 4)[..., 0, 0]).max()
        assert np.isfinite(Fn).all()
        assert np.abs(Fn - Fr).max() / scale < TOL, l["N"]


def test_noalloc_refuses_oversized_layer():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    l = _layer(73, N=128, L=256, M=256, P=4, tau=1.0, omega=0.9)
    t, w, c = _dev(l)
    F = torch.empty(1, dtype=torch.float64, device="cuda")
    st = torch.empty(1, dtype=torch.int32, device="cuda")
    with pytest.raises(binding.VbrdfError) as e:
        binding.solve_noalloc(128, 256, 256, 4, t, w, c, F, st, torch.cuda.current_stream().cuda_stream)
    assert e.value.code == binding.E_NOMEM
