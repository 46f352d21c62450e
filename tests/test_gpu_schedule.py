"""Scheduling and tile choices on an uneven batch, through the C-ABI: the eigensolver schedules (plan
order, longest first, persistent queue) give the same F_r bit for bit (every problem runs the same
arithmetic); the right-division tile shapes (4 and 8 rows split each dot product over a different number
of lanes, 16 rows solves by blocks on the matrix cores) sum in different orders, so they agree to
rounding and each meets the oracle gate; the autotuner keeps a valid choice."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dom
from paper_1707_05882_amd import binding
from paper_1707_05882_amd.api import BRDFSolver
from workloads.layers import hg_like_coefficients

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a ROCm device")
    binding.load()


def _batch():
    rng = np.random.default_rng(111)
    layers = []
    for k, N in enumerate([6, 40, 13, 33, 3, 21]):  # systems of 24 .. 160 rows, some above the LDS size
        L = min(2 * N, 24)
        coef = hg_like_coefficients(rng, L)[0]
        layers.append((N, L, min(L, 10), 5, 0.5 + k, 0.8 + 0.03 * k, coef))
    return layers


@pytest.mark.parametrize("graph", [False, True])
def test_every_schedule_and_tile_gives_the_same_result(graph):
    layers = _batch()
    N, L, M, P = ([l[k] for l in layers] for k in range(4))
    s = BRDFSolver(N, L, M, P, flags=binding.FLAG_GRAPH if graph else 0)
    t, w, c = s.upload([l[4] for l in layers], [l[5] for l in layers], [l[6] for l in layers])
    stream = torch.cuda.Stream()
    Fo = [dom.brdf(l[6], l[4], l[5], l[0], l[2], l[3]) for l in layers]
    ref = None
    for rows in (4, 8, 16):
        ref_rows = None
        for sched in (binding.EIGEN_PLAN_ORDER, binding.EIGEN_LONGEST_FIRST, binding.EIGEN_PERSISTENT):
            s.plan.set_tuning(sched, rows)
            assert s.plan.get_tuning() == {"eigen_schedule": sched, "trsm_rows": rows}
            s.F.fill_(float("nan"))
            torch.cuda.synchronize()
            with torch.cuda.stream(stream):
                s.solve_device(t, w, c, stream=stream)
            stream.synchronize()
            assert (s.status.cpu().numpy() == 0).all()
            if ref_rows is None:
                for i, l in enumerate(layers):
                    assert np.abs(s.layer(i).cpu().numpy() - Fo[i]).max() < 1e-10 * np.abs(Fo[i][..., 0, 0]).max()
            if ref is None:
                ref = s.F.clone()
            if ref_rows is None:
                ref_rows = s.F.clone()
                # blocked and lane-split sums differ in order: a few 1e-12 of max |F| here
                assert (s.F - ref).abs().max().item() < 1e-11 * ref.abs().max().item(), rows
            else:
                assert torch.equal(s.F, ref_rows), (sched, rows)


def test_autotune_picks_a_valid_choice():
    layers = _batch()
    N, L, M, P = ([l[k] for l in layers] for k in range(4))
    s = BRDFSolver(N, L, M, P)
    t, w, c = s.upload([l[4] for l in layers], [l[5] for l in layers], [l[6] for l in layers])
    ch = s.plan.autotune(t, w, c, s.F, s.status, torch.cuda.current_stream().cuda_stream)
    assert ch["eigen_schedule"] in (0, 1, 2) and ch["trsm_rows"] in (4, 8, 16)
    assert s.plan.get_tuning() == ch
    F1 = s.F.clone()
    s.solve_device(t, w, c)
    torch.cuda.synchronize()
    assert torch.equal(F1, s.F)
    with pytest.raises(binding.VbrdfError):
        s.plan.set_tuning(5, 8)
    with pytest.raises(binding.VbrdfError):
        s.plan.set_tuning(1, 12)
