"""Host-side checks of the C-ABI library (no GPU needed): loading, exported symbols, host-only
entry points and argument validation that fails before any device call."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1707_05882_amd import binding
from oracle.quadrature import double_gauss

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "vbrdf.h")


def declared_symbols():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(vbrdf_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    syms = declared_symbols()
    assert len(syms) >= 10
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(binding.EXPORTED)


def test_abi_version():
    assert binding.abi_version() == binding.ABI_VERSION == 3


@pytest.mark.parametrize("N", [1, 2, 3, 8, 32, 64, 128])
def test_gauss_nodes_match_library_rule(N):
    mu, al = binding.gauss_nodes(N)
    mo, ao = double_gauss(N)
    assert np.all(np.diff(mu) > 0)
    assert np.abs(mu - mo).max() < 1e-15
    assert np.abs(al - ao).max() < 1e-14 * max(1.0, ao.max() * 10)
    assert abs(al.sum() - 1.0) < 1e-14
    for k in range(2 * N):
        assert abs(np.sum(al * mu ** k) - 1.0 / (k + 1)) < 1e-13


def test_gauss_nodes_rejects_bad_order():
    with pytest.raises(binding.VbrdfError) as e:
        binding.gauss_nodes(0)
    assert e.value.code == binding.E_INVALID


@pytest.mark.parametrize("kw,code", [
    (dict(N=[8], L=[4], M=[5], n_dphi=[8]), binding.E_INVALID),       # M > L
    (dict(N=[0], L=[4], M=[2], n_dphi=[8]), binding.E_INVALID),       # N < 1
    (dict(N=[8], L=[4], M=[2], n_dphi=[0]), binding.E_INVALID),       # n_dphi < 1
    (dict(N=[129], L=[4], M=[2], n_dphi=[8]), binding.E_UNSUPPORTED),  # N above the maximum
    (dict(N=[8], L=[600], M=[600], n_dphi=[8]), binding.E_UNSUPPORTED),  # M above the maximum
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], precision=7), binding.E_UNSUPPORTED),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], flags=64), binding.E_UNSUPPORTED),  # unknown flag
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], flags=3), binding.E_UNSUPPORTED),  # timing + graph
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], flags=16), binding.E_INVALID),  # FP64 fallback flag on FP64
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], qr_sweep_cap=-1), binding.E_INVALID),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], refine_steps=1), binding.E_INVALID),  # refine steps on FP64
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], precision=1, refine_steps=-2), binding.E_INVALID),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], workspace=0x1000 + 8, workspace_bytes=1 << 30), binding.E_INVALID),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], workspace_bytes=4096), binding.E_INVALID),  # bytes, no pointer
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], workspace=0x100000, workspace_bytes=256), binding.E_NOMEM),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], workspace_cap_bytes=1024), binding.E_NOMEM),
    # stacks and bases
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], base=3), binding.E_UNSUPPORTED),  # unknown base kind
    (dict(N=[8, 8], L=[4, 4], M=[2, 2], n_dphi=[8, 8], below=[2, -1]), binding.E_INVALID),  # out of range
    (dict(N=[8, 8], L=[4, 4], M=[2, 2], n_dphi=[8, 8], below=[0, -1]), binding.E_INVALID),  # on itself
    (dict(N=[8] * 3, L=[4] * 3, M=[2] * 3, n_dphi=[8] * 3, below=[2, 2, -1]), binding.E_INVALID),  # two on one
    (dict(N=[8] * 3, L=[4] * 3, M=[2] * 3, n_dphi=[8] * 3, below=[1, 2, 1]), binding.E_INVALID),  # cycle
    (dict(N=[8, 6], L=[4, 4], M=[2, 2], n_dphi=[8, 8], below=[1, -1]), binding.E_INVALID),  # N differs
    (dict(N=[8, 8], L=[4, 4], M=[2, 3], n_dphi=[8, 8], below=[1, -1]), binding.E_INVALID),  # M differs
    (dict(N=[8, 8], L=[4, 4], M=[2, 2], n_dphi=[8, 8], below=[1, -1], flags=8), binding.E_UNSUPPORTED),
    (dict(N=[8, 8], L=[4, 4], M=[2, 2], n_dphi=[8, 8], below=[1, -1], flags=4), binding.E_UNSUPPORTED),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], base=1, flags=8), binding.E_UNSUPPORTED),  # base + adjoint
    (dict(N=[8] * 65, L=[4] * 65, M=[2] * 65, n_dphi=[8] * 65, below=list(range(1, 65)) + [-1]),
     binding.E_UNSUPPORTED),  # deeper than 64 layers
    # off-node beams
    (dict(N=[4], L=[4], M=[2], n_dphi=[8], mu0=[0.1, 0.2, 0.3, 0.4, 0.5]), binding.E_INVALID),  # n_mu0 > N
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], mu0=[0.5, 0.0]), binding.E_INVALID),  # mu0 = 0
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], mu0=[1.5]), binding.E_INVALID),       # mu0 > 1
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], mu0=[float("nan")]), binding.E_INVALID),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], mu0=[0.5], flags=8), binding.E_UNSUPPORTED),  # beams + adjoint
    (dict(N=[8, 8], L=[4, 4], M=[2, 2], n_dphi=[8, 8], mu0=[0.5], below=[1, -1]), binding.E_UNSUPPORTED),
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], mu0=[0.5], base=1), binding.E_UNSUPPORTED),
    (dict(N=[128], L=[4], M=[2], n_dphi=[8], mu0=[0.5] * 65), binding.E_INVALID),  # above 64 beams
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], mu_out=[0.5]), binding.E_INVALID),  # outgoing without beams
    (dict(N=[8], L=[4], M=[2], n_dphi=[8], mu0=[0.5], mu_out=[0.0]), binding.E_INVALID),
    (dict(N=[2], L=[4], M=[2], n_dphi=[8], mu0=[0.5], mu_out=[0.1, 0.2, 0.3]), binding.E_INVALID),  # > N
])
def test_plan_validation(kw, code):
    with pytest.raises(binding.VbrdfError) as e:
        binding.Plan(**kw)
    assert e.value.code == code
    assert binding.last_error() != ""


def test_null_plan_calls_are_rejected():
    lib = binding.load()
    assert lib.vbrdf_solve(None, None, None, None, None, None, None) == binding.E_INVALID
    assert lib.vbrdf_solve_base(None, None, None, None, None, None, None, None) == binding.E_INVALID
    assert lib.vbrdf_plan_base_bytes(None) == 0
    assert lib.vbrdf_solve_ex(None, None, None, None, None, None, None, None, None) == binding.E_INVALID
    assert lib.vbrdf_plan_beam_bytes(None) == 0
    assert lib.vbrdf_plan_destroy(None) == binding.OK
    assert lib.vbrdf_plan_output_bytes(None) == 0
    assert lib.vbrdf_stage_name(0).decode() == "validate"
    assert lib.vbrdf_stage_name(15).decode() == "stack"
    assert lib.vbrdf_stage_name(16).decode() == "synth"
    assert lib.vbrdf_stage_name(17) is None
    assert lib.vbrdf_stage_name(99) is None


def test_workspace_query_matches_the_item_blocks():
    """Eight n x n matrices, ten n-vectors and the Legendre table per (layer, order), 256-byte
    aligned: the figure a caller-owned workspace must reach."""
    N, L, M = [8, 5], [6, 9], [4, 9]
    got = binding.workspace_query(N, L, M, [3, 4])
    want = 0
    for n_, l_, m_ in zip(N, L, M):
        n = 4 * n_
        blk = 8 * n * n + 10 * n + l_ * n_ * 3
        want += m_ * ((blk + 31) // 32 * 32) * 8
    assert got == want
    with pytest.raises(binding.VbrdfError) as e:
        binding.workspace_query([8], [4], [5], [8])
    assert e.value.code == binding.E_INVALID


def test_noalloc_argument_checks_before_any_device_call():
    lib = binding.load()
    fake = 0x100000
    args = lambda N, L, M, P: (N, L, M, P, fake, fake, fake, fake, fake, None)
    assert lib.vbrdf_solve_noalloc(8, 4, 2, 8, None, fake, fake, fake, fake, None) == binding.E_INVALID
    assert lib.vbrdf_solve_noalloc(*args(0, 4, 2, 8)) == binding.E_INVALID
    assert lib.vbrdf_solve_noalloc(*args(8, 4, 5, 8)) == binding.E_INVALID
    assert lib.vbrdf_solve_noalloc(*args(129, 4, 2, 8)) == binding.E_UNSUPPORTED
    assert lib.vbrdf_solve_noalloc(*args(128, 256, 256, 8)) == binding.E_NOMEM
    assert "scratch" in binding.last_error()


def test_radiance_and_inspect_reject_a_null_plan():
    lib = binding.load()
    i0 = (ctypes.c_double * 4)(1.0, 0.0, 0.0, 0.0)
    assert lib.vbrdf_radiance(None, None, 0, 0, 0.0, i0, None, None) == binding.E_INVALID
    assert lib.vbrdf_plan_inspect(None, 0, 0, None, None, None, None, None) == binding.E_INVALID
    assert lib.vbrdf_plan_stage_times(None, None, 0) == binding.E_INVALID


def test_tuning_calls_reject_bad_arguments():
    lib = binding.load()
    t = binding.Tuning(0, 8)
    assert lib.vbrdf_plan_get_tuning(None, ctypes.byref(t)) == binding.E_INVALID
    assert lib.vbrdf_plan_set_tuning(None, ctypes.byref(t)) == binding.E_INVALID
    assert lib.vbrdf_plan_autotune(None, None, None, None, None, None, None, None) == binding.E_INVALID
    assert lib.vbrdf_backward(None, None, None, None, None, None, None, None, None) == binding.E_INVALID
