"""Convenience layer over the binding: torch tensors in, per-layer F_r tensors out.

torch is used only to hold device memory and to name the stream; every arithmetic step runs in
the HIP library.
"""

import numpy as np
import torch

from . import binding


def pack_coefficients(coefs):
    """Concatenate per-layer (6, L_l) coefficient arrays into the flat layout of vbrdf_solve."""
    return np.concatenate([np.ascontiguousarray(c, dtype=np.float64).ravel() for c in coefs])


class BRDFSolver:
    """Plan + device buffers for a fixed list of layer shapes.

    solver = BRDFSolver(N=[32], L=[64], M=[64], n_dphi=[64])
    F = solver(tau, omega, coefs)   # list of (N, N, n_dphi, 4, 4) float64 CUDA tensors
    """

    def __init__(self, N, L, M, n_dphi, device="cuda", precision=binding.PRECISION_FP64, flags=0, **plan_kw):
        if not torch.cuda.is_available():
            raise RuntimeError("BRDFSolver needs a ROCm GPU")
        self.device = torch.device(device)
        self.plan = binding.Plan(N, L, M, n_dphi, precision=precision, flags=flags, **plan_kw)
        sizes = self.plan.output_sizes()
        self.F = torch.empty(sum(sizes), dtype=torch.float64, device=self.device)
        self.status = torch.empty(self.plan.n_layers, dtype=torch.int32, device=self.device)
        self._views = []
        off = 0
        for n, p, s in zip(self.plan.N, self.plan.n_dphi, sizes):
            self._views.append(self.F[off:off + s].view(n, n, p, 4, 4))
            off += s
        self.F_beam = None
        self._beam_views = []
        if self.plan.mu0:
            nb, no = len(self.plan.mu0), len(self.plan.mu_out)
            self.F_beam = torch.empty(self.plan.beam_bytes() // 8, dtype=torch.float64, device=self.device)
            off = 0
            for n, p in zip(self.plan.N, self.plan.n_dphi):
                sz = (n + no) * nb * p * 16
                self._beam_views.append(self.F_beam[off:off + sz].view(n + no, nb, p, 4, 4))
                off += sz

    def upload(self, tau, omega, coefs):
        dev = self.device
        t = torch.as_tensor(np.asarray(tau, dtype=np.float64), device=dev)
        w = torch.as_tensor(np.asarray(omega, dtype=np.float64), device=dev)
        c = torch.as_tensor(pack_coefficients(coefs), device=dev)
        return t, w, c

    def solve_device(self, tau_d, omega_d, coef_d, stream=None, base_d=None):
        """Enqueue on `stream` (default: torch's current stream) with device-resident inputs
        (base_d: the base data of a plan with a reflecting base)."""
        s = torch.cuda.current_stream(self.device) if stream is None else stream
        if self.F_beam is not None:
            self.plan.solve_ex(tau_d, omega_d, coef_d, base_d, self.F, self.F_beam, self.status, s.cuda_stream)
        elif self.plan.below is None and self.plan.base == binding.BASE_BLACK:
            self.plan.solve(tau_d, omega_d, coef_d, self.F, self.status, s.cuda_stream)
        else:
            self.plan.solve_base(tau_d, omega_d, coef_d, base_d, self.F, self.status, s.cuda_stream)

    def check(self):
        st = self.status.cpu().numpy()
        bad = np.nonzero(st)[0]
        if len(bad):
            raise binding.VbrdfError(int(st[bad[0]]), f"layer(s) {bad.tolist()} failed with status {st[bad].tolist()}")

    def __call__(self, tau, omega, coefs, base=None):
        t, w, c = self.upload(tau, omega, coefs)
        b = None if base is None else torch.as_tensor(np.ascontiguousarray(base, dtype=np.float64).ravel(),
                                                      device=self.device)
        self.solve_device(t, w, c, base_d=b)
        torch.cuda.synchronize(self.device)
        self.check()
        return self._views

    def layer(self, i):
        return self._views[i]

    def beams(self, i):
        """(N + n_mu_out, n_mu0, n_dphi, 4, 4) view of layer i's off-node beam BRDF (plans built with
        mu0): outgoing Gauss nodes first, then the extra outgoing directions mu_out."""
        return self._beam_views[i]


class VbrdfFunction(torch.autograd.Function):
    """F_r (flat, all layers packed) as a differentiable function of tau, omega and the packed
    coefficients; the backward pass is the library's adjoint (vbrdf_backward).

    F = VbrdfFunction.apply(tau, omega, coef, solver)   # solver: BRDFSolver with save_for_backward
    """

    @staticmethod
    def forward(ctx, tau, omega, coef, solver):
        tau, omega, coef = (x.detach().contiguous() for x in (tau, omega, coef))
        solver.solve_device(tau, omega, coef)
        torch.cuda.synchronize(solver.device)
        solver.check()
        solver.version += 1
        ctx.version = solver.version
        ctx.solver = solver
        ctx.save_for_backward(tau, omega, coef)
        return solver.F.clone()

    @staticmethod
    def backward(ctx, gF):
        tau, omega, coef = ctx.saved_tensors
        solver = ctx.solver
        if solver.version != ctx.version:  # another forward ran since: recompute this one's state
            solver.solve_device(tau, omega, coef)
            solver.version += 1
            ctx.version = solver.version
        dtau, domega, dcoef = torch.empty_like(tau), torch.empty_like(omega), torch.empty_like(coef)
        s = torch.cuda.current_stream(solver.device)
        solver.plan.backward(tau, omega, coef, gF.contiguous(), dtau, domega, dcoef, s.cuda_stream)
        return dtau, domega, dcoef, None


class DifferentiableBRDF:
    """Layers of fixed shapes whose F_r is differentiable with respect to tau, omega and coef.

    model = DifferentiableBRDF(N=[32] * 64, L=[64] * 64, M=[32] * 64, n_dphi=[32] * 64)
    F = model(tau, omega, coef)   # tau, omega: (n_layers,), coef: packed (sum 6 L,) CUDA tensors
    loss(F).backward()            # gradients in tau.grad, omega.grad, coef.grad
    """

    def __init__(self, N, L, M, n_dphi, device="cuda"):
        self.solver = BRDFSolver(N, L, M, n_dphi, device=device, flags=binding.FLAG_SAVE_FOR_BACKWARD)
        self.solver.version = 0

    def __call__(self, tau, omega, coef):
        return VbrdfFunction.apply(tau, omega, coef, self.solver)

    def views(self, F):
        """Per-layer (N, N, n_dphi, 4, 4) views of a flat F."""
        out, off = [], 0
        for n, p in zip(self.solver.plan.N, self.solver.plan.n_dphi):
            out.append(F[off:off + n * n * p * 16].view(n, n, p, 4, 4))
            off += n * n * p * 16
        return out


class SpectralBRDF:
    """Spectral batching: n_materials x n_wavelengths layers of one shape solved in one plan (one
    launch per stage over every (material, wavelength, order) problem).

    sb = SpectralBRDF(n_materials=8, n_wavelengths=9, N=32, L=64, M=64, n_dphi=32)
    F = sb(tau, omega, coef)   # tau, omega: (n_materials, n_wavelengths); coef: (..., 6, L)
    F[a][w]                    # (N, N, n_dphi, 4, 4) tensor of material a at wavelength w
    """

    def __init__(self, n_materials, n_wavelengths, N, L, M, n_dphi, device="cuda", precision="fp64"):
        self.shape = (int(n_materials), int(n_wavelengths))
        n = self.shape[0] * self.shape[1]
        self.solver = BRDFSolver([N] * n, [L] * n, [M] * n, [n_dphi] * n, device=device,
                                 precision=_PRECISIONS[precision])

    def __call__(self, tau, omega, coef):
        A, W = self.shape
        tau = np.asarray(tau, dtype=np.float64).reshape(A * W)
        omega = np.asarray(omega, dtype=np.float64).reshape(A * W)
        coef = np.asarray(coef, dtype=np.float64).reshape(A * W, 6, -1)
        views = self.solver(tau, omega, list(coef))
        return [[views[a * W + w] for w in range(W)] for a in range(A)]


_PRECISIONS = {"fp64": binding.PRECISION_FP64, "fp32_refined": binding.PRECISION_FP32_REFINED}
_BASES = {"black": binding.BASE_BLACK, "lambertian": binding.BASE_LAMBERTIAN, "mueller": binding.BASE_MUELLER}


def brdf_beam(tau, omega, coef, N, M, n_dphi, mu0, mu_out=None, precision="fp64", device="cuda"):
    """BRDF of one layer for incidence at arbitrary cosines mu0 (a sequence, each in (0, 1]) towards
    the Gauss nodes and then towards the arbitrary outgoing cosines mu_out: a
    (N + len(mu_out), len(mu0), n_dphi, 4, 4) float64 tensor (outgoing direction, incident j,
    azimuth difference 2 pi k / n_dphi, Mueller row, column)."""
    L = np.asarray(coef).shape[1]
    s = BRDFSolver([N], [L], [M], [n_dphi], device=device, precision=_PRECISIONS[precision], mu0=mu0,
                   mu_out=mu_out)
    s([tau], [omega], [coef])
    return s.beams(0).clone()


def stack_brdf(tau, omega, coef, N, M, n_dphi, base="black", rho=0.0, Rb=None, precision="fp64", device="cuda"):
    """BRDF of a stack of layers (listed from the top down) over a base, on the Gauss-node grid.

    tau, omega: sequences over the layers; coef: sequence of (6, L_l) arrays; every layer shares N,
    M and n_dphi. base: "black", "lambertian" (albedo rho) or "mueller" (Rb: (M, 4N, 4N) per-order
    base blocks Rb^m[(i, r), (j, p)], see VBRDF_BASE_MUELLER). Returns the (N, N, n_dphi, 4, 4) F_r
    of the whole stack (the top layer's output).
    """
    nl = len(tau)
    below = list(range(1, nl)) + [-1]
    Ls = [np.asarray(c).shape[1] for c in coef]
    s = BRDFSolver([N] * nl, Ls, [M] * nl, [n_dphi] * nl, device=device, precision=_PRECISIONS[precision],
                   below=below, base=_BASES[base])
    data = None
    if base == "lambertian":
        data = np.full(nl, float(rho))
    elif base == "mueller":
        data = np.asarray(Rb, dtype=np.float64)
    return s(tau, omega, coef, base=data)[0].clone()


def brdf(tau, omega, coef, N, M, n_dphi, precision="fp64", device="cuda"):
    """Polarized BRDF Mueller matrices of one or more layers on the Gauss-node grid.

    tau, omega: scalars or sequences (one per layer); coef: a (6, L) array or a sequence of them;
    N, M, n_dphi: ints or sequences. Returns a (N, N, n_dphi, 4, 4) float64 tensor on `device`
    (outgoing node i, incident node q, azimuth difference 2 pi k / n_dphi, Mueller row, column),
    or a list of them for several layers. Raises VbrdfError when a layer fails.
    """
    many = np.ndim(tau) > 0
    taus = list(np.atleast_1d(np.asarray(tau, dtype=np.float64)))
    oms = list(np.atleast_1d(np.asarray(omega, dtype=np.float64)))
    coefs = list(coef) if many else [coef]
    nl = len(taus)
    per = lambda v: [int(x) for x in v] if np.ndim(v) > 0 else [int(v)] * nl
    Ls = [np.asarray(c).shape[1] for c in coefs]
    s = BRDFSolver(per(N), Ls, per(M), per(n_dphi), device=device, precision=_PRECISIONS[precision])
    out = [v.clone() for v in s(taus, oms, coefs)]
    return out if many else out[0]
