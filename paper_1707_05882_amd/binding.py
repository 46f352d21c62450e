"""ctypes binding of the C-ABI in include/vbrdf.h (argument marshalling only).

Every entry point keeps the name of the C function without the ``vbrdf_`` prefix. Device buffers
are passed as raw pointers (torch tensors are accepted and their ``data_ptr()`` is used); the
stream is a hipStream_t handle as an integer (``torch.cuda.current_stream().cuda_stream``).
The library is loaded from this directory; if it has not been built, loading raises instead of
falling back to anything else.
"""

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvbrdf.so")

OK = 0
E_INVALID = -1
E_UNSUPPORTED = -2
E_NOMEM = -3
E_DEVICE = -4
E_NUMERIC = -5
E_NONCONVERGED = -6
PRECISION_FP64 = 0
PRECISION_FP32_REFINED = 1
FLAG_STAGE_TIMING = 1
FLAG_GRAPH = 2
FLAG_EMIT_TRANSMISSION = 4
FLAG_SAVE_FOR_BACKWARD = 8
FLAG_DISABLE_FP64_FALLBACK = 16
ABI_VERSION = 3
BASE_BLACK = 0
BASE_LAMBERTIAN = 1
BASE_MUELLER = 2
MAX_N = 128
NOALLOC_SCRATCH_BYTES = 80 << 20

STATUS_NAMES = {OK: "OK", E_INVALID: "INVALID", E_UNSUPPORTED: "UNSUPPORTED", E_NOMEM: "NOMEM",
                E_DEVICE: "DEVICE", E_NUMERIC: "NUMERIC", E_NONCONVERGED: "NONCONVERGED"}

EXPORTED = (
    "vbrdf_abi_version", "vbrdf_last_error", "vbrdf_gauss_nodes", "vbrdf_plan_create",
    "vbrdf_workspace_query", "vbrdf_plan_destroy", "vbrdf_plan_output_bytes", "vbrdf_plan_workspace_bytes",
    "vbrdf_solve", "vbrdf_plan_inspect", "vbrdf_radiance", "vbrdf_plan_stage_times", "vbrdf_stage_name",
    "vbrdf_solve_noalloc", "vbrdf_backward", "vbrdf_plan_get_tuning", "vbrdf_plan_set_tuning",
    "vbrdf_plan_autotune", "vbrdf_solve_base", "vbrdf_plan_base_bytes", "vbrdf_solve_ex",
    "vbrdf_plan_beam_bytes",
)
MAX_BEAMS = 64
EIGEN_PLAN_ORDER = 0
EIGEN_LONGEST_FIRST = 1
EIGEN_PERSISTENT = 2


class Tuning(ctypes.Structure):
    _fields_ = [("eigen_schedule", ctypes.c_int32), ("trsm_rows", ctypes.c_int32)]


class VbrdfError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"vbrdf {STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class PlanDesc(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("n_layers", ctypes.c_int32),
        ("N", ctypes.POINTER(ctypes.c_int32)),
        ("L", ctypes.POINTER(ctypes.c_int32)),
        ("M", ctypes.POINTER(ctypes.c_int32)),
        ("n_dphi", ctypes.POINTER(ctypes.c_int32)),
        ("precision", ctypes.c_int32),
        ("flags", ctypes.c_int32),
        ("workspace_cap_bytes", ctypes.c_uint64),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64),
        ("qr_sweep_cap", ctypes.c_int32),
        ("refine_steps", ctypes.c_int32),
        ("below", ctypes.POINTER(ctypes.c_int32)),
        ("base", ctypes.c_int32),
        ("n_mu0", ctypes.c_int32),
        ("mu0", ctypes.POINTER(ctypes.c_double)),
        ("n_mu_out", ctypes.c_int32),
        ("mu_out", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def load():
    """Load libvbrdf.so (raises OSError if it is missing or cannot be loaded)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise OSError(f"{LIB_PATH} is not built; build it with paper_1707_05882_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    i32, vp, dp = ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)
    L.vbrdf_abi_version.restype = i32
    L.vbrdf_abi_version.argtypes = []
    L.vbrdf_last_error.restype = ctypes.c_char_p
    L.vbrdf_last_error.argtypes = []
    L.vbrdf_gauss_nodes.restype = i32
    L.vbrdf_gauss_nodes.argtypes = [i32, dp, dp]
    L.vbrdf_plan_create.restype = i32
    L.vbrdf_plan_create.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(vp)]
    L.vbrdf_workspace_query.restype = i32
    L.vbrdf_workspace_query.argtypes = [ctypes.POINTER(PlanDesc), ctypes.POINTER(ctypes.c_uint64)]
    L.vbrdf_plan_destroy.restype = i32
    L.vbrdf_plan_destroy.argtypes = [vp]
    L.vbrdf_plan_output_bytes.restype = ctypes.c_size_t
    L.vbrdf_plan_output_bytes.argtypes = [vp]
    L.vbrdf_plan_workspace_bytes.restype = ctypes.c_size_t
    L.vbrdf_plan_workspace_bytes.argtypes = [vp]
    L.vbrdf_solve.restype = i32
    L.vbrdf_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.vbrdf_plan_inspect.restype = i32
    L.vbrdf_plan_inspect.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    L.vbrdf_radiance.restype = i32
    L.vbrdf_radiance.argtypes = [vp, vp, i32, i32, ctypes.c_double, dp, vp, vp]
    L.vbrdf_plan_stage_times.restype = i32
    L.vbrdf_plan_stage_times.argtypes = [vp, ctypes.POINTER(ctypes.c_float), i32]
    L.vbrdf_stage_name.restype = ctypes.c_char_p
    L.vbrdf_stage_name.argtypes = [i32]
    L.vbrdf_solve_noalloc.restype = i32
    L.vbrdf_solve_noalloc.argtypes = [i32, i32, i32, i32, vp, vp, vp, vp, vp, vp]
    L.vbrdf_backward.restype = i32
    L.vbrdf_backward.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.vbrdf_plan_get_tuning.restype = i32
    L.vbrdf_plan_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.vbrdf_plan_set_tuning.restype = i32
    L.vbrdf_plan_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.vbrdf_plan_autotune.restype = i32
    L.vbrdf_plan_autotune.argtypes = [vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(Tuning)]
    L.vbrdf_solve_base.restype = i32
    L.vbrdf_solve_base.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    L.vbrdf_plan_base_bytes.restype = ctypes.c_size_t
    L.vbrdf_plan_base_bytes.argtypes = [vp]
    L.vbrdf_solve_ex.restype = i32
    L.vbrdf_solve_ex.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.vbrdf_plan_beam_bytes.restype = ctypes.c_size_t
    L.vbrdf_plan_beam_bytes.argtypes = [vp]
    if L.vbrdf_abi_version() != ABI_VERSION:
        raise OSError("libvbrdf.so ABI version mismatch")
    _lib = L
    return L


def _check(code):
    if code != OK:
        raise VbrdfError(code, load().vbrdf_last_error().decode())


def _ptr(x):
    if x is None:
        return None
    if hasattr(x, "data_ptr"):
        return ctypes.c_void_p(x.data_ptr())
    if isinstance(x, np.ndarray):
        return ctypes.c_void_p(x.ctypes.data)
    return ctypes.c_void_p(int(x))


def abi_version():
    return load().vbrdf_abi_version()


def last_error():
    return load().vbrdf_last_error().decode()


def gauss_nodes(N):
    """Host call: (mu, alpha) double-Gauss nodes and weights, ascending."""
    mu = np.zeros(max(N, 0))
    al = np.zeros(max(N, 0))
    dp = ctypes.POINTER(ctypes.c_double)
    _check(load().vbrdf_gauss_nodes(int(N), mu.ctypes.data_as(dp), al.ctypes.data_as(dp)))
    return mu, al


def solve_noalloc(N, L, M, n_dphi, tau, omega, coef, F_r, layer_status, stream=0):
    """One layer without device allocation (the library's static scratch array); device pointers."""
    _check(load().vbrdf_solve_noalloc(int(N), int(L), int(M), int(n_dphi), _ptr(tau), _ptr(omega), _ptr(coef),
                                      _ptr(F_r), _ptr(layer_status), ctypes.c_void_p(int(stream))))


def _as_list(v):
    return [int(x) for x in (v if hasattr(v, "__len__") else [v])]


class _Desc:
    """Keeps a PlanDesc and the shape arrays it points to alive together."""

    def __init__(self, N, L, M, n_dphi, precision, flags, workspace_cap_bytes, workspace, workspace_bytes,
                 qr_sweep_cap, refine_steps=0, below=None, base=BASE_BLACK, mu0=None, mu_out=None):
        self.N, self.L, self.M, self.n_dphi = (_as_list(v) for v in (N, L, M, n_dphi))
        nl = len(self.N)
        if not (len(self.L) == len(self.M) == len(self.n_dphi) == nl):
            raise ValueError("shape lists differ in length")
        arr = lambda v: (ctypes.c_int32 * nl)(*v)
        self.keep = [arr(self.N), arr(self.L), arr(self.M), arr(self.n_dphi)]
        ws = _ptr(workspace) if workspace is not None else None
        bl = None
        if below is not None:
            below = [int(b) for b in below]
            if len(below) != nl:
                raise ValueError("below needs one entry per layer")
            bl = arr(below)
            self.keep.append(bl)
        m0 = None
        n_mu0 = 0
        if mu0 is not None:
            vals = [float(x) for x in np.atleast_1d(mu0)]
            n_mu0 = len(vals)
            m0 = (ctypes.c_double * max(n_mu0, 1))(*vals)
            self.keep.append(m0)
        mo = None
        n_mu_out = 0
        if mu_out is not None:
            vals = [float(x) for x in np.atleast_1d(mu_out)]
            n_mu_out = len(vals)
            mo = (ctypes.c_double * max(n_mu_out, 1))(*vals)
            self.keep.append(mo)
        dp = ctypes.POINTER(ctypes.c_double)
        self.desc = PlanDesc(ABI_VERSION, nl, *self.keep[:4], int(precision), int(flags), int(workspace_cap_bytes),
                             ws, int(workspace_bytes), int(qr_sweep_cap), int(refine_steps), bl, int(base),
                             n_mu0, ctypes.cast(m0, dp) if m0 is not None else None,
                             n_mu_out, ctypes.cast(mo, dp) if mo is not None else None)
        self.n_layers = nl


def workspace_query(N, L, M, n_dphi, precision=PRECISION_FP64, flags=0, below=None, base=BASE_BLACK, mu0=None,
                    mu_out=None):
    """Bytes of device workspace a plan of these shapes needs (host call)."""
    d = _Desc(N, L, M, n_dphi, precision, flags, 0, None, 0, 0, 0, below, base, mu0, mu_out)
    out = ctypes.c_uint64()
    _check(load().vbrdf_workspace_query(ctypes.byref(d.desc), ctypes.byref(out)))
    return int(out.value)


class Plan:
    """Owns a vbrdf_plan. Shapes are per-layer lists (or scalars for one layer)."""

    def __init__(self, N, L, M, n_dphi, precision=PRECISION_FP64, flags=0, workspace_cap_bytes=0,
                 workspace=None, workspace_bytes=0, qr_sweep_cap=0, refine_steps=0, below=None, base=BASE_BLACK,
                 mu0=None, mu_out=None):
        d = _Desc(N, L, M, n_dphi, precision, flags, workspace_cap_bytes, workspace, workspace_bytes, qr_sweep_cap,
                  refine_steps, below, base, mu0, mu_out)
        self.mu0 = None if mu0 is None else [float(x) for x in np.atleast_1d(mu0)]
        self.mu_out = [] if mu_out is None else [float(x) for x in np.atleast_1d(mu_out)]
        self.below = None if below is None else [int(b) for b in below]
        self.base = int(base)
        self.N, self.L, self.M, self.n_dphi = d.N, d.L, d.M, d.n_dphi
        self.flags = int(flags)
        self.precision = int(precision)
        self._workspace = workspace  # the caller's buffer must outlive the plan
        h = ctypes.c_void_p()
        _check(load().vbrdf_plan_create(ctypes.byref(d.desc), ctypes.byref(h)))
        self._h = h
        self.n_layers = d.n_layers

    @property
    def handle(self):
        return self._h

    def output_bytes(self):
        return load().vbrdf_plan_output_bytes(self._h)

    def workspace_bytes(self):
        return load().vbrdf_plan_workspace_bytes(self._h)

    def output_sizes(self):
        return [n * n * p * 16 for n, p in zip(self.N, self.n_dphi)]

    def solve(self, tau, omega, coef, F_r, layer_status, stream=0):
        _check(load().vbrdf_solve(self._h, _ptr(tau), _ptr(omega), _ptr(coef), _ptr(F_r), _ptr(layer_status),
                                  ctypes.c_void_p(int(stream))))

    def solve_base(self, tau, omega, coef, base, F_r, layer_status, stream=0):
        """vbrdf_solve_base: stacks and reflecting bases (base: device doubles, or None if black)."""
        _check(load().vbrdf_solve_base(self._h, _ptr(tau), _ptr(omega), _ptr(coef), _ptr(base), _ptr(F_r),
                                       _ptr(layer_status), ctypes.c_void_p(int(stream))))

    def base_bytes(self):
        return load().vbrdf_plan_base_bytes(self._h)

    def solve_ex(self, tau, omega, coef, base, F_r, F_beam, layer_status, stream=0):
        """vbrdf_solve_ex: stacks, bases and off-node beams (device pointers; None where absent)."""
        _check(load().vbrdf_solve_ex(self._h, _ptr(tau), _ptr(omega), _ptr(coef), _ptr(base), _ptr(F_r),
                                     _ptr(F_beam), _ptr(layer_status), ctypes.c_void_p(int(stream))))

    def beam_bytes(self):
        return load().vbrdf_plan_beam_bytes(self._h)

    def get_tuning(self):
        t = Tuning()
        _check(load().vbrdf_plan_get_tuning(self._h, ctypes.byref(t)))
        return {"eigen_schedule": t.eigen_schedule, "trsm_rows": t.trsm_rows}

    def set_tuning(self, eigen_schedule, trsm_rows):
        t = Tuning(int(eigen_schedule), int(trsm_rows))
        _check(load().vbrdf_plan_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, tau, omega, coef, F_r, layer_status, stream=0):
        """Time the candidate schedules and tile shapes on these inputs and keep the fastest."""
        t = Tuning()
        _check(load().vbrdf_plan_autotune(self._h, _ptr(tau), _ptr(omega), _ptr(coef), _ptr(F_r),
                                          _ptr(layer_status), ctypes.c_void_p(int(stream)), ctypes.byref(t)))
        return {"eigen_schedule": t.eigen_schedule, "trsm_rows": t.trsm_rows}

    def backward(self, tau, omega, coef, dF, dtau, domega, dcoef, stream=0):
        """Gradients of a loss with respect to tau, omega and coef given dLoss/dF_r (device
        pointers; the plan needs FLAG_SAVE_FOR_BACKWARD and a preceding solve on the same inputs)."""
        _check(load().vbrdf_backward(self._h, _ptr(tau), _ptr(omega), _ptr(coef), _ptr(dF), _ptr(dtau),
                                     _ptr(domega), _ptr(dcoef), ctypes.c_void_p(int(stream))))

    def inspect(self, layer, m, stream=0, transmission=False):
        """Host copies of R^m (4N x 4N) and the eigenvalues of FE for one (layer, order); with
        transmission=True also T^m (plan created with FLAG_EMIT_TRANSMISSION)."""
        n = 4 * self.N[layer]
        R = np.zeros((n, n))
        lr = np.zeros(n)
        li = np.zeros(n)
        T = np.zeros((n, n)) if transmission else None
        _check(load().vbrdf_plan_inspect(self._h, int(layer), int(m), _ptr(R), _ptr(lr), _ptr(li), _ptr(T),
                                         ctypes.c_void_p(int(stream))))
        if transmission:
            return R, lr + 1j * li, T
        return R, lr + 1j * li

    def stage_times(self):
        """{stage name: ms} of the last solve (plan created with FLAG_STAGE_TIMING)."""
        buf = (ctypes.c_float * 64)()
        n = load().vbrdf_plan_stage_times(self._h, buf, 64)
        if n < 0:
            _check(n)
        return {load().vbrdf_stage_name(i).decode(): float(buf[i]) for i in range(n)}

    def radiance(self, F_r, layer, q, I0, I_out, stream=0, phi0=0.0):
        i0 = (ctypes.c_double * 4)(*[float(v) for v in I0])
        _check(load().vbrdf_radiance(self._h, _ptr(F_r), int(layer), int(q), float(phi0), i0, _ptr(I_out),
                                     ctypes.c_void_p(int(stream))))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().vbrdf_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
