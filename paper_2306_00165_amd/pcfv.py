"""Thin ctypes binding of libpcfv (C ABI in include/pcfv.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libpcfv.so.  PyTorch provides device memory (the caller's fields
and the context workspace) and the HIP stream.  Fields are complex128 tensors
of shape (3, 2Kx+1, Kz+1, Ny) on the GPU (layout documented in pcfv.h).

Importing this module loads libpcfv.so and fails loudly if it is missing: there
is no fallback path.
"""

import ctypes
import os

import numpy as np
# torch must be loaded first: its HIP runtime (SONAME libamdhip64.so.7) then
# satisfies libpcfv's dependency, so both share one runtime and one device
# context.  Loading libpcfv first would pull in a second HIP runtime.
import torch  # noqa: F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "libpcfv.so")

OK, EINVAL, ENOMEM, EDEVICE, ENAN, EDIVERGED, ENOTCONV = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "PCFV_OK", -1: "PCFV_EINVAL", -2: "PCFV_ENOMEM", -3: "PCFV_EDEVICE",
                -4: "PCFV_ENAN", -5: "PCFV_EDIVERGED", -6: "PCFV_ENOTCONV"}

EXPORTS = [
    "pcfv_workspace_bytes", "pcfv_create", "pcfv_destroy", "pcfv_get_layout", "pcfv_set_stream",
    "pcfv_residual", "pcfv_cost", "pcfv_jvp", "pcfv_adjoint", "pcfv_project", "pcfv_descend",
    "pcfv_norms", "pcfv_pack_state", "pcfv_unpack_state", "pcfv_check_state",
    "pcfv_time_kernels", "pcfv_last_error", "pcfv_host_table", "pcfv_dmd_extrapolate",
    "pcfv_host_dmd", "pcfv_set_precision", "pcfv_autotune", "pcfv_get_tuning", "pcfv_set_tuning",
    "pcfv_group_create", "pcfv_group_workspace_bytes", "pcfv_group_set_stream", "pcfv_group_descend_tol",
    "pcfv_group_destroy", "pcfv_group_descend", "pcfv_group_last_error",
    "pcfv_mlp_param_count", "pcfv_mlp_workspace_bytes", "pcfv_mlp_create", "pcfv_mlp_destroy",
    "pcfv_mlp_last_error", "pcfv_mlp_set_params", "pcfv_mlp_get_params", "pcfv_mlp_forward", "pcfv_mlp_grad",
    "pcfv_mlp_adam_step", "pcfv_mlp_read", "pcfv_mlp_fit", "pcfv_pod_scratch_bytes", "pcfv_pod_build",
    "pcfv_pod_project_scratch_bytes", "pcfv_pod_project", "pcfv_pod_reconstruct", "pcfv_learned_scratch_bytes",
    "pcfv_learned_propose", "pcfv_learned_prepare", "pcfv_time_descent_kernels", "pcfv_pod_project_noalloc",
]

NOALLOC_SCRATCH_BYTES = 8 << 20

MLP_MAX_LAYERS = 8
MLP_ACT, MLP_OUT, MLP_DZ, MLP_GRAD = 0, 1, 2, 3

FP64, MIXED = 0, 1


class Config(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_double), ("Lz", ctypes.c_double), ("Re", ctypes.c_double),
                ("Nx", ctypes.c_int), ("Ny", ctypes.c_int), ("Nz", ctypes.c_int),
                ("dt_im", ctypes.c_double), ("precision", ctypes.c_int), ("batch", ctypes.c_int)]


class Layout(ctypes.Structure):
    _fields_ = [("Kx", ctypes.c_int), ("Kz", ctypes.c_int), ("Ny", ctypes.c_int),
                ("nkx", ctypes.c_int), ("nkz", ctypes.c_int), ("n_modes", ctypes.c_longlong),
                ("n_complex", ctypes.c_longlong), ("n_state", ctypes.c_longlong),
                ("batch", ctypes.c_int), ("stride_b", ctypes.c_longlong), ("stride_c", ctypes.c_longlong),
                ("stride_kx", ctypes.c_longlong), ("stride_kz", ctypes.c_longlong)]


class DescentOpts(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_longlong), ("dtau", ctypes.c_double),
                ("rel_tol", ctypes.c_double), ("check_every", ctypes.c_int),
                ("grow_tol", ctypes.c_double), ("max_halvings", ctypes.c_int),
                ("dmd_window", ctypes.c_int), ("dmd_stride", ctypes.c_int), ("dmd_gap", ctypes.c_int),
                ("dmd_start", ctypes.c_double), ("dmd_accept", ctypes.c_double),
                ("dmd_buffer", ctypes.c_void_p), ("fp64_below", ctypes.c_double),
                ("learned", ctypes.c_void_p), ("no_cost_checks", ctypes.c_int),
                ("dmd_stride_max", ctypes.c_int), ("dmd_grow_ratio", ctypes.c_double)]


class MlpConfig(ctypes.Structure):
    _fields_ = [("n_layers", ctypes.c_int), ("dims", ctypes.c_int * (MLP_MAX_LAYERS + 1)),
                ("max_batch", ctypes.c_int)]


class LearnedModel(ctypes.Structure):
    _fields_ = [("window", ctypes.c_int), ("use_base", ctypes.c_int), ("r", ctypes.c_int), ("pod_mean", ctypes.c_void_p),
                ("pod_basis", ctypes.c_void_p), ("in_mu", ctypes.c_void_p), ("in_isd", ctypes.c_void_p),
                ("out_mu", ctypes.c_void_p), ("out_isd", ctypes.c_void_p), ("mlp", ctypes.c_void_p),
                ("n_scales", ctypes.c_int), ("scales", ctypes.c_double * 8), ("scratch", ctypes.c_void_p)]


class TuneEntry(ctypes.Structure):
    _fields_ = [("xs", ctypes.c_int), ("plane_threads", ctypes.c_int), ("mode_threads", ctypes.c_int),
                ("ms_per_step", ctypes.c_double)]


class DescentReport(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_longlong), ("tau", ctypes.c_double), ("cost", ctypes.c_double),
                ("rel_res", ctypes.c_double), ("dtau_final", ctypes.c_double),
                ("n_halvings", ctypes.c_int), ("n_dmd", ctypes.c_int), ("n_dmd_accepted", ctypes.c_int),
                ("steps_fp32", ctypes.c_longlong), ("n_learned_accepted", ctypes.c_int),
                ("dmd_stride_final", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class GroupOpts(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_longlong), ("rel_tol", ctypes.c_double), ("check_every", ctypes.c_int),
                ("fp64_below", ctypes.c_double), ("dmd_window", ctypes.c_int), ("dmd_stride", ctypes.c_int),
                ("dmd_accept", ctypes.c_double), ("dmd_buffers", ctypes.POINTER(ctypes.c_void_p))]


def load_library(path=_LIB_PATH):
    if not os.path.exists(path):
        raise RuntimeError(f"libpcfv.so not built ({path}); run __graft_entry__.build()")
    lib = ctypes.CDLL(path)
    vp, dp, i, d = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_double
    cfgp = ctypes.POINTER(Config)
    lib.pcfv_workspace_bytes.restype = ctypes.c_size_t
    lib.pcfv_workspace_bytes.argtypes = [cfgp]
    lib.pcfv_create.restype = i
    lib.pcfv_create.argtypes = [cfgp, vp, vp, ctypes.POINTER(vp)]
    lib.pcfv_destroy.restype = None
    lib.pcfv_destroy.argtypes = [vp]
    lib.pcfv_get_layout.restype = i
    lib.pcfv_get_layout.argtypes = [vp, ctypes.POINTER(Layout)]
    lib.pcfv_set_stream.restype = i
    lib.pcfv_set_stream.argtypes = [vp, vp]
    lib.pcfv_set_precision.restype = i
    lib.pcfv_set_precision.argtypes = [vp, i]
    lib.pcfv_residual.restype = i
    lib.pcfv_residual.argtypes = [vp, vp, vp, dp]
    lib.pcfv_cost.restype = i
    lib.pcfv_cost.argtypes = [vp, vp, dp]
    for name in ("pcfv_jvp", "pcfv_adjoint"):
        getattr(lib, name).restype = i
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
    for name in ("pcfv_project", "pcfv_pack_state", "pcfv_unpack_state"):
        getattr(lib, name).restype = i
        getattr(lib, name).argtypes = [vp, vp, vp]
    lib.pcfv_descend.restype = i
    lib.pcfv_descend.argtypes = [vp, vp, ctypes.POINTER(DescentOpts), ctypes.POINTER(DescentReport)]
    for name in ("pcfv_norms", "pcfv_check_state"):
        getattr(lib, name).restype = i
        getattr(lib, name).argtypes = [vp, vp, dp]
    lib.pcfv_time_descent_kernels.restype = i
    lib.pcfv_time_descent_kernels.argtypes = [vp, vp, d, i, dp]
    lib.pcfv_time_kernels.restype = i
    lib.pcfv_time_kernels.argtypes = [vp, vp, i, dp, ctypes.POINTER(i)]
    lib.pcfv_last_error.restype = ctypes.c_char_p
    lib.pcfv_last_error.argtypes = [vp]
    lib.pcfv_host_table.restype = ctypes.c_size_t
    lib.pcfv_host_table.argtypes = [cfgp, i, dp, ctypes.c_size_t]
    lib.pcfv_dmd_extrapolate.restype = i
    lib.pcfv_dmd_extrapolate.argtypes = [vp, vp, i, d, vp, dp, ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.pcfv_host_dmd.restype = i
    lib.pcfv_host_dmd.argtypes = [dp, dp, i, d, dp, ctypes.POINTER(i), i]
    lib.pcfv_autotune.restype = i
    lib.pcfv_autotune.argtypes = [vp, vp, i, ctypes.POINTER(TuneEntry), i, ctypes.POINTER(i)]
    lib.pcfv_get_tuning.restype = i
    lib.pcfv_get_tuning.argtypes = [vp, ctypes.POINTER(i), ctypes.POINTER(i), ctypes.POINTER(i)]
    lib.pcfv_set_tuning.restype = i
    lib.pcfv_set_tuning.argtypes = [vp, i, i, i]
    lib.pcfv_group_workspace_bytes.restype = ctypes.c_size_t
    lib.pcfv_group_workspace_bytes.argtypes = [ctypes.POINTER(vp), i]
    lib.pcfv_group_create.restype = i
    lib.pcfv_group_create.argtypes = [ctypes.POINTER(vp), i, vp, vp, ctypes.POINTER(vp)]
    lib.pcfv_group_set_stream.restype = i
    lib.pcfv_group_set_stream.argtypes = [vp, vp]
    lib.pcfv_group_descend_tol.restype = i
    lib.pcfv_group_descend_tol.argtypes = [vp, ctypes.POINTER(vp), dp, ctypes.POINTER(GroupOpts),
                                           ctypes.POINTER(DescentReport), ctypes.POINTER(i)]
    lib.pcfv_group_destroy.restype = None
    lib.pcfv_group_destroy.argtypes = [vp]
    lib.pcfv_group_descend.restype = i
    lib.pcfv_group_descend.argtypes = [vp, ctypes.POINTER(vp), dp, ctypes.c_longlong, i]
    lib.pcfv_group_last_error.restype = ctypes.c_char_p
    lib.pcfv_group_last_error.argtypes = [vp]
    mcp = ctypes.POINTER(MlpConfig)
    fp = ctypes.POINTER(ctypes.c_float)
    lib.pcfv_mlp_param_count.restype = ctypes.c_longlong
    lib.pcfv_mlp_param_count.argtypes = [mcp]
    lib.pcfv_mlp_workspace_bytes.restype = ctypes.c_size_t
    lib.pcfv_mlp_workspace_bytes.argtypes = [mcp]
    lib.pcfv_mlp_create.restype = i
    lib.pcfv_mlp_create.argtypes = [mcp, vp, vp, ctypes.POINTER(vp)]
    lib.pcfv_mlp_destroy.restype = None
    lib.pcfv_mlp_destroy.argtypes = [vp]
    lib.pcfv_mlp_last_error.restype = ctypes.c_char_p
    lib.pcfv_mlp_last_error.argtypes = [vp]
    for name in ("pcfv_mlp_set_params", "pcfv_mlp_get_params"):
        getattr(lib, name).restype = i
        getattr(lib, name).argtypes = [vp, fp]
    lib.pcfv_mlp_forward.restype = i
    lib.pcfv_mlp_forward.argtypes = [vp, vp, vp, i]
    lib.pcfv_mlp_grad.restype = i
    lib.pcfv_mlp_grad.argtypes = [vp, vp, vp, i, fp]
    lib.pcfv_mlp_adam_step.restype = i
    lib.pcfv_mlp_adam_step.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float]
    lib.pcfv_mlp_read.restype = i
    lib.pcfv_mlp_read.argtypes = [vp, i, i, vp, ctypes.c_size_t]
    lib.pcfv_mlp_fit.restype = i
    lib.pcfv_mlp_fit.argtypes = [vp, vp, vp, i, i, i, ctypes.c_float, ctypes.c_ulonglong, vp, vp, vp, fp]
    lib.pcfv_pod_scratch_bytes.restype = ctypes.c_size_t
    lib.pcfv_pod_scratch_bytes.argtypes = [i, ctypes.c_longlong, i]
    lib.pcfv_pod_build.restype = i
    lib.pcfv_pod_build.argtypes = [vp, vp, i, ctypes.c_longlong, i, vp, vp, dp, vp]
    lib.pcfv_pod_project_scratch_bytes.restype = ctypes.c_size_t
    lib.pcfv_pod_project_scratch_bytes.argtypes = [i, ctypes.c_longlong, i]
    lib.pcfv_pod_project.restype = i
    lib.pcfv_pod_project.argtypes = [vp, vp, i, ctypes.c_longlong, i, vp, vp, vp, vp]
    lib.pcfv_pod_project_noalloc.restype = i
    lib.pcfv_pod_project_noalloc.argtypes = [vp, vp, i, ctypes.c_longlong, i, vp, vp, vp]
    lib.pcfv_pod_reconstruct.restype = i
    lib.pcfv_pod_reconstruct.argtypes = [vp, vp, i, ctypes.c_longlong, i, vp, vp, vp]
    lib.pcfv_learned_scratch_bytes.restype = ctypes.c_size_t
    lib.pcfv_learned_scratch_bytes.argtypes = [vp, i, i]
    lib.pcfv_learned_propose.restype = i
    lib.pcfv_learned_propose.argtypes = [vp, ctypes.POINTER(LearnedModel), vp, vp, vp, dp]
    lib.pcfv_learned_prepare.restype = i
    lib.pcfv_learned_prepare.argtypes = [vp, i, i, i, vp, vp, vp, i, vp, vp, vp, vp, vp, vp]
    return lib


_lib = load_library()


class PcfvError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def make_config(Nx, Ny, Nz, Lx=2 * np.pi / 1.14, Lz=2 * np.pi / 2.5, Re=400.0, dt_im=0.25,
                batch=1, precision=FP64):
    return Config(float(Lx), float(Lz), float(Re), int(Nx), int(Ny), int(Nz), float(dt_im),
                  int(precision), int(batch))


def workspace_bytes(cfg):
    return int(_lib.pcfv_workspace_bytes(ctypes.byref(cfg)))


def host_table(cfg, which):
    """Host-side copy of a setup table (no device needed), as a numpy array."""
    n = _lib.pcfv_host_table(ctypes.byref(cfg), int(which), None, 0)
    if n == 0:
        raise ValueError("invalid configuration or table index")
    out = np.empty(n, dtype=np.float64)
    _lib.pcfv_host_table(ctypes.byref(cfg), int(which),
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n)
    return out


def host_dmd(Ge_hi, dtau, Ge_lo=None):
    """Host DMD algebra (test hook): the candidates [(rank, kind, coef)] of a
    window from the Gram matrix of its snapshot differences."""
    hi = np.ascontiguousarray(Ge_hi, dtype=np.float64)
    M = hi.shape[0]
    lo = None if Ge_lo is None else np.ascontiguousarray(Ge_lo, dtype=np.float64)
    dptr = ctypes.POINTER(ctypes.c_double)
    n = _lib.pcfv_host_dmd(hi.ctypes.data_as(dptr), None if lo is None else lo.ctypes.data_as(dptr), int(M),
                           float(dtau), None, None, 0)
    if n < 0:
        raise ValueError("invalid DMD input")
    coef = np.zeros((max(n, 1), M - 1))
    labels = np.zeros(2 * max(n, 1), dtype=np.int32)
    _lib.pcfv_host_dmd(hi.ctypes.data_as(dptr), None if lo is None else lo.ctypes.data_as(dptr), int(M),
                       float(dtau), coef.ctypes.data_as(dptr), labels.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                       int(n))
    return [(int(labels[2 * i]), int(labels[2 * i + 1]), coef[i]) for i in range(n)]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One discretisation (box, Re, grid) on one GPU, holding `batch` guesses.
    Owns its workspace tensor.  Fields have shape (3, 2Kx+1, Kz+1, Ny) for
    batch = 1 and (batch, 3, 2Kx+1, Kz+1, Ny) otherwise."""

    def __init__(self, Nx, Ny, Nz, Lx=2 * np.pi / 1.14, Lz=2 * np.pi / 2.5, Re=400.0,
                 dt_im=0.25, device="cuda:0", stream=None, batch=1, precision=FP64):
        self.torch = torch
        self.device = torch.device(device)
        self.batch = int(batch)
        self.cfg = make_config(Nx, Ny, Nz, Lx, Lz, Re, dt_im, self.batch, precision)
        nbytes = workspace_bytes(self.cfg)
        if nbytes == 0:
            raise PcfvError(EINVAL, "invalid configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws_ptr = ctypes.c_void_p(self.workspace.data_ptr() + off)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        st = _lib.pcfv_create(ctypes.byref(self.cfg), ctypes.c_void_p(stream.cuda_stream),
                              self._ws_ptr, ctypes.byref(h))
        if st != OK:
            raise PcfvError(st, "pcfv_create failed: " + _lib.pcfv_last_error(None).decode())
        self._h = h
        lay = Layout()
        _lib.pcfv_get_layout(self._h, ctypes.byref(lay))
        self.layout = lay
        one = (3, lay.nkx, lay.nkz, lay.Ny)
        self.shape = one if self.batch == 1 else (self.batch,) + one
        self.n_state = lay.n_state

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pcfv_destroy(h)
            self._h = None

    # -- helpers -----------------------------------------------------------
    def _check(self, st):
        if st != OK:
            raise PcfvError(st, _lib.pcfv_last_error(self._h).decode())
        return st

    def _field(self, x):
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.asarray(x, dtype=np.complex128))
        x = x.to(self.device, t.complex128).contiguous()
        if tuple(x.shape) != self.shape:
            raise ValueError(f"field shape {tuple(x.shape)} != {self.shape}")
        return x

    def empty(self):
        return self.torch.empty(self.shape, dtype=self.torch.complex128, device=self.device)

    # -- the C ABI -----------------------------------------------------------
    def _scalars(self, n):
        return (ctypes.c_double * (n * self.batch))()

    def _unbatch(self, vals, n):
        vals = list(vals)
        rows = [tuple(vals[i * n:(i + 1) * n]) if n > 1 else vals[i] for i in range(self.batch)]
        return rows[0] if self.batch == 1 else rows

    def residual(self, u, want_cost=False):
        u = self._field(u)
        r = self.empty()
        c = self._scalars(1)
        self._check(_lib.pcfv_residual(self._h, _ptr(u), _ptr(r), c if want_cost else None))
        return (r, self._unbatch(c, 1)) if want_cost else r

    def cost(self, u):
        u = self._field(u)
        c = self._scalars(1)
        self._check(_lib.pcfv_cost(self._h, _ptr(u), c))
        return self._unbatch(c, 1)

    def jvp(self, u, v):
        u, v = self._field(u), self._field(v)
        out = self.empty()
        self._check(_lib.pcfv_jvp(self._h, _ptr(u), _ptr(v), _ptr(out)))
        return out

    def adjoint(self, u, w):
        u, w = self._field(u), self._field(w)
        out = self.empty()
        self._check(_lib.pcfv_adjoint(self._h, _ptr(u), _ptr(w), _ptr(out)))
        return out

    def project(self, g, out=None):
        g = self._field(g)
        out = self.empty() if out is None else out
        self._check(_lib.pcfv_project(self._h, _ptr(g), _ptr(out)))
        return out

    def set_precision(self, precision):
        """FP64 or MIXED (FP32 transforms and products) for later calls."""
        self._check(_lib.pcfv_set_precision(self._h, int(precision)))

    def descend(self, u, max_steps, dtau, rel_tol=0.0, check_every=None, grow_tol=0.0,
                max_halvings=0, dmd_window=0, dmd_stride=1, dmd_gap=0, dmd_start=0.0,
                dmd_accept=10.0, fp64_below=0.0, learned=None, no_cost_checks=False, dmd_stride_max=0,
                dmd_grow_ratio=0.0):
        """Advance u (a contiguous complex128 device tensor) in place; returns
        (status, report dict).  dmd_window > 0 enables DMD extrapolation (with
        dmd_stride_max > dmd_stride the stride grows fourfold after a window
        that gained less than dmd_grow_ratio); fp64_below > 0 on a MIXED
        context switches to FP64 below that relative residual."""
        if not (u.is_contiguous() and u.dtype == self.torch.complex128 and tuple(u.shape) == self.shape):
            raise ValueError("u must be a contiguous complex128 device tensor of the context shape")
        buf = None
        if dmd_window > 0:
            buf = self.torch.empty(int(dmd_window) * self.batch * self.n_state, dtype=self.torch.float64,
                                   device=self.device)
        o = DescentOpts(int(max_steps), float(dtau), float(rel_tol),
                        int(check_every or max(1, max_steps)), float(grow_tol), int(max_halvings),
                        int(dmd_window), int(dmd_stride), int(dmd_gap), float(dmd_start), float(dmd_accept),
                        ctypes.c_void_p(buf.data_ptr()) if buf is not None else None, float(fp64_below),
                        ctypes.cast(ctypes.pointer(learned.model), ctypes.c_void_p) if learned is not None else None,
                        int(bool(no_cost_checks)), int(dmd_stride_max), float(dmd_grow_ratio))
        rep = DescentReport()
        st = _lib.pcfv_descend(self._h, _ptr(u), ctypes.byref(o), ctypes.byref(rep))
        if st not in (OK, ENOTCONV, ENAN, EDIVERGED):
            self._check(st)
        return st, rep.as_dict()

    def dmd_extrapolate(self, snaps, dtau_snap, with_kind=False):
        """snaps: device float64 tensor [M][batch][n_state] (M state vectors per
        guess, oldest first).  Returns (u_s, cost(s), rank(s)) and, with
        with_kind, the candidate kind(s) as a fourth item."""
        t = self.torch
        snaps = t.as_tensor(snaps).to(self.device, t.float64).contiguous()
        M = snaps.shape[0]
        if snaps.numel() != M * self.batch * self.n_state:
            raise ValueError("snapshots have the wrong size")
        out = self.empty()
        cost = self._scalars(1)
        rank = (ctypes.c_int * self.batch)()
        kind = (ctypes.c_int * self.batch)()
        self._check(_lib.pcfv_dmd_extrapolate(self._h, _ptr(snaps), int(M), float(dtau_snap), _ptr(out),
                                              cost, rank, kind))
        res = (out, self._unbatch(cost, 1), self._unbatch(rank, 1))
        return res + (self._unbatch(kind, 1),) if with_kind else res

    def norms(self, u):
        u = self._field(u)
        out = self._scalars(3)
        self._check(_lib.pcfv_norms(self._h, _ptr(u), out))
        return self._unbatch(out, 3)

    def check_state(self, u):
        u = self._field(u)
        out = self._scalars(3)
        self._check(_lib.pcfv_check_state(self._h, _ptr(u), out))
        return self._unbatch(out, 3)

    def pack(self, u):
        u = self._field(u)
        shape = (self.n_state,) if self.batch == 1 else (self.batch, self.n_state)
        psi = self.torch.empty(shape, dtype=self.torch.float64, device=self.device)
        self._check(_lib.pcfv_pack_state(self._h, _ptr(u), _ptr(psi)))
        return psi

    def unpack(self, psi):
        t = self.torch
        psi = t.as_tensor(psi).to(self.device, t.float64).contiguous()
        if psi.numel() != self.n_state * self.batch:
            raise ValueError("psi has the wrong length")
        u = self.empty()
        self._check(_lib.pcfv_unpack_state(self._h, _ptr(psi), _ptr(u)))
        return u

    def time_kernels(self, u, nrep=20):
        u = self._field(u)
        out = (ctypes.c_double * 8)()
        n = ctypes.c_int(0)
        self._check(_lib.pcfv_time_kernels(self._h, _ptr(u), int(nrep), out, ctypes.byref(n)))
        return list(out)[:n.value]

    def time_descent_kernels(self, u, dtau, nsteps=50):
        """Advance u by nsteps descent steps, timing each kernel inside the
        steps; returns ms per launch [plane_fwd, mode_res, plane_adj, mode_grad]."""
        if not (u.is_contiguous() and u.dtype == self.torch.complex128 and tuple(u.shape) == self.shape):
            raise ValueError("u must be a contiguous complex128 device tensor of the context shape")
        out = (ctypes.c_double * 4)()
        self._check(_lib.pcfv_time_descent_kernels(self._h, _ptr(u), float(dtau), int(nsteps), out))
        return list(out)

    def synchronize(self):
        self.stream.synchronize()

    def autotune(self, u, steps=20):
        """Time every launch-shape candidate on a copy of u and keep the
        fastest; returns the list of (xs, plane_threads, mode_threads, ms_per_step)."""
        u = self._field(u)
        cap = 256
        ent = (TuneEntry * cap)()
        n = ctypes.c_int(0)
        self._check(_lib.pcfv_autotune(self._h, _ptr(u), int(steps), ent, cap, ctypes.byref(n)))
        return [(e.xs, e.plane_threads, e.mode_threads, e.ms_per_step) for e in ent[:n.value]]

    def tuning(self):
        xs, nt, mt = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_int(0)
        self._check(_lib.pcfv_get_tuning(self._h, ctypes.byref(xs), ctypes.byref(nt), ctypes.byref(mt)))
        return xs.value, nt.value, mt.value

    def set_tuning(self, xs, plane_threads, mode_threads):
        """Pin the launch shape (x-slab width, work-group sizes)."""
        self._check(_lib.pcfv_set_tuning(self._h, int(xs), int(plane_threads), int(mode_threads)))


class Group:
    """Several contexts (different grids, Re, batch; one precision) advanced
    together with one launch per stage of each descent step.  The group's
    device records live in a workspace tensor owned here, and its launches go
    to a stream created here (default priority), so that its steps can be
    captured in a HIP graph."""

    def __init__(self, contexts, stream=None):
        self.contexts = list(contexts)
        arr = (ctypes.c_void_p * len(self.contexts))(*[c._h.value for c in self.contexts])
        nbytes = _lib.pcfv_group_workspace_bytes(arr, len(self.contexts))
        if nbytes == 0:
            raise PcfvError(EINVAL, "invalid group members")
        dev = self.contexts[0].device
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        off = (-self.workspace.data_ptr()) % 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        h = ctypes.c_void_p()
        st = _lib.pcfv_group_create(arr, len(self.contexts), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.c_void_p(self.workspace.data_ptr() + off), ctypes.byref(h))
        if st != OK:
            raise PcfvError(st, "pcfv_group_create failed: " + _lib.pcfv_last_error(None).decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pcfv_group_destroy(h)
            self._h = None

    def _fields(self, fields, dtaus):
        if len(fields) != len(self.contexts) or len(dtaus) != len(self.contexts):
            raise ValueError("one field and one dtau per member")
        for c, f in zip(self.contexts, fields):
            if not (f.is_contiguous() and f.dtype == c.torch.complex128 and tuple(f.shape) == c.shape):
                raise ValueError("fields must be contiguous complex128 device tensors of the member shapes")
        ptrs = (ctypes.c_void_p * len(fields))(*[f.data_ptr() for f in fields])
        dt = (ctypes.c_double * len(fields))(*[float(x) for x in dtaus])
        return ptrs, dt

    def descend(self, fields, dtaus, steps, graph_steps=0):
        """Advance fields[k] (contiguous complex128 device tensors of member
        k's shape) in place by `steps` descent steps with dtaus[k]."""
        ptrs, dt = self._fields(fields, dtaus)
        torch.cuda.current_stream(self.contexts[0].device).synchronize()
        st = _lib.pcfv_group_descend(self._h, ptrs, dt, int(steps), int(graph_steps))
        if st != OK:
            raise PcfvError(st, _lib.pcfv_group_last_error(self._h).decode())

    def descend_tol(self, fields, dtaus, max_steps, rel_tol, check_every=100, fp64_below=0.0, dmd_window=0,
                    dmd_stride=1, dmd_accept=1.0):
        """Descend every member to rel_tol (see pcfv_group_descend_tol);
        returns (status, per-member statuses, per-member report dicts)."""
        ptrs, dt = self._fields(fields, dtaus)
        n = len(self.contexts)
        bufs = []
        if dmd_window > 0:
            bufs = [torch.empty(int(dmd_window) * c.batch * c.n_state, dtype=torch.float64, device=c.device)
                    for c in self.contexts]
        barr = (ctypes.c_void_p * max(n, 1))(*[b.data_ptr() for b in bufs]) if bufs else None
        o = GroupOpts(int(max_steps), float(rel_tol), int(check_every), float(fp64_below), int(dmd_window),
                      int(dmd_stride), float(dmd_accept),
                      ctypes.cast(barr, ctypes.POINTER(ctypes.c_void_p)) if barr is not None else None)
        reps = (DescentReport * n)()
        stats = (ctypes.c_int * n)()
        torch.cuda.current_stream(self.contexts[0].device).synchronize()
        st = _lib.pcfv_group_descend_tol(self._h, ptrs, dt, ctypes.byref(o), reps, stats)
        if st not in (OK, ENOTCONV, ENAN):
            raise PcfvError(st, _lib.pcfv_group_last_error(self._h).decode())
        return st, list(stats), [r.as_dict() for r in reps]


def _cuda_stream_ptr(torch_mod, device):
    return ctypes.c_void_p(torch_mod.cuda.current_stream(device).cuda_stream)


class MLP:
    """The extrapolator's multilayer perceptron (BF16 matrix cores, FP32
    master weights, Adam).  dims: layer widths, e.g. [2048, 512, 512, 512, 256]."""

    def __init__(self, dims, max_batch, device="cuda:0"):
        self.torch = torch
        self.device = torch.device(device)
        cfg = MlpConfig()
        cfg.n_layers = len(dims) - 1
        for k, d in enumerate(dims):
            cfg.dims[k] = int(d)
        cfg.max_batch = int(max_batch)
        self.cfg, self.dims = cfg, list(dims)
        self.n_params = _lib.pcfv_mlp_param_count(ctypes.byref(cfg))
        nbytes = _lib.pcfv_mlp_workspace_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            raise PcfvError(EINVAL, "invalid MLP configuration")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        h = ctypes.c_void_p()
        st = _lib.pcfv_mlp_create(ctypes.byref(cfg), _cuda_stream_ptr(torch, self.device),
                                  ctypes.c_void_p(self.workspace.data_ptr() + off), ctypes.byref(h))
        if st != OK:
            raise PcfvError(st, _lib.pcfv_mlp_last_error(None).decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.pcfv_mlp_destroy(h)
            self._h = None

    def _check(self, st):
        if st != OK:
            raise PcfvError(st, _lib.pcfv_mlp_last_error(self._h).decode())

    def set_params(self, params):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != self.n_params:
            raise ValueError("wrong parameter count")
        self._check(_lib.pcfv_mlp_set_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        p = np.zeros(self.n_params, dtype=np.float32)
        self._check(_lib.pcfv_mlp_get_params(self._h, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    def _rows(self, X, width):
        X = self.torch.as_tensor(X).to(self.device, self.torch.float32).contiguous()
        if X.dim() != 2 or X.shape[1] != width:
            raise ValueError("bad matrix shape")
        return X

    def forward(self, X):
        X = self._rows(X, self.dims[0])
        Y = self.torch.empty((X.shape[0], self.dims[-1]), dtype=self.torch.float32, device=self.device)
        self._check(_lib.pcfv_mlp_forward(self._h, _ptr(X), _ptr(Y), int(X.shape[0])))
        return Y

    def grad(self, X, T):
        X, T = self._rows(X, self.dims[0]), self._rows(T, self.dims[-1])
        loss = ctypes.c_float(0)
        self._check(_lib.pcfv_mlp_grad(self._h, _ptr(X), _ptr(T), int(X.shape[0]), ctypes.byref(loss)))
        return loss.value

    def adam_step(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(_lib.pcfv_mlp_adam_step(self._h, lr, beta1, beta2, eps))

    def read(self, what, layer, B):
        if what == MLP_ACT:
            out = np.zeros((B, self.dims[layer]), dtype=np.uint16)
        elif what == MLP_DZ:
            out = np.zeros((B, self.dims[layer + 1]), dtype=np.uint16)
        elif what == MLP_OUT:
            out = np.zeros((B, self.dims[-1]), dtype=np.float32)
        else:
            out = np.zeros(self.n_params, dtype=np.float32)
        self._check(_lib.pcfv_mlp_read(self._h, int(what), int(layer), out.ctypes.data_as(ctypes.c_void_p),
                                       out.nbytes))
        return out

    def fit(self, X, T, batch, epochs, lr=1e-3, seed=0):
        X, T = self._rows(X, self.dims[0]), self._rows(T, self.dims[-1])
        N = X.shape[0]
        t = self.torch
        idx = t.empty(N, dtype=t.int32, device=self.device)
        Xb = t.empty((batch, self.dims[0]), dtype=t.float32, device=self.device)
        Tb = t.empty((batch, self.dims[-1]), dtype=t.float32, device=self.device)
        hist = np.zeros(max(1, epochs), dtype=np.float32)
        self._check(_lib.pcfv_mlp_fit(self._h, _ptr(X), _ptr(T), int(N), int(batch), int(epochs), float(lr),
                                      int(seed), _ptr(idx), _ptr(Xb), _ptr(Tb),
                                      hist.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return hist[:epochs]


def pod_build(X, r):
    """POD of the rows of X (device float64 S x n): (mean, basis r x n, sigma)."""
    X = torch.as_tensor(X).to("cuda:0" if not torch.is_tensor(X) else X.device, torch.float64).contiguous()
    S, n = X.shape
    mean = torch.empty(n, dtype=torch.float64, device=X.device)
    basis = torch.empty((r, n), dtype=torch.float64, device=X.device)
    nb = _lib.pcfv_pod_scratch_bytes(int(S), int(n), int(r))
    if nb == 0:
        raise ValueError("invalid POD sizes")
    scratch = torch.empty(nb, dtype=torch.uint8, device=X.device)
    sigma = np.zeros(r)
    st = _lib.pcfv_pod_build(_cuda_stream_ptr(torch, X.device), _ptr(X), int(S), int(n), int(r), _ptr(mean),
                             _ptr(basis), sigma.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(scratch))
    if st != OK:
        raise PcfvError(st, "pcfv_pod_build failed")
    return mean, basis, sigma


def pod_project(X, mean, basis):
    X = torch.as_tensor(X).to(basis.device, torch.float64).contiguous()
    m, n = X.shape
    r = basis.shape[0]
    coef = torch.empty((m, r), dtype=torch.float64, device=basis.device)
    nb = _lib.pcfv_pod_project_scratch_bytes(int(m), int(n), int(r))
    scratch = torch.empty(max(nb, 8), dtype=torch.uint8, device=basis.device)
    st = _lib.pcfv_pod_project(_cuda_stream_ptr(torch, basis.device), _ptr(X), int(m), int(n), int(r), _ptr(mean),
                               _ptr(basis), _ptr(coef), _ptr(scratch))
    if st != OK:
        raise PcfvError(st, "pcfv_pod_project failed")
    return coef


def pod_project_noalloc(X, mean, basis, coef=None):
    """pcfv_pod_project without a workspace: the library's device-resident
    scratch holds the split-K partials.  coef (m x r, device float64) may be
    passed in so that the call itself allocates nothing."""
    m, n = X.shape
    r = basis.shape[0]
    if coef is None:
        coef = torch.empty((m, r), dtype=torch.float64, device=basis.device)
    st = _lib.pcfv_pod_project_noalloc(_cuda_stream_ptr(torch, basis.device), _ptr(X), int(m), int(n), int(r),
                                       _ptr(mean), _ptr(basis), _ptr(coef))
    if st != OK:
        raise PcfvError(st, _lib.pcfv_last_error(None).decode())
    return coef


def pod_reconstruct(coef, mean, basis):
    coef = torch.as_tensor(coef).to(basis.device, torch.float64).contiguous()
    m, r = coef.shape
    n = basis.shape[1]
    X = torch.empty((m, n), dtype=torch.float64, device=basis.device)
    st = _lib.pcfv_pod_reconstruct(_cuda_stream_ptr(torch, basis.device), _ptr(coef), int(m), int(n), int(r),
                                   _ptr(mean), _ptr(basis), _ptr(X))
    if st != OK:
        raise PcfvError(st, "pcfv_pod_reconstruct failed")
    return X


def learned_prepare(c, ct=None, stats=None, cb=None):
    """Features (and targets) of the extrapolator from POD coefficients c
    (device [W][B][r]), limit coefficients ct ([B][r]) and, for a model with a
    base candidate, the candidates' coefficients cb ([B][r]).  stats None:
    fit the normalisation and return it as (in_mu, in_isd, out_mu, out_isd)."""
    c = c.contiguous()
    W, B, r = c.shape
    dev = c.device
    F = (W + (1 if cb is not None else 0)) * r
    f32 = lambda *s: torch.empty(s, dtype=torch.float32, device=dev)
    fit = stats is None
    if fit:
        stats = (f32(F), f32(F), f32(r), f32(r))
    X = f32(B, F)
    T = f32(B, r) if ct is not None else None
    st = _lib.pcfv_learned_prepare(_cuda_stream_ptr(torch, dev), int(W), int(B), int(r), _ptr(c),
                                   _ptr(cb.contiguous()) if cb is not None else None,
                                   _ptr(ct.contiguous()) if ct is not None else None, int(fit),
                                   *[_ptr(x) for x in stats], _ptr(X), _ptr(T) if T is not None else None)
    if st != OK:
        raise PcfvError(st, "pcfv_learned_prepare failed")
    return X, T, stats


class Learned:
    """A trained extrapolator bound to one context (its batch and grid)."""

    def __init__(self, ctx, window, mean, basis, stats, mlp, use_base=False, scales=(1.0,)):
        self.ctx, self.mlp = ctx, mlp
        self.mean, self.basis, self.stats = mean.contiguous(), basis.contiguous(), stats
        r = basis.shape[0]
        nb = _lib.pcfv_learned_scratch_bytes(ctx._h, int(window), int(r))
        self.scratch = torch.empty(nb + 256, dtype=torch.uint8, device=ctx.device)
        m = LearnedModel()
        m.window, m.r, m.use_base = int(window), int(r), int(bool(use_base))
        m.pod_mean, m.pod_basis = self.mean.data_ptr(), self.basis.data_ptr()
        m.in_mu, m.in_isd, m.out_mu, m.out_isd = [x.data_ptr() for x in stats]
        m.mlp = mlp._h.value
        m.n_scales = len(scales)
        for k, a in enumerate(scales):
            m.scales[k] = float(a)
        m.scratch = self.scratch.data_ptr() + ((-self.scratch.data_ptr()) % 256)
        self.model = m

    def propose(self, snaps, base=None):
        """snaps: device float64 [W][batch][n_state]; base: [batch][n_state]
        state vectors of the base candidates (models with a base); returns
        (u, cost(s))."""
        c = self.ctx
        snaps = torch.as_tensor(snaps).to(c.device, torch.float64).contiguous()
        if base is not None:
            base = torch.as_tensor(base).to(c.device, torch.float64).contiguous()
        out = c.empty()
        cost = c._scalars(1)
        c._check(_lib.pcfv_learned_propose(c._h, ctypes.byref(self.model), _ptr(snaps),
                                           _ptr(base) if base is not None else None, _ptr(out), cost))
        return out, c._unbatch(cost, 1)
