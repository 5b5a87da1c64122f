"""Python binding of the ENUF HIP library (``libenuf.so``, C ABI in
``include/enuf.h``).

Argument marshalling only: every step of an evaluation runs in the library's
HIP kernels.  PyTorch provides device memory (tensors are passed by
``data_ptr()``) and the stream (``torch.cuda.current_stream()``).  There is no
CPU fallback: if the library is missing or no GPU is present, calls raise.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libenuf.so")

ENUF_OK, ENUF_EINVAL, ENUF_ENOMEM, ENUF_EDEVICE, ENUF_ENONFINITE, ENUF_ESTATE, ENUF_EUNSUPPORTED = range(7)
ENUF_FP64, ENUF_FP32 = 0, 1
(OPT_KE, OPT_TIMING, OPT_GRAPH, OPT_CHECK, OPT_FORCE_MODE, OPT_SLATER, OPT_WINDOW, OPT_OVERSAMPLING,
 OPT_SKIN, OPT_SPREAD_F16, OPT_DETERMINISTIC) = range(11)
WINDOWS = {"bspline": 0, "gaussian": 1}
FORCE_MODES = {"ik": 0, "analytic": 1}
STAGE_GRID, STAGE_SPECTRUM, STAGE_FIELDS, STAGE_SORTED, STAGE_COUNTS, STAGE_CELLS = range(6)
PHASES = ("prep", "sort", "spread", "fft_fwd", "influence_z", "fft_inv", "gather", "pair", "finalize")

# every symbol include/enuf.h declares
EXPORTS = (
    "enuf_create", "enuf_workspace_bytes", "enuf_set_workspace", "enuf_alloc_workspace", "enuf_destroy",
    "enuf_set_option", "enuf_set_stream", "enuf_energy_forces", "enuf_energy_forces_noalloc",
    "enuf_energy_grad", "enuf_eval_token", "enuf_energy_grad_dev", "enuf_get_flags", "enuf_stage_copy",
    "enuf_stage_bytes", "enuf_get_timings", "enuf_get_step_timings", "enuf_status_string", "enuf_last_error",
    "enuf_device_count", "enuf_select_params", "enuf_select_last_error", "enuf_copy_probe",
)

_lib = None


class EnufError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"ENUF error {status}: {message}")
        self.status = status


def load_library():
    """Load libenuf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"ENUF HIP library not built: {LIB_PATH} is missing "
                           "(run `python -m paper_2004_12484_amd.build`)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, d, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    lib.enuf_create.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(d), i64, d, d, ctypes.POINTER(i32), i32, i32, vp]
    lib.enuf_workspace_bytes.argtypes = [vp, ctypes.POINTER(sz)]
    lib.enuf_set_workspace.argtypes = [vp, vp, sz]
    lib.enuf_alloc_workspace.argtypes = [vp]
    lib.enuf_destroy.argtypes = [vp]
    lib.enuf_set_option.argtypes = [vp, i32, d]
    lib.enuf_set_stream.argtypes = [vp, vp]
    lib.enuf_energy_forces.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.enuf_energy_forces_noalloc.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.enuf_energy_grad.argtypes = [vp, d, vp, vp]
    lib.enuf_eval_token.argtypes = [vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.enuf_energy_grad_dev.argtypes = [vp, ctypes.c_uint64, vp, vp, vp]
    lib.enuf_get_step_timings.argtypes = [vp, ctypes.POINTER(d), i32, ctypes.POINTER(i32)]
    lib.enuf_get_flags.argtypes = [vp, ctypes.POINTER(i32)]
    lib.enuf_stage_copy.argtypes = [vp, i32, vp, sz]
    lib.enuf_stage_bytes.argtypes = [vp, i32, ctypes.POINTER(sz)]
    lib.enuf_get_timings.argtypes = [vp, ctypes.POINTER(d), i32, ctypes.POINTER(i32)]
    lib.enuf_status_string.argtypes = [i32]
    lib.enuf_status_string.restype = ctypes.c_char_p
    lib.enuf_last_error.argtypes = [vp]
    lib.enuf_last_error.restype = ctypes.c_char_p
    lib.enuf_device_count.restype = i32
    lib.enuf_select_params.argtypes = [ctypes.POINTER(d), i64, d, d, ctypes.c_char_p, ctypes.POINTER(d),
                                       ctypes.POINTER(d), ctypes.POINTER(i32), ctypes.POINTER(i32),
                                       ctypes.POINTER(i32)]
    lib.enuf_select_last_error.restype = ctypes.c_char_p
    lib.enuf_copy_probe.argtypes = [vp, vp, sz, vp]
    for name in EXPORTS:
        if name not in ("enuf_status_string", "enuf_last_error", "enuf_device_count", "enuf_select_last_error"):
            getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(status, handle=None):
    if status != ENUF_OK:
        lib = load_library()
        msg = lib.enuf_last_error(handle).decode(errors="replace")
        raise EnufError(status, msg or lib.enuf_status_string(status).decode())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class Enuf:
    """One ENUF context: fixed box, particle count, parameters and precision.

    Positions/charges/outputs are CUDA (HIP) tensors of dtype float64
    (precision "f64") or float32 ("f32"); energies are always float64.
    """

    def __init__(self, box, n, alpha, r_c, M, p, precision="f64", ke=1.0, device=None, check=False,
                 force_mode="ik", slater=None, workspace=True, window="bspline", oversampling=1.0, skin=0.0):
        """slater: decay length lambda_e of ENUF-DPD Slater-type smeared
        charges (paper Sec. 2.4); None for point charges.  workspace: give
        the context a workspace held in a torch uint8 tensor (False: none).
        window ("bspline" or "gaussian", the paper's NFFT window of cutoff
        m = p/2 - 1) and oversampling (sigma >= 1: only the modes |n_d| <
        K_d/2, K_d = 2 floor(M_d / 2 sigma), are kept).  skin > 0: persistent
        binning for MD (the sort is kept while no particle has moved more
        than skin/2)."""
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("ENUF needs a HIP GPU; torch.cuda.is_available() is False")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if dev.type != "cuda":
            raise ValueError(f"ENUF runs on a HIP device, got {dev}")
        self.device = torch.device("cuda", dev.index if dev.index is not None else torch.cuda.current_device())
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.n = int(n)
        self.box = tuple(float(b) for b in box)
        self.alpha, self.r_c, self.p = float(alpha), float(r_c), int(p)
        self.M = tuple(int(m) for m in (M if hasattr(M, "__len__") else (M, M, M)))
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream().cuda_stream
            boxa = (ctypes.c_double * 3)(*self.box)
            Ma = (ctypes.c_int32 * 3)(*self.M)
            st = lib.enuf_create(ctypes.byref(self._h), boxa, self.n, self.alpha, self.r_c, Ma, self.p,
                                 ENUF_FP64 if precision == "f64" else ENUF_FP32, ctypes.c_void_p(stream))
            if st != ENUF_OK:
                msg = lib.enuf_last_error(None).decode(errors="replace")
                raise EnufError(st, msg)
        self._ws = None
        if skin:
            self.set_option(OPT_SKIN, float(skin))
        if workspace:
            nb = ctypes.c_size_t()
            _check(lib.enuf_workspace_bytes(self._h, ctypes.byref(nb)), self._h)
            with torch.cuda.device(self.device):
                self._ws = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
                self._bind_stream()
                _check(lib.enuf_set_workspace(self._h, _ptr(self._ws), nb.value), self._h)
        self._ke = float(ke)
        if ke != 1.0:
            self.set_option(OPT_KE, ke)
        if check:
            self.set_option(OPT_CHECK, 1)
        self.force_mode = force_mode
        if force_mode != "ik":
            self.set_option(OPT_FORCE_MODE, FORCE_MODES[force_mode])
        self.slater = slater
        if slater is not None:
            self.set_option(OPT_SLATER, float(slater))
        self.window, self.oversampling = window, float(oversampling)
        if window != "bspline":
            self.set_option(OPT_WINDOW, WINDOWS[window])
        if oversampling != 1.0:
            self.set_option(OPT_OVERSAMPLING, float(oversampling))
        self._E = torch.zeros(5, dtype=torch.float64, device=self.device)

    # -- plumbing ---------------------------------------------------------
    def set_option(self, opt, value):
        _check(load_library().enuf_set_option(self._h, int(opt), float(value)), self._h)
        if opt == OPT_KE:
            self._ke = float(value)
        elif opt == OPT_SLATER:
            self.slater = float(value) if value > 0 else None
        elif opt == OPT_FORCE_MODE:
            self.force_mode = "analytic" if value == 1 else "ik"

    def options(self):
        """The options an evaluation depends on: (ke, Slater length, force mode)."""
        return (self._ke, self.slater, self.force_mode)

    def set_options(self, opts):
        ke, slater, mode = opts
        if ke != self._ke:
            self.set_option(OPT_KE, ke)
        if slater != self.slater:
            self.set_option(OPT_SLATER, 0.0 if slater is None else slater)
        if mode != self.force_mode:
            self.set_option(OPT_FORCE_MODE, FORCE_MODES[mode])

    def _bind_stream(self):
        stream = torch.cuda.current_stream(self.device).cuda_stream
        _check(load_library().enuf_set_stream(self._h, ctypes.c_void_p(stream)), self._h)

    def _in(self, t, shape):
        if not isinstance(t, torch.Tensor) or t.device != self.device or t.dtype != self.dtype:
            raise TypeError(f"expected a {self.dtype} tensor on {self.device}")
        if tuple(t.shape) != shape:
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t.contiguous()

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load_library().enuf_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- evaluation -------------------------------------------------------
    def energy_forces(self, x, q, forces=True, potential=False, out=None):
        """Returns (E, F, phi): E float64[5] = (total, real, reciprocal, self,
        background); F [N,3] or None; phi [N] (dE/dq) or None."""
        x = self._in(x, (self.n, 3))
        q = self._in(q, (self.n,))
        self._bind_stream()
        E = torch.empty(5, dtype=torch.float64, device=self.device) if out is None else out
        F = torch.empty((self.n, 3), dtype=self.dtype, device=self.device) if forces else None
        phi = torch.empty(self.n, dtype=self.dtype, device=self.device) if potential else None
        _check(load_library().enuf_energy_forces(self._h, _ptr(x), _ptr(q), _ptr(E), _ptr(F), _ptr(phi)),
               self._h)
        self._keep = (x, q)
        return E, F, phi

    def energy_forces_noalloc(self, x, q, E, F=None, phi=None):
        """enuf_energy_forces_noalloc: one evaluation in the library's static
        device scratch (no device allocation by the library; the outputs E,
        F, phi are the caller's preallocated tensors).  The engine's adjoint
        state is not changed."""
        x = self._in(x, (self.n, 3))
        q = self._in(q, (self.n,))
        self._bind_stream()
        _check(load_library().enuf_energy_forces_noalloc(self._h, _ptr(x), _ptr(q), _ptr(E), _ptr(F), _ptr(phi)),
               self._h)
        return E, F, phi

    def token(self):
        """Identifier of the last evaluation on this context."""
        t = ctypes.c_uint64()
        _check(load_library().enuf_eval_token(self._h, ctypes.byref(t)), self._h)
        return int(t.value)

    def energy_grad(self, grad_E=1.0, dx=True, dq=True):
        """Exact gradient of the last evaluated energy, scaled by grad_E."""
        self._bind_stream()
        gx = torch.empty((self.n, 3), dtype=self.dtype, device=self.device) if dx else None
        gq = torch.empty(self.n, dtype=self.dtype, device=self.device) if dq else None
        _check(load_library().enuf_energy_grad(self._h, float(grad_E), _ptr(gx), _ptr(gq)), self._h)
        return gx, gq

    def energy_grad_dev(self, token, grad_E, dx=True, dq=True):
        """Exact gradient of the evaluation `token`, scaled by the device
        float64 scalar grad_E (no host synchronisation).  Raises EnufError
        with status ENUF_ESTATE if the context has evaluated since."""
        self._bind_stream()
        g = grad_E.detach().to(device=self.device, dtype=torch.float64).reshape(1).contiguous()
        gx = torch.empty((self.n, 3), dtype=self.dtype, device=self.device) if dx else None
        gq = torch.empty(self.n, dtype=self.dtype, device=self.device) if dq else None
        _check(load_library().enuf_energy_grad_dev(self._h, ctypes.c_uint64(token), _ptr(g), _ptr(gx), _ptr(gq)),
               self._h)
        self._keep_grad = g
        return gx, gq

    def flags(self):
        f = ctypes.c_int32()
        _check(load_library().enuf_get_flags(self._h, ctypes.byref(f)), self._h)
        return int(f.value)

    def stage(self, which):
        """Copy of an internal buffer of the last evaluation (see enuf_stage)."""
        lib = load_library()
        nb = ctypes.c_size_t()
        _check(lib.enuf_stage_bytes(self._h, int(which), ctypes.byref(nb)), self._h)
        buf = torch.empty(nb.value, dtype=torch.uint8, device=self.device)
        _check(lib.enuf_stage_copy(self._h, int(which), _ptr(buf), nb.value), self._h)
        G = self.M[0] * self.M[1] * self.M[2]
        Mx, My, Mz = self.M
        if which == STAGE_GRID:
            return buf.view(self.dtype).view(Mz, My, Mx)
        if which == STAGE_SPECTRUM:
            return buf.view(self.dtype).view(Mz, My, Mx // 2, 2)
        if which == STAGE_FIELDS:
            if nb.value == G * buf.view(self.dtype).element_size():
                return buf.view(self.dtype).view(Mz, My, Mx)  # analytic mode: psi alone
            return buf.view(self.dtype).view(Mz, My, Mx, 4)
        return buf.view(torch.int32)

    def timings(self):
        lib = load_library()
        arr = (ctypes.c_double * len(PHASES))()
        cnt = ctypes.c_int32()
        _check(lib.enuf_get_timings(self._h, arr, len(PHASES), ctypes.byref(cnt)), self._h)
        return dict(zip(PHASES, list(arr)[: cnt.value]))

    def step_timings(self, cap=4096):
        """Per-evaluation phase times in ms, shape [evaluations, phases]."""
        import numpy as np

        lib = load_library()
        arr = (ctypes.c_double * (cap * len(PHASES)))()
        cnt = ctypes.c_int32()
        _check(lib.enuf_get_step_timings(self._h, arr, cap, ctypes.byref(cnt)), self._h)
        return np.array(arr[: cnt.value * len(PHASES)], dtype=np.float64).reshape(cnt.value, len(PHASES))


class EnufEnergy(torch.autograd.Function):
    """E = ENUF energy of (x, q); backward gives the exact dE/dx and dE/dq of
    the computed energy through the library's adjoint kernels.

    The adjoint reads what the engine kept from its last evaluation.  Each
    graph node records the evaluation token and the options of its own
    forward; if the engine has evaluated since (several energies on one
    engine before one backward), the node evaluates its saved (x, q) again
    with its own options before the adjoint, so every node gets the gradient
    of its own configuration.  The upstream gradient stays on the device."""

    @staticmethod
    def forward(ctx, x, q, engine):
        E, _, _ = engine.energy_forces(x.detach(), q.detach(), forces=False, potential=True)
        ctx.engine = engine
        ctx.token = engine.token()
        ctx.opts = engine.options()
        ctx.save_for_backward(x, q)
        return E[0].clone()

    @staticmethod
    def backward(ctx, gE):
        eng = ctx.engine
        x, q = ctx.saved_tensors
        token = ctx.token
        if eng.token() != token:
            current = eng.options()
            eng.set_options(ctx.opts)
            try:
                eng.energy_forces(x.detach(), q.detach(), forces=False, potential=True)
                token = eng.token()
            finally:
                eng.set_options(current)
        dx, dq = eng.energy_grad_dev(token, gE, dx=ctx.needs_input_grad[0], dq=ctx.needs_input_grad[1])
        return dx, dq, None


def enuf_energy(x, q, engine):
    return EnufEnergy.apply(x, q, engine)


def device_count() -> int:
    return int(load_library().enuf_device_count())


def copy_probe(src, dst, stream=None):
    """Copy device tensor src into dst (same byte size, a multiple of 16)
    with the library's plain copy kernel on `stream` (default: torch's
    current stream): the achievable-bandwidth probe."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst differ in size")
    if stream is None:
        stream = torch.cuda.current_stream(src.device).cuda_stream
    _check(load_library().enuf_copy_probe(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                          nbytes, ctypes.c_void_p(stream)))
