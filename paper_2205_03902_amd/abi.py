"""ctypes binding of libimsp (include/ms.h).

Argument marshalling only: every step of the multislice path runs in the HIP
kernels behind the C ABI.  PyTorch provides device memory (the caller's
tensors and the plan workspace) and the current stream.  There is no CPU
fallback: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libimsp.so")

MS_OK, MS_ERR_INVALID_ARG, MS_ERR_UNSUPPORTED, MS_ERR_BUDGET, MS_ERR_HIP = 0, -1, -2, -3, -4
MS_ERR_NOT_FINITE = -5
MS_PATH_AUTO, MS_PATH_FUSED, MS_PATH_LINES = 0, 1, 2
MS_BANDS_NONE, MS_BANDS_ROWS, MS_BANDS_ALL = 0, 1, 2
MS_OBJECTIVE_AMPLITUDE, MS_OBJECTIVE_POISSON = 0, 1

# every entry point declared in include/ms.h
SYMBOLS = ("ms_workspace_size", "ms_plan_create", "ms_plan_destroy", "ms_plan_batch", "ms_plan_shift_classes",
           "ms_plan_checkpoint_every", "ms_plan_set_path", "ms_plan_set_bands", "ms_plan_has_bands",
           "ms_plan_set_kept_windows", "ms_plan_kept_windows", "ms_plan_set_layer_carry",
           "ms_plan_set_objective",
           "ms_make_probe", "ms_make_probe_aberrated", "ms_forward", "ms_adjoint", "ms_adjoint_scratch", "ms_layer_step", "ms_full_step", "ms_probe_step", "ms_position_grad", "ms_position_step", "ms_reconstruction_error",
           "ms_profile_begin",
           "ms_profile_end", "ms_last_error")


class MsError(RuntimeError):
    def __init__(self, status: int, what: str, message: str):
        super().__init__(f"{what} failed ({status}): {message}")
        self.status = status


class MsProblem(C.Structure):
    _fields_ = [("n", C.c_int32), ("obj_h", C.c_int32), ("obj_w", C.c_int32), ("n_slices", C.c_int32),
                ("n_pos", C.c_int64), ("positions", C.c_void_p), ("dz", C.c_void_p),
                ("pixel_size", C.c_double), ("wavelength", C.c_double),
                ("tilt_y", C.c_double), ("tilt_x", C.c_double), ("checkpoint_every", C.c_int32)]


_lib = None


def lib():
    """Loads libimsp.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2205_03902_amd.build.build() "
                               "(or __graft_entry__.build()); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.ms_workspace_size.restype = I32
        L.ms_workspace_size.argtypes = [C.POINTER(MsProblem), C.c_size_t, C.POINTER(C.c_size_t)]
        L.ms_plan_create.restype = I32
        L.ms_plan_create.argtypes = [C.POINTER(MsProblem), P, C.c_size_t, C.POINTER(P)]
        L.ms_plan_destroy.restype = None
        L.ms_plan_destroy.argtypes = [P]
        L.ms_plan_batch.restype = I64
        L.ms_plan_batch.argtypes = [P]
        L.ms_plan_shift_classes.restype = I32
        L.ms_plan_shift_classes.argtypes = [P]
        L.ms_plan_checkpoint_every.restype = I32
        L.ms_plan_checkpoint_every.argtypes = [P]
        L.ms_plan_set_path.restype = I32
        L.ms_plan_set_path.argtypes = [P, I32]
        L.ms_plan_set_bands.restype = I32
        L.ms_plan_set_bands.argtypes = [P, I32]
        L.ms_plan_has_bands.restype = I32
        L.ms_plan_has_bands.argtypes = [P]
        L.ms_plan_set_kept_windows.restype = I32
        L.ms_plan_set_kept_windows.argtypes = [P, I32]
        L.ms_plan_kept_windows.restype = I32
        L.ms_plan_kept_windows.argtypes = [P]
        L.ms_plan_set_layer_carry.restype = I32
        L.ms_plan_set_layer_carry.argtypes = [P, I32]
        L.ms_plan_set_objective.restype = I32
        L.ms_plan_set_objective.argtypes = [P, I32]
        L.ms_make_probe.restype = I32
        L.ms_make_probe.argtypes = [P, P, D, D, P]
        L.ms_make_probe_aberrated.restype = I32
        L.ms_make_probe_aberrated.argtypes = [P, P, D, P, P]
        L.ms_forward.restype = I32
        L.ms_forward.argtypes = [P, P, P, P, P, P]
        L.ms_adjoint.restype = I32
        L.ms_adjoint.argtypes = [P, P, P, P, P, P, P, P]
        L.ms_adjoint_scratch.restype = I32
        L.ms_adjoint_scratch.argtypes = [C.POINTER(MsProblem), P, P, P, P, P, P, P]
        L.ms_layer_step.restype = I32
        L.ms_layer_step.argtypes = [P, P, I32, I32, P, P, P, P, P]
        L.ms_full_step.restype = I32
        L.ms_full_step.argtypes = [P, P, I32, D, P, P, P, P, P]
        L.ms_probe_step.restype = I32
        L.ms_probe_step.argtypes = [P, P, I32, P, P, P, P, I64, P, P]
        L.ms_position_grad.restype = I32
        L.ms_position_grad.argtypes = [P, P, P, P, P, P, P, P]
        L.ms_position_step.restype = I32
        L.ms_position_step.argtypes = [P, P, D, P, P, P, P, P]
        L.ms_reconstruction_error.restype = I32
        L.ms_reconstruction_error.argtypes = [P, P, P, P, I32, I32, I32, I32, P, P, P]
        L.ms_profile_begin.restype = I32
        L.ms_profile_begin.argtypes = [P, I32]
        L.ms_profile_end.restype = I32
        L.ms_profile_end.argtypes = [P, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.ms_last_error.restype = C.c_char_p
        L.ms_last_error.argtypes = []
        _lib = L
    return _lib


def reconstruction_error(est, ref, mask=None, out=None, max_shift: int = 0, shift=None):
    """The relative reconstruction error of Sec. 5 after the model's ambiguities
    (ms_reconstruction_error): device float64 [M + 1], the slices' errors and their mean, at the
    best common translation |d| <= max_shift of the estimate (written to `shift`, a device int32 [2],
    if given).  est, ref: complex64 (M, H, W); mask: float32 (H, W) or None."""
    torch = _torch()
    M, H, W = est.shape
    if ref.shape != est.shape or est.dtype != torch.complex64 or ref.dtype != torch.complex64:
        raise ValueError("est and ref must be complex64 tensors of one shape (M, H, W)")
    if mask is not None and (tuple(mask.shape) != (H, W) or mask.dtype != torch.float32):
        raise ValueError("mask must be float32 (H, W)")
    if out is None:
        out = torch.empty(M + 1, dtype=torch.float64, device=est.device)
    side = 2 * int(max_shift) + 1
    work = torch.empty(side * side * (M + 1), dtype=torch.float64, device=est.device)
    stream = _torch().cuda.current_stream(est.device).cuda_stream
    _check(lib().ms_reconstruction_error(stream, est.data_ptr(), ref.data_ptr(), _ptr(mask), int(M), int(H), int(W),
                                         int(max_shift), work.data_ptr(), out.data_ptr(), _ptr(shift)),
           "ms_reconstruction_error")
    return out


def check_finite(values, what: str):
    """Raises MsError(MS_ERR_NOT_FINITE) if any loss value read back from the device is NaN or
    infinite (a diverged iteration: the kernels themselves never fail on such values)."""
    arr = np.asarray(values, dtype=np.float64).reshape(-1)
    bad = np.flatnonzero(~np.isfinite(arr))
    if bad.size:
        raise MsError(MS_ERR_NOT_FINITE, what, f"loss {arr[bad[0]]} at entry {int(bad[0])} of {arr.size}")


def _check(status: int, what: str):
    if status != MS_OK:
        raise MsError(status, what, lib().ms_last_error().decode())


def make_problem(n, obj_h, obj_w, n_slices, positions, dz, pixel_size, wavelength, tilt_y=0.0, tilt_x=0.0,
                 checkpoint_every=0):
    """Returns (MsProblem, keepalive) with host arrays owned by the caller's keepalive tuple.
    checkpoint_every: which incident waves the adjoint stores (1 all, k every k-th, >= M none,
    0 chosen from the workspace budget; include/ms.h)."""
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    dzs = np.ascontiguousarray(np.asarray(dz, dtype=np.float64).reshape(-1))
    if dzs.size == 0:
        dzs = np.zeros(1)
    pb = MsProblem(int(n), int(obj_h), int(obj_w), int(n_slices), pos.shape[0], pos.ctypes.data, dzs.ctypes.data,
                   float(pixel_size), float(wavelength), float(tilt_y), float(tilt_x), int(checkpoint_every))
    return pb, (pos, dzs)


def adjoint_scratch(pb: MsProblem, probe, slices, measured, want_probe: bool = True):
    """ms_adjoint_scratch: loss and gradients of problem pb without a plan or workspace (the library's
    static device array).  probe (N, N), slices (M, H, W) complex64 and measured (S, N, N) float32 on
    one CUDA device; enqueued on torch's current stream there.  Returns (loss (1,) float64,
    dL/dconj(slices), dL/dconj(probe) or None)."""
    torch = _torch()
    n, M, H, W, S = pb.n, pb.n_slices, pb.obj_h, pb.obj_w, pb.n_pos
    for t, shape, dtype, name in ((probe, (n, n), torch.complex64, "probe"), (slices, (M, H, W), torch.complex64, "slices"),
                                  (measured, (S, n, n), torch.float32, "measured")):
        if not isinstance(t, torch.Tensor) or tuple(t.shape) != shape or t.dtype != dtype or not t.is_contiguous() \
                or t.device != probe.device or t.device.type != "cuda":
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor of shape {shape} on the probe's device")
    dev = probe.device
    with torch.cuda.device(dev):
        gs = torch.empty_like(slices)
        gp = torch.empty_like(probe) if want_probe else None
        lo = torch.empty(1, dtype=torch.float64, device=dev)
        stream = torch.cuda.current_stream(dev).cuda_stream
        _check(lib().ms_adjoint_scratch(C.byref(pb), stream, _ptr(probe), _ptr(slices), _ptr(measured), _ptr(gs),
                                        _ptr(gp), _ptr(lo)), "ms_adjoint_scratch")
    return lo, gs, gp


def workspace_size(pb: MsProblem, budget_bytes: int = 0) -> int:
    out = C.c_size_t(0)
    _check(lib().ms_workspace_size(C.byref(pb), int(budget_bytes), C.byref(out)), "ms_workspace_size")
    return out.value


def _torch():
    import torch
    return torch


def _indexed(dev):
    """A CUDA device with its index made explicit ('cuda' -> 'cuda:<current>')."""
    torch = _torch()
    if dev.type == "cuda" and dev.index is None:
        return torch.device("cuda", torch.cuda.current_device())
    return dev


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Plan:
    """A multislice plan bound to one device: geometry, tables and workspace.

    Every method enqueues on torch's current stream of the plan's device and
    returns without synchronising.  Calls on one plan must not overlap.
    """

    def __init__(self, n, obj_h, obj_w, n_slices, positions, dz, pixel_size, wavelength,
                 tilt_y=0.0, tilt_x=0.0, budget_bytes: int = 0, device=None, checkpoint_every: int = 0):
        torch = _torch()
        self.device = _indexed(torch.device(device if device is not None else "cuda"))
        self.n, self.obj_h, self.obj_w, self.n_slices = int(n), int(obj_h), int(obj_w), int(n_slices)
        self.pb, self._keep = make_problem(n, obj_h, obj_w, n_slices, positions, dz, pixel_size, wavelength,
                                           tilt_y, tilt_x, checkpoint_every)
        self.n_pos = self.pb.n_pos
        ws = workspace_size(self.pb, budget_bytes)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        handle = C.c_void_p()
        _check(lib().ms_plan_create(C.byref(self.pb), self.workspace.data_ptr(), ws, C.byref(handle)),
               "ms_plan_create")
        self._h = handle
        self.batch = lib().ms_plan_batch(handle)
        self.shift_classes = lib().ms_plan_shift_classes(handle)
        self.checkpoint_every = lib().ms_plan_checkpoint_every(handle)
        self.has_bands = int(lib().ms_plan_has_bands(handle))   # bit 0 even slices, bit 1 odd slices
        self.workspace_bytes = ws
        self.budget_bytes = int(budget_bytes)
        self._path, self._objective, self._bands = MS_PATH_AUTO, MS_OBJECTIVE_AMPLITUDE, MS_BANDS_ALL
        self._kept_windows = 1

    def positions(self):
        """The scan positions (S, 2) this plan was built from (host float64 copy)."""
        return self._keep[0].copy()

    def with_positions(self, positions):
        """A plan of the same geometry, path and objective at other scan positions."""
        pb = self.pb
        plan = Plan(self.n, self.obj_h, self.obj_w, self.n_slices, positions, self._keep[1][: max(self.n_slices - 1, 0)],
                    pb.pixel_size, pb.wavelength, pb.tilt_y, pb.tilt_x, budget_bytes=self.budget_bytes,
                    device=self.device, checkpoint_every=pb.checkpoint_every)
        plan.set_path(self._path)
        plan.set_objective(self._objective)
        plan.set_bands(self._bands)
        plan.set_kept_windows(self._kept_windows)
        return plan

    @classmethod
    def from_geometry(cls, geo, positions=None, budget_bytes=0, device=None, checkpoint_every=0):
        pos = geo.positions() if positions is None else positions
        return cls(geo.n, geo.obj_h, geo.obj_w, geo.n_slices, pos, geo.gaps(), geo.pixel_size, geo.wavelength,
                   budget_bytes=budget_bytes, device=device, checkpoint_every=checkpoint_every)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.ms_plan_destroy(h)
            self._h = None

    # -- helpers -------------------------------------------------------------
    def _stream(self):
        return _torch().cuda.current_stream(self.device).cuda_stream

    def _expect(self, t, shape: Sequence[int], dtype, name: str):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, the plan on {self.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _probe(self, t, name="probe"):
        self._expect(t, (self.n, self.n), _torch().complex64, name)

    def _slices(self, t, name="slices"):
        self._expect(t, (self.n_slices, self.obj_h, self.obj_w), _torch().complex64, name)

    def _patterns(self, t, name="measured"):
        self._expect(t, (self.n_pos, self.n, self.n), _torch().float32, name)

    def set_path(self, path: int):
        """MS_PATH_AUTO, MS_PATH_FUSED or MS_PATH_LINES (see include/ms.h)."""
        _check(lib().ms_plan_set_path(self._h, int(path)), "ms_plan_set_path")
        self._path = int(path)

    def set_bands(self, mode: int):
        """MS_BANDS_ALL, MS_BANDS_ROWS or MS_BANDS_NONE (see include/ms.h)."""
        _check(lib().ms_plan_set_bands(self._h, int(mode)), "ms_plan_set_bands")
        self._bands = int(mode)

    def set_kept_windows(self, on: int):
        """1: the plain adjoint's forward chain keeps windows in place of waves where it can; 0:
        stores waves (see include/ms.h)."""
        _check(lib().ms_plan_set_kept_windows(self._h, int(on)), "ms_plan_set_kept_windows")
        self._kept_windows = int(on)

    def set_layer_carry(self, on: int):
        """1: layer steps carry the incident wave of their layer to the next step (line path, one
        batch; the caller changes the probe, slices and measured data only through layer steps
        in between); 0: every layer step runs the whole chain (see include/ms.h)."""
        _check(lib().ms_plan_set_layer_carry(self._h, int(on)), "ms_plan_set_layer_carry")

    @property
    def kept_windows(self) -> bool:
        """Whether the next adjoint keeps windows (line path, bands in both frames)."""
        return bool(lib().ms_plan_kept_windows(self._h))

    def set_objective(self, objective: int):
        """MS_OBJECTIVE_AMPLITUDE or MS_OBJECTIVE_POISSON (see include/ms.h)."""
        _check(lib().ms_plan_set_objective(self._h, int(objective)), "ms_plan_set_objective")
        self._objective = int(objective)

    # -- kernel timing ---------------------------------------------------------
    def profile_begin(self, max_launches: int):
        _check(lib().ms_profile_begin(self._h, int(max_launches)), "ms_profile_begin")

    def profile_end(self):
        """Returns (summed fused-kernel milliseconds, launches timed)."""
        ms, n = C.c_double(0.0), C.c_int64(0)
        _check(lib().ms_profile_end(self._h, C.byref(ms), C.byref(n)), "ms_profile_end")
        return ms.value, n.value

    # -- entry points --------------------------------------------------------
    def make_probe(self, alpha: float, defocus: float):
        torch = _torch()
        out = torch.empty((self.n, self.n), dtype=torch.complex64, device=self.device)
        _check(lib().ms_make_probe(self._h, self._stream(), float(alpha), float(defocus), _ptr(out)),
               "ms_make_probe")
        return out

    def make_probe_aberrated(self, alpha: float, c1: float, a1: float = 0.0, phi_a1: float = 0.0, c3: float = 0.0):
        """Probe with defocus C1, twofold astigmatism A1 at phi_A1 and spherical aberration C3 (A, rad)."""
        torch = _torch()
        out = torch.empty((self.n, self.n), dtype=torch.complex64, device=self.device)
        ab = np.array([c1, a1, phi_a1, c3], dtype=np.float64)
        _check(lib().ms_make_probe_aberrated(self._h, self._stream(), float(alpha), ab.ctypes.data, _ptr(out)),
               "ms_make_probe_aberrated")
        return out

    def forward(self, probe, slices, exit_waves: bool = False, out=None):
        torch = _torch()
        self._probe(probe)
        self._slices(slices)
        inten = out if out is not None else torch.empty((self.n_pos, self.n, self.n), dtype=torch.float32,
                                                        device=self.device)
        self._patterns(inten, "intensity_out")
        ew = torch.empty((self.n_pos, self.n, self.n), dtype=torch.complex64, device=self.device) if exit_waves \
            else None
        _check(lib().ms_forward(self._h, self._stream(), _ptr(probe), _ptr(slices), _ptr(inten), _ptr(ew)),
               "ms_forward")
        return (inten, ew) if exit_waves else inten

    def adjoint(self, probe, slices, measured, want_probe: bool = True, grad_slices=None, grad_probe=None,
                loss=None):
        """Returns (loss (1,) float64, dL/dconj(slices), dL/dconj(probe) or None)."""
        torch = _torch()
        self._probe(probe)
        self._slices(slices)
        self._patterns(measured)
        gs = grad_slices if grad_slices is not None else torch.empty_like(slices)
        self._slices(gs, "grad_slices")
        gp = None
        if want_probe:
            gp = grad_probe if grad_probe is not None else torch.empty_like(probe)
            self._probe(gp, "grad_probe")
        lo = loss if loss is not None else torch.empty(1, dtype=torch.float64, device=self.device)
        _check(lib().ms_adjoint(self._h, self._stream(), _ptr(probe), _ptr(slices), _ptr(measured), _ptr(gs),
                                _ptr(gp), _ptr(lo)), "ms_adjoint")
        return lo, gs, gp

    def layer_step(self, layer: int, k_steps: int, probe, slices, measured, loss=None, mu=None):
        """In place on slices[layer]; loss / mu: optional float64 device scalars (views)."""
        self._probe(probe)
        self._slices(slices)
        self._patterns(measured)
        _check(lib().ms_layer_step(self._h, self._stream(), int(layer), int(k_steps), _ptr(probe), _ptr(slices),
                                   _ptr(measured), _ptr(loss), _ptr(mu)), "ms_layer_step")

    def full_step(self, k_steps: int, probe, slices, measured, loss=None, mu=None, step_scale: float = 1.0):
        """In place on every slice; loss: optional float64 device scalar, mu: optional float64 device [M]."""
        self._probe(probe)
        self._slices(slices)
        self._patterns(measured)
        _check(lib().ms_full_step(self._h, self._stream(), int(k_steps), float(step_scale), _ptr(probe), _ptr(slices),
                                  _ptr(measured), _ptr(loss), _ptr(mu)), "ms_full_step")

    def probe_step(self, k_steps: int, probe, slices, measured, subset=None, loss=None, mu=None):
        """In place on probe; subset: host sequence of position indices or None for all."""
        self._probe(probe)
        self._slices(slices)
        self._patterns(measured)
        sub = None
        n_sub = 0
        if subset is not None:
            sub = np.ascontiguousarray(np.asarray(subset, dtype=np.int64).reshape(-1))
            n_sub = sub.size
        _check(lib().ms_probe_step(self._h, self._stream(), int(k_steps), _ptr(probe), _ptr(slices), _ptr(measured),
                                   None if sub is None else sub.ctypes.data, n_sub, _ptr(loss), _ptr(mu)),
               "ms_probe_step")

    def _positions(self, t, name):
        self._expect(t, (self.n_pos, 2), _torch().float64, name)

    def position_grad(self, probe, slices, measured, grad=None, curv=None, loss=None):
        """dL/dposition and the curvature bound per axis, device float64 [S, 2] each (y, x)."""
        torch = _torch()
        self._probe(probe)
        self._slices(slices)
        self._patterns(measured)
        grad = torch.empty((self.n_pos, 2), dtype=torch.float64, device=self.device) if grad is None else grad
        curv = torch.empty((self.n_pos, 2), dtype=torch.float64, device=self.device) if curv is None else curv
        self._positions(grad, "grad")
        self._positions(curv, "curv")
        _check(lib().ms_position_grad(self._h, self._stream(), _ptr(probe), _ptr(slices), _ptr(measured), _ptr(grad),
                                      _ptr(curv), _ptr(loss)), "ms_position_grad")
        return grad, curv

    def position_step(self, positions, probe, slices, measured, step_scale: float = 1.0, loss=None):
        """positions: device float64 [S, 2] holding this plan's positions; updated in place."""
        self._probe(probe)
        self._slices(slices)
        self._patterns(measured)
        self._positions(positions, "positions")
        _check(lib().ms_position_step(self._h, self._stream(), float(step_scale), _ptr(probe), _ptr(slices),
                                      _ptr(measured), _ptr(positions), _ptr(loss)), "ms_position_step")
        return positions
