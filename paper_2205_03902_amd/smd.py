"""ctypes binding of the sparse matrix decomposition (include/smd.h, Algorithm 2).

Argument marshalling only: every step runs in the HIP kernels behind the C ABI; torch
provides device memory and the stream.  N^2 x N^2 matrices are column-major on the
boundary: the row-major tensor a call returns is the matrix transposed.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import abi

SYMBOLS = ("smd_workspace_size", "smd_plan_create", "smd_plan_destroy", "smd_set_probe", "smd_compose",
           "smd_estimate", "smd_decompose", "smd_result", "smd_last_error")


class SmdProblem(C.Structure):
    _fields_ = [("n", C.c_int32), ("n_slices", C.c_int32), ("n_pos", C.c_int64), ("positions", C.c_void_p),
                ("dz", C.c_void_p), ("pixel_size", C.c_double), ("wavelength", C.c_double)]


_bound = False


def lib():
    global _bound
    L = abi.lib()
    if not _bound:
        P, I32 = C.c_void_p, C.c_int32
        L.smd_workspace_size.restype = I32
        L.smd_workspace_size.argtypes = [C.POINTER(SmdProblem), C.POINTER(C.c_size_t)]
        L.smd_plan_create.restype = I32
        L.smd_plan_create.argtypes = [C.POINTER(SmdProblem), P, C.c_size_t, C.POINTER(P)]
        L.smd_plan_destroy.restype = None
        L.smd_plan_destroy.argtypes = [P]
        L.smd_set_probe.restype = I32
        L.smd_set_probe.argtypes = [P, P, P]
        L.smd_compose.restype = I32
        L.smd_compose.argtypes = [P, P, P, P, P]
        L.smd_estimate.restype = I32
        L.smd_estimate.argtypes = [P, P, P, P, I32, P]
        L.smd_decompose.restype = I32
        L.smd_decompose.argtypes = [P, P, P, P, P, P]
        L.smd_result.restype = I32
        L.smd_result.argtypes = [P, P, P, P, P]
        L.smd_last_error.restype = C.c_char_p
        L.smd_last_error.argtypes = []
        _bound = True
    return L


def _check(status: int, what: str):
    if status != abi.MS_OK:
        raise abi.MsError(status, what, lib().smd_last_error().decode())


def make_problem(n, n_slices, positions, dz, pixel_size, wavelength):
    """Returns (SmdProblem, keepalive); positions (S, 2) integer (y, x) shifts."""
    pos = np.ascontiguousarray(np.asarray(positions, dtype=np.float64).reshape(-1, 2))
    dzs = np.ascontiguousarray(np.asarray(dz, dtype=np.float64).reshape(-1))
    if dzs.size == 0:
        dzs = np.zeros(1)
    pb = SmdProblem(int(n), int(n_slices), pos.shape[0], pos.ctypes.data, dzs.ctypes.data, float(pixel_size),
                    float(wavelength))
    return pb, (pos, dzs)


def workspace_size(pb: SmdProblem) -> int:
    out = C.c_size_t(0)
    _check(lib().smd_workspace_size(C.byref(pb), C.byref(out)), "smd_workspace_size")
    return out.value


class SmdPlan:
    """Algorithm 2 on one device (full-field model, N = 16, 32, 64).  Methods enqueue on torch's
    current stream; set_probe and decompose synchronise it."""

    def __init__(self, n, n_slices, positions, dz, pixel_size, wavelength, device=None):
        torch = abi._torch()
        self.device = abi._indexed(torch.device(device if device is not None else "cuda"))
        self.n, self.n_slices = int(n), int(n_slices)
        self.pb, self._keep = make_problem(n, n_slices, positions, dz, pixel_size, wavelength)
        self.n_pos = self.pb.n_pos
        ws = workspace_size(self.pb)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
            handle = C.c_void_p()
            _check(lib().smd_plan_create(C.byref(self.pb), self.workspace.data_ptr(), ws, C.byref(handle)),
                   "smd_plan_create")
        self._h = handle

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and abi._lib is not None:
            abi._lib.smd_plan_destroy(h)
            self._h = None

    def _stream(self):
        return abi._torch().cuda.current_stream(self.device).cuda_stream

    def _expect(self, t, shape, dtype, name):
        torch = abi._torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device != self.device or t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)} on {self.device}, "
                             f"got {t.dtype} {tuple(t.shape)} on {t.device}")

    def _matrix(self, t, name):
        n2 = self.n * self.n
        self._expect(t, (n2, n2), abi._torch().complex64, name)

    def _slices(self, t, name="slices"):
        self._expect(t, (self.n_slices, self.n, self.n), abi._torch().complex64, name)

    def empty_matrix(self):
        n2 = self.n * self.n
        return abi._torch().empty((n2, n2), dtype=abi._torch().complex64, device=self.device)

    def set_probe(self, probe):
        self._expect(probe, (self.n, self.n), abi._torch().complex64, "probe")
        _check(lib().smd_set_probe(self._h, self._stream(), probe.data_ptr()), "smd_set_probe")

    def compose(self, slices, lam=1.0 + 0j, out=None):
        self._slices(slices)
        out = self.empty_matrix() if out is None else out
        self._matrix(out, "a_out")
        lv = (C.c_double * 2)(complex(lam).real, complex(lam).imag)
        _check(lib().smd_compose(self._h, self._stream(), slices.data_ptr(), lv, out.data_ptr()), "smd_compose")
        return out

    def estimate(self, measured, a, steps: int, loss_first=None):
        self._expect(measured, (self.n_pos, self.n, self.n), abi._torch().float32, "measured")
        self._matrix(a, "a")
        if loss_first is not None:
            self._expect(loss_first, (1,), abi._torch().float64, "loss_first")
        _check(lib().smd_estimate(self._h, self._stream(), measured.data_ptr(), a.data_ptr(), int(steps),
                                  abi._ptr(loss_first)), "smd_estimate")
        return a

    def decompose(self, a_hat, slices, lam: complex, a_tilde=None) -> complex:
        """One decomposition pass in place on `slices`; returns the new lambda."""
        self._matrix(a_hat, "a_hat")
        self._slices(slices)
        if a_tilde is not None:
            self._matrix(a_tilde, "a_tilde")
        lv = (C.c_double * 2)(complex(lam).real, complex(lam).imag)
        _check(lib().smd_decompose(self._h, self._stream(), a_hat.data_ptr(), slices.data_ptr(), lv,
                                   abi._ptr(a_tilde)), "smd_decompose")
        return complex(lv[0], lv[1])

    def result(self, slices, lam: complex, out=None):
        self._slices(slices)
        out = abi._torch().empty_like(slices) if out is None else out
        self._slices(out, "out")
        lv = (C.c_double * 2)(complex(lam).real, complex(lam).imag)
        _check(lib().smd_result(self._h, self._stream(), slices.data_ptr(), lv, out.data_ptr()), "smd_result")
        return out

    def iterate(self, measured, slices, lam: complex, iterations: int, a_steps: int, losses=None):
        """`iterations` rounds of Algorithm 2 from `slices` (in place) and lambda, after
        set_probe; losses (device float64 [iterations] or None) receives the matrix loss
        before each round.  Returns the final lambda."""
        a = self.compose(slices, lam)
        for it in range(int(iterations)):
            self.estimate(measured, a, a_steps, None if losses is None else losses[it:it + 1])
            lam = self.decompose(a, slices, lam)
            self.compose(slices, lam, out=a)
        return lam

    def algorithm2(self, probe, measured, slices0, iterations: int, a_steps: int):
        """Algorithm 2: returns (lambda^(1/M) O_m, lambda, matrix loss before each iteration)."""
        torch = abi._torch()
        self.set_probe(probe)
        slices = slices0.clone()
        losses = torch.zeros(max(int(iterations), 1), dtype=torch.float64, device=self.device)
        lam = self.iterate(measured, slices, 1.0 + 0j, iterations, a_steps, losses)
        return self.result(slices, lam), lam, losses[:int(iterations)]
